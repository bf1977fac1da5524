"""The no-allocation solve (mesh_sdd_solve_interfaces_noalloc) through the
C-ABI against the allocating solve (mesh_sdd_solve_interfaces) of the same
instance and step: the same kernels and chunk plan, so the results must be
identical bit for bit.  Two calls in a row, the second with a smaller input
(the array keeps the first call's contents), an FP64 call, and the refusals
(host pointers, a solve larger than the scratch)."""
import numpy as np
import pytest

from paper_1504_00084_amd import workloads as W
from gpu_helpers import say

pytestmark = pytest.mark.gpu

FIELDS = ("mean_x", "mean_y", "se_x", "se_y", "exit_frac")


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_00084_amd import mesh_sdd
    mesh_sdd.load()
    return mesh_sdd


def device_inputs(inst):
    import torch
    d = torch.device("cuda:0")
    return [torch.from_numpy(np.ascontiguousarray(a)).to(d) for a in (inst.x, inst.y, inst.bnd_t0, inst.bnd_t1)]


def both(M, ctx, inst, precision, n_paths):
    """(allocating, no-allocation) results of one instance, device in / out."""
    import torch
    h = M.mesh_sdd_create(ctx, M.desc_for(inst, precision))
    try:
        M.mesh_sdd_set_monitor(h, inst.rho)
        m = M.mesh_sdd_num_interface_nodes(h)
        x, y, b0, b1 = device_inputs(inst)
        st = M.make_step(x, y, b0, b1, paths_per_node=n_paths, mesh_step=inst.mesh_step)
        out = []
        for fn in (M.mesh_sdd_solve_interfaces, M.mesh_sdd_solve_interfaces_noalloc):
            arrs = [torch.full((max(m, 1),), float("nan"), dtype=torch.float64, device="cuda:0") for _ in FIELDS]
            res = M.make_result(*arrs)
            fn(h, st, res)
            torch.cuda.synchronize()
            d = {k: a[:m].cpu().numpy() for k, a in zip(FIELDS, arrs)}
            d["executed_path_steps"] = int(res.executed_path_steps)
            out.append(d)
        return out
    finally:
        M.mesh_sdd_destroy(h)


def same_bits(a, b, label):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k], equal_nan=True), (label, k)
    assert a["executed_path_steps"] == b["executed_path_steps"], label
    say("%s: no-allocation == allocating (bitwise), %d nodes, %.3e path-steps"
        % (label, len(a["mean_x"]), a["executed_path_steps"]))


def test_noalloc_equals_allocating_twice_then_smaller(M):
    ctx = M.mesh_sdd_ctx_create(0)
    try:
        big = W.config2(n_paths=8192)          # 129^2, 4x4: the LDS-table kernel
        a, b = both(M, ctx, big, M.FP32, big.n_paths)
        same_bits(a, b, "rotbump129 N=8192")
        mid = W.config3(n_paths=1024)          # 257^2 periodic front: the windowed kernel
        a, b = both(M, ctx, mid, M.FP32, mid.n_paths)
        same_bits(a, b, "front257 N=1024")
        small = W.config1(n_paths=1000)        # 33^2, 31 nodes: smaller than the calls before
        a, b = both(M, ctx, small, M.FP32, small.n_paths)
        same_bits(a, b, "bump33 N=1000")
        a, b = both(M, ctx, small, M.FP64, 512)
        same_bits(a, b, "bump33 fp64 N=512")
    finally:
        M.mesh_sdd_ctx_destroy(ctx)


def test_noalloc_refusals(M):
    import torch
    ctx = M.mesh_sdd_ctx_create(0)
    inst = W.config2(n_paths=1000)
    h = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
    try:
        M.mesh_sdd_set_monitor(h, inst.rho)
        m = M.mesh_sdd_num_interface_nodes(h)
        arrs = [torch.empty(m, dtype=torch.float64, device="cuda:0") for _ in FIELDS]
        res = M.make_result(*arrs)
        host = M.make_step(inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, paths_per_node=1000)
        with pytest.raises(M.MeshSddError) as e:
            M.mesh_sdd_solve_interfaces_noalloc(h, host, res)
        assert e.value.code == M.E_INVAL
        x, y, b0, b1 = device_inputs(inst)
        huge = M.make_step(x, y, b0, b1, paths_per_node=400_000)   # partials alone: 753 x 3125 x 48 B > 64 MiB
        with pytest.raises(M.MeshSddError) as e:
            M.mesh_sdd_solve_interfaces_noalloc(h, huge, res)
        assert e.value.code == M.E_INVAL and "scratch" in str(e.value)
        strided = M.make_step(x, y, b0, b1, paths_per_node=1000, interface_stride=4)
        with pytest.raises(M.MeshSddError) as e:
            M.mesh_sdd_solve_interfaces_noalloc(h, strided, res)
        assert e.value.code == M.E_STATE
        # after an allocating solve with that stride the lists exist, and the
        # no-allocation solve gives its bits
        harrs, hres = M.host_result(m)
        hstep = M.make_step(inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, paths_per_node=1000, interface_stride=4)
        M.mesh_sdd_solve_interfaces(h, hstep, hres)
        M.mesh_sdd_solve_interfaces_noalloc(h, strided, res)
        torch.cuda.synchronize()
        for k, a, ha in zip(FIELDS, arrs, harrs):
            assert np.array_equal(a.cpu().numpy(), ha[:m], equal_nan=True), k
        say("stride 4: no-allocation == allocating (bitwise)")
    finally:
        M.mesh_sdd_destroy(h)
        M.mesh_sdd_ctx_destroy(ctx)
