"""End states of the FP32 kernels: a lane whose path ends stores the path's
end state and the value is evaluated when the work item drains; a path
whose winding numbers do not fit the stored fields has its value evaluated
at once instead.  Both must give the values the per-path debug entry point
computes for the same paths."""
import numpy as np
import pytest

from paper_1504_00084_amd import workloads as W
from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_00084_amd import mesh_sdd
    mesh_sdd.load()
    return mesh_sdd


@pytest.fixture(scope="module")
def ctx(M):
    c = M.mesh_sdd_ctx_create(0)
    yield c
    M.mesh_sdd_ctx_destroy(c)


@pytest.mark.parametrize("tau,monitor_table", [(1e8, 0), (1e8, 1), (0.02, 0)],
                         ids=["wide_winding_lds", "wide_winding_l2", "small_winding_lds"])
def test_solve_means_equal_debug_path_values(M, ctx, tau, monitor_table):
    """Doubly periodic 17x17, 2x2 subdomains, constant monitor (pure
    diffusion), K = 200, 256 paths per node.  With tau = 1e8 each substep
    moves a path by ~1000 periods, so the windings pass 8192 and every
    value is evaluated by its own lane at once; with tau = 0.02 the end
    states are stored and evaluated at the drain.  Per node, the mean of the
    debug values (v - v_ref rounded to FP32, as the kernels do) equals the
    solve's mean."""
    n, K, N = 17, 200, 256
    x, y = W.uniform_mesh(n, n)
    rho = np.ones_like(x)
    b = W.boundary_from_mesh(x, y)
    inst = W.Instance("wind17", n, n, 2, 2, 1, 1, 1.0, 1.0, tau, K, N, rho, x, y, b, b.copy(), seed=77,
                      instance_id=5)
    if monitor_table:
        M.mesh_sdd_set_launch(ctx, M.make_launch(monitor_table=1))
    try:
        h = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
        try:
            M.mesh_sdd_set_monitor(h, rho)
            m = M.mesh_sdd_num_interface_nodes(h)
            arrs, res = M.host_result(m)
            st = M.make_step(x, y, b, b, paths_per_node=N)
            M.mesh_sdd_solve_interfaces(h, st, res)
            got = {k: np.array(v) for k, v in M.result_dict(arrs, res, m).items() if k in ("mean_x", "mean_y")}
            level = M.mesh_sdd_get_launch(h).table_level
            ni, nj = M.mesh_sdd_interface_nodes(h)
            worst, wmax = 0.0, 0.0
            for r in (0, 7, m - 1):
                d = M.mesh_sdd_debug_paths(h, st, r, 0, N, K)
                i, j = int(ni[r]), int(nj[r])
                for comp, ref in (("x", x[j, i]), ("y", y[j, i])):
                    v = d["v" + comp]
                    dv = (v - ref).astype(np.float32).astype(np.float64)
                    want = ref + dv.sum() / N
                    worst = max(worst, abs(want - got["mean_" + comp][r]) / max(1.0, abs(want)))
                    wmax = max(wmax, float(np.max(np.abs(v - ref))))
        finally:
            M.mesh_sdd_destroy(h)
    finally:
        if monitor_table:
            M.mesh_sdd_set_launch(ctx, None)
    say("tau %g, LDS table level %d: max |v - v_ref| %.3g, max rel |debug mean - solve mean| %.2e"
        % (tau, level, wmax, worst))
    assert level == (0 if monitor_table else 2)
    assert (wmax > 8192.0) == (tau > 1.0)
    assert worst <= 1e-12


def test_debug_paths_address_ranks_on_a_blocked_grid(M, ctx):
    """161 x 161, 4 x 4 subdomains: the node lists are stored block by
    block, so positions differ from ranks; the debug entry point takes a
    rank, and the mean of its per-path values must equal the solve's mean
    at that rank."""
    n, K, N = 161, 40, 256
    x, y = W.uniform_mesh(n, n)
    rho = 1.0 + 2.0 * np.exp(-((x - 0.3) ** 2 + (y - 0.7) ** 2) / 0.02)
    b = W.boundary_from_mesh(x, y)
    inst = W.Instance("blocked161", n, n, 4, 4, 0, 0, 1.0, 1.0, 0.01, K, N, rho, x, y, b, b.copy(), seed=5,
                      instance_id=9)
    h = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
    try:
        M.mesh_sdd_set_monitor(h, rho)
        m = M.mesh_sdd_num_interface_nodes(h)
        ranks, blocks = M.mesh_sdd_desc_work_order(M.desc_for(inst, M.FP32))
        assert len(blocks) > 1 and not np.array_equal(ranks, np.arange(m))
        arrs, res = M.host_result(m)
        st = M.make_step(x, y, b, b, paths_per_node=N)
        M.mesh_sdd_solve_interfaces(h, st, res)
        got = M.result_dict(arrs, res, m)
        ni, nj = M.mesh_sdd_interface_nodes(h)
        worst = 0.0
        for r in (0, int(ranks[len(ranks) // 2]), m - 1):
            d = M.mesh_sdd_debug_paths(h, st, r, 0, N, K)
            i, j = int(ni[r]), int(nj[r])
            for comp, ref in (("x", x[j, i]), ("y", y[j, i])):
                dv = (d["v" + comp] - ref).astype(np.float32).astype(np.float64)
                worst = max(worst, abs(ref + dv.sum() / N - got["mean_" + comp][r]))
    finally:
        M.mesh_sdd_destroy(h)
    say("161x161 blocked lists: max |debug mean - solve mean| %.2e" % worst)
    assert worst <= 1e-12
