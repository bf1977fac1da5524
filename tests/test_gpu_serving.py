"""Batching and serving through the C-ABI: one persistent launch over many
instances, submit/poll with continuous batching and HBM admission, error
paths, device pointers.  A request's result is a pure function of its
inputs and RNG identity, so alone, batched and served results must agree
exactly (same chunk plan, fixed-order FP64 sums)."""
import ctypes
import time

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


def mix(count=8, n_paths=3000, seed=3):
    insts = W.config4(count=count, seed=seed, n_paths=n_paths, sizes=(33, 65, 129))
    for q, it in enumerate(insts):
        it.K = 100 + 7 * q          # uneven K too (some not multiples of 4)
        it.instance_id = 100 + q
    return insts


class Handles:
    def __init__(self, M, ctx, insts, precision):
        self.M, self.h, self.m = M, [], []
        for it in insts:
            h = M.mesh_sdd_create(ctx, M.desc_for(it, precision))
            M.mesh_sdd_set_monitor(h, it.rho)
            self.h.append(h)
            self.m.append(M.mesh_sdd_num_interface_nodes(h))

    def close(self):
        for h in self.h:
            self.M.mesh_sdd_destroy(h)


def steps_for(M, insts):
    return [M.make_step(it.x, it.y, it.bnd_t0, it.bnd_t1, paths_per_node=it.n_paths, mesh_step=it.mesh_step)
            for it in insts]


def solve_alone(M, H, insts):
    out = []
    for h, m, st in zip(H.h, H.m, steps_for(M, insts)):
        arrs, res = M.host_result(m)
        M.mesh_sdd_solve_interfaces(h, st, res)
        out.append(M.result_dict(arrs, res, m))
    return out


def same(a, b):
    for k in ("mean_x", "mean_y", "se_x", "se_y", "exit_frac"):
        if not np.array_equal(a[k], b[k], equal_nan=True):
            return False
    return a["executed_path_steps"] == b["executed_path_steps"]


def test_batch_equals_alone(M, ctx):
    insts = mix()
    H = Handles(M, ctx, insts, M.FP32)
    try:
        alone = solve_alone(M, H, insts)
        pairs = [M.host_result(m) for m in H.m]
        status = M.mesh_sdd_solve_batch(H.h, steps_for(M, insts), [p[1] for p in pairs])
        assert status == [0] * len(insts)
        for q, (arrs, res) in enumerate(pairs):
            b = M.result_dict(arrs, res, H.m[q])
            assert same(alone[q], b), q
        say("batch of %d instances == alone (bitwise)" % len(insts))
    finally:
        H.close()


def test_serving_equals_alone_and_pending(M, ctx):
    insts = mix(count=10, seed=4)
    H = Handles(M, ctx, insts, M.FP32)
    try:
        alone = solve_alone(M, H, insts)
        st = steps_for(M, insts)
        tickets = [M.mesh_sdd_submit(h, s) for h, s in zip(H.h, st)]
        pend = [M.mesh_sdd_poll(ctx, tickets[-1], None)]    # most likely still pending
        outs = []
        for q, t in enumerate(tickets):
            arrs, res = M.host_result(H.m[q])
            assert M.mesh_sdd_wait(ctx, t, res, 120_000)
            outs.append(M.result_dict(arrs, res, H.m[q]))
        for q in range(len(insts)):
            assert same(alone[q], outs[q]), q
        s = M.mesh_sdd_ctx_stats(ctx)
        say("served %d, ticks %d, p50 %.1f ms, p99 %.1f ms, first poll pending=%s"
            % (s.completed, s.ticks, s.p50_ms, s.p99_ms, not pend[0]))
        assert s.completed >= len(insts) and s.failed == 0
        with pytest.raises(M.MeshSddError):      # tickets are released once done
            M.mesh_sdd_poll(ctx, tickets[0], None)
    finally:
        H.close()


def test_admission_with_small_budget(M):
    insts = W.config4(count=6, seed=5, n_paths=3000, sizes=(33, 65))
    for q, it in enumerate(insts):
        it.K = 120
        it.instance_id = 200 + q
    # about two small requests fit next to the resident tables at a time
    c = M.mesh_sdd_ctx_create(0, 3 << 20)
    try:
        H = Handles(M, c, insts, M.FP32)
        try:
            alone = solve_alone(M, H, insts)
            st = steps_for(M, insts)
            tickets = [M.mesh_sdd_submit(h, s) for h, s in zip(H.h, st)]
            seen_queue = M.mesh_sdd_ctx_stats(c).queued
            for q, t in enumerate(tickets):
                arrs, res = M.host_result(H.m[q])
                assert M.mesh_sdd_wait(c, t, res, 120_000)
                assert same(alone[q], M.result_dict(arrs, res, H.m[q])), q
            s = M.mesh_sdd_ctx_stats(c)
            say("small budget: queued right after submit %d, in use %d of %d B, ticks %d"
                % (seen_queue, s.hbm_in_use, s.hbm_budget, s.ticks))
            assert s.hbm_in_use <= s.hbm_budget and s.completed == len(insts)
        finally:
            H.close()
        # a request larger than the whole budget is refused at submit
        big = W.config2(n_paths=1_000_000)
        h = M.mesh_sdd_create(c, M.desc_for(big, M.FP32))
        try:
            M.mesh_sdd_set_monitor(h, big.rho)
            with pytest.raises(M.MeshSddError) as e:
                M.mesh_sdd_submit(h, M.make_step(big.x, big.y, big.bnd_t0, big.bnd_t1, paths_per_node=big.n_paths))
            assert e.value.code == M.E_BUDGET
        finally:
            M.mesh_sdd_destroy(h)
    finally:
        M.mesh_sdd_ctx_destroy(c)


def test_error_paths(M, ctx):
    inst = W.config1(500)
    inst.K = 20
    h = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
    try:
        m = M.mesh_sdd_num_interface_nodes(h)
        arrs, res = M.host_result(m)
        st = M.make_step(inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, paths_per_node=500)
        with pytest.raises(M.MeshSddError) as e:          # before set_monitor
            M.mesh_sdd_solve_interfaces(h, st, res)
        assert e.value.code == M.E_STATE
        bad_rho = inst.rho.copy()
        bad_rho[3, 3] = -1.0
        with pytest.raises(M.MeshSddError) as e:
            M.mesh_sdd_set_monitor(h, bad_rho)
        assert e.value.code == M.E_INVAL
        M.mesh_sdd_set_monitor(h, inst.rho)
        b = inst.bnd_t1.copy()
        b[0] += 1e-3                                      # corner (xi=0, eta=0) disagrees
        with pytest.raises(M.MeshSddError) as e:
            M.mesh_sdd_solve_interfaces(h, M.make_step(inst.x, inst.y, inst.bnd_t0, b, paths_per_node=500), res)
        assert e.value.code == M.E_INVAL
        with pytest.raises(M.MeshSddError) as e:
            M.mesh_sdd_solve_interfaces(h, M.make_step(inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, paths_per_node=0), res)
        assert e.value.code == M.E_INVAL
        # destroy with a request in flight is refused
        t = M.mesh_sdd_submit(h, st)
        try:
            M.mesh_sdd_destroy(h)
            destroyed = True
        except M.MeshSddError as e2:
            destroyed = False
            assert e2.code == M.E_STATE
        if not destroyed:
            assert M.mesh_sdd_wait(ctx, t, res, 60_000)
        else:   # the request finished before destroy: nothing left to wait for
            h = None
    finally:
        if h is not None:
            M.mesh_sdd_destroy(h)


def test_requests_beyond_32_bit_item_numbers_are_rejected(M, ctx):
    """The kernels number (node, chunk) work items in 32 bits: a request with
    more than 2^32 - 2^20 of them (FP32), or an FP64 request of 2^24 or more
    256-path blocks, is refused with E_INVAL when it is staged, before any
    allocation or launch.  Here 753 nodes at N = 2^31: 753 * 2^24 FP32 items,
    753 * 2^23 FP64 blocks.  In a batch the other request is still solved,
    with its results bitwise those of a solve alone; submitted for serving,
    the request is refused too (its partials alone exceed the budget)."""
    big, small = W.config2(1 << 31), W.config1(640)
    big.K = small.K = 20
    huge = {"paths_per_node": 1 << 31}
    for prec in (M.FP32, M.FP64):
        h = M.mesh_sdd_create(ctx, M.desc_for(big, prec))
        try:
            M.mesh_sdd_set_monitor(h, big.rho)
            arrs, res = M.host_result(M.mesh_sdd_num_interface_nodes(h))
            with pytest.raises(M.MeshSddError) as e:
                M.mesh_sdd_solve_interfaces(h, M.make_step(big.x, big.y, big.bnd_t0, big.bnd_t1, **huge), res)
            assert e.value.code == M.E_INVAL and ("work items" in str(e.value) or "FP64" in str(e.value)), str(e.value)
        finally:
            M.mesh_sdd_destroy(h)
    H = Handles(M, ctx, [big, small], M.FP32)
    try:
        st_small = M.make_step(small.x, small.y, small.bnd_t0, small.bnd_t1, paths_per_node=small.n_paths)
        a1, r1 = M.host_result(H.m[1])
        M.mesh_sdd_solve_interfaces(H.h[1], st_small, r1)
        alone = M.result_dict(a1, r1, H.m[1])
        pairs = [M.host_result(m) for m in H.m]
        st_big = M.make_step(big.x, big.y, big.bnd_t0, big.bnd_t1, **huge)
        with pytest.raises(M.MeshSddError) as e:
            M.mesh_sdd_solve_batch(H.h, [st_big, st_small], [r for _, r in pairs])
        assert e.value.code == M.E_INVAL
        assert same(alone, M.result_dict(pairs[1][0], pairs[1][1], H.m[1]))
        with pytest.raises(M.MeshSddError) as e:
            t = M.mesh_sdd_submit(H.h[0], st_big)
            M.mesh_sdd_wait(ctx, t, pairs[0][1], 60_000)
        assert e.value.code in (M.E_BUDGET, M.E_INVAL)
    finally:
        H.close()


def test_degenerate_cases(M, ctx):
    # no interface node at all
    inst = W.constant_problem(9, 1, 0, 0, tau=0.01, K=10, n_paths=100)
    h = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
    try:
        M.mesh_sdd_set_monitor(h, inst.rho)
        assert M.mesh_sdd_num_interface_nodes(h) == 0
        arrs, res = M.host_result(0)
        M.mesh_sdd_solve_interfaces(h, M.make_step(inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, paths_per_node=100), res)
        assert res.executed_path_steps == 0
    finally:
        M.mesh_sdd_destroy(h)
    # one path per node: SE is NaN, the mean is the single path's value
    inst = W.config1(1)
    inst.K = 30
    for prec in (M.FP32, M.FP64):
        g = M.solve_instance(ctx, inst, prec)
        assert np.all(np.isnan(g["se_x"])) and np.all(np.isfinite(g["mean_x"]))


def test_device_pointers_match_host(M, ctx):
    import torch
    inst = W.config1(2000)
    inst.K = 60
    dev = torch.device("cuda:0")
    h = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
    try:
        m = M.mesh_sdd_num_interface_nodes(h)
        M.mesh_sdd_set_monitor(h, torch.from_numpy(inst.rho).to(dev))
        tx, ty = torch.from_numpy(inst.x).to(dev), torch.from_numpy(inst.y).to(dev)
        t0, t1 = torch.from_numpy(inst.bnd_t0).to(dev), torch.from_numpy(inst.bnd_t1).to(dev)
        outs = [torch.full((m,), float("nan"), dtype=torch.float64, device=dev) for _ in range(5)]
        torch.cuda.synchronize()
        res = M.make_result(*outs)
        M.mesh_sdd_solve_interfaces(h, M.make_step(tx, ty, t0, t1, paths_per_node=2000), res)
        torch.cuda.synchronize()
        g_dev = {k: o.cpu().numpy() for k, o in zip(("mean_x", "mean_y", "se_x", "se_y", "exit_frac"), outs)}
        g_dev["executed_path_steps"] = int(res.executed_path_steps)
        M.mesh_sdd_set_monitor(h, inst.rho)
        arrs, res2 = M.host_result(m)
        M.mesh_sdd_solve_interfaces(h, M.make_step(inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, paths_per_node=2000), res2)
        assert same(g_dev, M.result_dict(arrs, res2, m))
    finally:
        M.mesh_sdd_destroy(h)


def test_target_se_sets_path_count(M, ctx):
    inst = W.config1(1)
    inst.K = 40
    h = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
    try:
        M.mesh_sdd_set_monitor(h, inst.rho)
        m = M.mesh_sdd_num_interface_nodes(h)
        arrs, res = M.host_result(m)
        se = 3e-3
        st = M.make_step(inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, target_se=se)
        M.mesh_sdd_solve_interfaces(h, st, res)
        want = int(np.ceil(2 * inst.tau * 1.0 / se ** 2))
        assert res.paths_per_node == want
        g = M.result_dict(arrs, res, m)
        assert np.max(np.maximum(g["se_x"], g["se_y"])) <= se
    finally:
        M.mesh_sdd_destroy(h)


def test_lds_and_l2_monitor_give_identical_results(M, ctx):
    """A single-instance launch reads rho and dt rho_xi from an LDS copy of
    the node tables (level 2, 8 B per node), or, on grids too large for
    that, from 140 x 140-node windows of them around blocks of interface
    nodes, falling back to the cell records for paths outside the window
    (level 3); with monitor_table = 1 it reads the same corner values from
    the cell records in L2.  All must give bitwise equal results.  The 257^2
    instance runs with tau = 0.05 (path spread sqrt(2 tau) = 0.32, against
    window margins of 45 cells = 0.18), so most of its paths leave their
    window."""
    rng = np.random.default_rng(9)
    insts = [W.random_instance(rng, q, n_paths=4000, sizes=(n,)) for q, n in enumerate((33, 129, 161, 65, 257))]
    for q, it in enumerate(insts):
        it.K = 60 + 13 * q
        it.instance_id = 300 + q
    insts[4].tau = 0.05
    H = Handles(M, ctx, insts, M.FP32)
    try:
        levels = [M.mesh_sdd_get_launch(h).table_level for h in H.h]
        assert levels == [2, 2, 3, 2, 3], levels
        lds = solve_alone(M, H, insts)
        M.mesh_sdd_set_launch(ctx, M.make_launch(monitor_table=1))
        try:
            assert all(M.mesh_sdd_get_launch(h).table_level == 0 for h in H.h)
            l2 = solve_alone(M, H, insts)
        finally:
            M.mesh_sdd_set_launch(ctx, None)
        for q in range(len(insts)):
            assert same(lds[q], l2[q]), insts[q].name
        say("LDS tables (levels %s) == L2 records (bitwise) on %s" % (levels, ", ".join(it.name for it in insts)))
    finally:
        H.close()


def non_square(n_xi, n_eta, sub_xi, sub_eta, per_xi, Lx, Ly, instance_id):
    x, y = W.uniform_mesh(n_xi, n_eta, Lx, Ly)
    if per_xi:
        ux, uy = W.tanh_front_grad(x, y, 0.0, 0.05 * Lx, Lx=Lx, phase=0.3 * Lx)
    else:
        ux, uy = W.gaussian_bump_grad(x, y, 0.4 * Lx, 0.6 * Ly, 0.02 * max(Lx, Ly) ** 2)
    rho = W.arc_length_monitor(ux, uy, 1.0)
    b = W.boundary_from_mesh(x, y)
    return W.Instance("rect%dx%d" % (n_xi, n_eta), n_xi, n_eta, sub_xi, sub_eta, per_xi, 0, Lx, Ly, 0.02, 80, 3000,
                      rho, x, y, b, b.copy(), seed=11, instance_id=instance_id)


def test_windows_of_non_square_grids(M, ctx, oracle_lib):
    """449 x 65 (xi periodic, Lx = 3, Ly = 0.5) and 65 x 449 (Dirichlet):
    too large for the whole tables, so both run the windowed kernel with
    301 x 65 and 65 x 301 windows over blocks of 211 nodes along the long
    axis.  Alone, batched together, and from the cell records: bitwise
    equal; sampled nodes of the periodic one against the oracle."""
    from gpu_helpers import compare, oracle_solve
    insts = [non_square(449, 65, 8, 2, 1, 3.0, 0.5, 41), non_square(65, 449, 2, 8, 0, 0.5, 3.0, 42)]
    H = Handles(M, ctx, insts, M.FP32)
    try:
        assert [M.mesh_sdd_get_launch(h).table_level for h in H.h] == [3, 3]
        alone = solve_alone(M, H, insts)
        pairs = [M.host_result(m) for m in H.m]
        M.mesh_sdd_solve_batch(H.h, steps_for(M, insts), [r for _, r in pairs])
        batched = [M.result_dict(a, r, m) for (a, r), m in zip(pairs, H.m)]
        M.mesh_sdd_set_launch(ctx, M.make_launch(monitor_table=1))
        try:
            l2 = solve_alone(M, H, insts)
        finally:
            M.mesh_sdd_set_launch(ctx, None)
        for q, it in enumerate(insts):
            assert same(alone[q], batched[q]), it.name
            assert same(alone[q], l2[q]), it.name
        nodes = np.unique(np.linspace(0, H.m[0] - 1, 5).astype(np.int32))
        ora = oracle_solve(oracle_lib, insts[0], nodes=nodes)
        s = compare(alone[0], ora, nodes=nodes, label="rect449x65 windowed vs oracle")
        assert s["err"] <= 1e-5
        say("non-square windows: alone == batched == cell records (bitwise) on %s"
            % ", ".join(it.name for it in insts))
    finally:
        H.close()


def edge_instance(n, sub, per_xi, K, N, instance_id):
    x, y = W.uniform_mesh(n, n)
    ux, uy = W.gaussian_bump_grad(x, y, 0.45, 0.55, 0.05)
    rho = W.arc_length_monitor(ux, uy, 2.0)
    b = W.boundary_from_mesh(x, y)
    return W.Instance("edge%d_%dx%d_K%d_N%d" % (n, sub[0], sub[1], K, N), n, n, sub[0], sub[1], per_xi, 0, 1.0, 1.0,
                      0.01, K, N, rho, x, y, b, b.copy(), seed=3, instance_id=instance_id)


def test_edge_instances_alone_batched_and_against_the_oracle(M, ctx, oracle_lib):
    """Limits of the stepping loop and of the windows, in one batch and
    alone: the smallest grid (4 x 4, every interior node an interface node)
    with K = 1 and a single partial chunk (N = 65); a 5 x 5 grid periodic in
    xi with K = 3 (less than one quarter of four substeps) and N = 129 (a full
    chunk and one path); a 161^2 grid cut into window blocks with K = 7.
    Alone and batched must agree bitwise; every node of the small grids and
    sampled nodes of the large one against the oracle."""
    from gpu_helpers import compare, oracle_solve
    insts = [edge_instance(4, (3, 3), 0, 1, 65, 51), edge_instance(5, (4, 1), 1, 3, 129, 52),
             edge_instance(161, (8, 8), 0, 7, 200, 53)]
    H = Handles(M, ctx, insts, M.FP32)
    try:
        alone = solve_alone(M, H, insts)
        pairs = [M.host_result(m) for m in H.m]
        M.mesh_sdd_solve_batch(H.h, steps_for(M, insts), [r for _, r in pairs])
        batched = [M.result_dict(a, r, m) for (a, r), m in zip(pairs, H.m)]
        for q, it in enumerate(insts):
            assert same(alone[q], batched[q]), it.name
            nodes = None if H.m[q] < 100 else np.unique(np.linspace(0, H.m[q] - 1, 6).astype(np.int32))
            ora = oracle_solve(oracle_lib, it, nodes=nodes)
            s = compare(alone[q], ora, nodes=nodes, label=it.name)
            assert s["err"] <= 1e-5 and s["flips"] == 0, it.name
            steps = alone[q]["executed_path_steps"]
            assert 0 < steps <= H.m[q] * it.n_paths * it.K
    finally:
        H.close()


def test_serving_blocked_grids_over_several_ticks(M):
    """Served requests on grids cut into window blocks, each large enough
    (~10^10 path-steps) to be split over several scheduler ticks, so the
    windowed jobs of a tick cover partial runs of a block's items: the
    results must equal the requests solved alone, bitwise."""
    rng = np.random.default_rng(21)
    insts = [W.random_instance(rng, 0, n_paths=20000, sizes=(257,), subs=(8,)),
             W.random_instance(rng, 1, n_paths=20000, sizes=(161,), subs=(8,)),
             W.random_instance(rng, 2, n_paths=3000, sizes=(65,))]
    for q, it in enumerate(insts):
        it.instance_id = 400 + q
    c = M.mesh_sdd_ctx_create(0)
    H = Handles(M, c, insts, M.FP32)
    try:
        assert [M.mesh_sdd_get_launch(h).table_level for h in H.h[:2]] == [3, 3]
        alone = solve_alone(M, H, insts)
        ticks0 = M.mesh_sdd_ctx_stats(c).ticks
        tickets = [M.mesh_sdd_submit(h, s) for h, s in zip(H.h, steps_for(M, insts))]
        outs = []
        for q, t in enumerate(tickets):
            arrs, res = M.host_result(H.m[q])
            assert M.mesh_sdd_wait(c, t, res, 120_000)
            outs.append(M.result_dict(arrs, res, H.m[q]))
        ticks = M.mesh_sdd_ctx_stats(c).ticks - ticks0
        work = [H.m[q] * it.n_paths * it.K for q, it in enumerate(insts)]
        say("served %s over %d ticks (nominal %.2e path-steps)" % ([it.name for it in insts], ticks, sum(work)))
        assert ticks >= 3
        for q, it in enumerate(insts):
            assert same(alone[q], outs[q]), it.name
    finally:
        H.close()
        M.mesh_sdd_ctx_destroy(c)
