"""Interface subsampling on the GPU (interface_stride > 1): the nodes that
run paths reproduce the full run bit for bit (they keep their random
streams), the others equal the oracle's Keys interpolation along their
interface line of the same estimates, and the whole result matches the
oracle's estimate-then-interpolate on the same streams.  Dirichlet and
periodic axes, strides down to two segments per line, FP64 and FP32, the
serving path, the mesh step, and the full-size rotating bump."""

import numpy as np
import pytest

import oracle
from oracle import mp_oracle
from oracle import subsample as ss
from paper_1504_00084_amd import workloads as W
from gpu_helpers import THREADS, say

pytestmark = pytest.mark.gpu

KEYS = ("mean_x", "mean_y", "se_x", "se_y", "exit_frac")


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


def small_instance(n, sub, per_xi, per_eta, K=60, N=1500):
    """n x n grid, sub_xi x sub_eta subdomains, a bump monitor periodic in
    both directions, and boundary data at t^{n+1} that slides the boundary
    nodes along their sides (corners fixed)."""
    x, y = W.uniform_mesh(n, n)
    rho = 1.0 + 3.0 * np.exp(-(np.sin(np.pi * (x - 0.4)) ** 2 + np.sin(np.pi * (y - 0.6)) ** 2) / 0.05)
    b0 = W.boundary_from_mesh(x, y)
    b1 = W.boundary_from_mesh(x + 0.02 * np.sin(np.pi * x), y + 0.02 * np.sin(np.pi * y))
    name = "n%d_%dx%d_per%d%d" % (n, sub[0], sub[1], per_xi, per_eta)
    return W.Instance(name, n, n, sub[0], sub[1], per_xi, per_eta, 1.0, 1.0, 0.01, K, N, rho, x, y, b0, b1)


def solve(M, ctx, inst, precision, stride, n_paths=None):
    h = M.mesh_sdd_create(ctx, M.desc_for(inst, precision))
    try:
        M.mesh_sdd_set_monitor(h, np.ascontiguousarray(inst.rho))
        m = M.mesh_sdd_num_interface_nodes(h)
        arrs, res = M.host_result(m)
        st = M.make_step(inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, paths_per_node=n_paths or inst.n_paths,
                         mesh_step=inst.mesh_step, interface_stride=stride)
        M.mesh_sdd_solve_interfaces(h, st, res)
        return M.result_dict(arrs, res, m)
    finally:
        M.mesh_sdd_destroy(h)


def check_against_full(P, full, sub, stride, bnd1, label):
    """Sampled ranks equal the full run; the others equal the oracle's
    interpolation of the full run's values at the sampled ranks."""
    m = ss.sampled(P, stride)
    for k in KEYS:
        assert np.array_equal(sub[k][m], full[k][m]), (label, k)
    want = ss.interpolate(P, full["mean_x"], full["mean_y"], full["se_x"], full["se_y"], full["exit_frac"],
                          bnd1, stride)
    dm = max(np.max(np.abs(sub["mean_x"][~m] - want[0][~m])), np.max(np.abs(sub["mean_y"][~m] - want[1][~m])))
    dse = max(np.max(np.abs(sub["se_x"][~m] / want[2][~m] - 1.0)), np.max(np.abs(sub["se_y"][~m] / want[3][~m] - 1.0)))
    say("%s stride %d: %d of %d nodes run paths; interpolated max|d mean| %.2e, max rel d se %.2e"
        % (label, stride, int(m.sum()), len(m), dm, dse))
    assert dm <= 1e-13 and dse <= 1e-12
    assert np.isnan(sub["exit_frac"][~m]).all()
    return m


CASES = [((33, (2, 1), 0, 0), (2, 4, 16)),      # one vertical line; stride 16 leaves two segments
         ((33, (4, 4), 0, 0), (2, 4, 8)),
         ((33, (4, 4), 1, 0), (2, 8)),         # periodic xi: the seam column is a line too
         ((33, (2, 2), 1, 1), (4, 8)),         # doubly periodic
         ((257, (8, 8), 1, 0), (2, 4))]        # grid above 140^2: windowed kernel, sampled lists in block order


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case,strides", CASES,
                         ids=["33_2x1", "33_4x4", "33_4x4_perxi", "33_2x2_perboth", "257_8x8_perxi"])
def test_sampled_nodes_equal_full_run_and_rest_interpolated(M, ctx, case, strides, precision):
    n, sub, px, py = case
    inst = small_instance(n, sub, px, py)
    prec = M.FP64 if precision == "fp64" else M.FP32
    label = inst.name + "_" + precision
    say("case %s" % label)
    P = oracle.Problem(**inst.problem_kwargs())
    full = solve(M, ctx, inst, prec, 0)
    for s in strides:
        sub_res = solve(M, ctx, inst, prec, s)
        m = check_against_full(P, full, sub_res, s, inst.bnd_t1, label)
        steps_ratio = sub_res["executed_path_steps"] / full["executed_path_steps"]
        assert 0.0 < steps_ratio < 1.0 and abs(steps_ratio - m.mean()) < 0.25


def test_fp64_against_oracle_estimate_then_interpolate(M, ctx):
    inst = small_instance(33, (4, 4), 1, 0, N=1000)
    P = oracle.Problem(**inst.problem_kwargs())
    stride = 4
    m = ss.sampled(P, stride)
    ranks = np.nonzero(m)[0]
    say("oracle FP64 on %d sampled nodes" % len(ranks))
    ora = oracle.solve(P, inst.rho, inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, inst.n_paths, nodes=ranks,
                       threads=THREADS)
    full = {k: np.zeros(len(m)) for k in KEYS}
    for k in KEYS:
        full[k][ranks] = ora[k]
    want = ss.interpolate(P, full["mean_x"], full["mean_y"], full["se_x"], full["se_y"], full["exit_frac"],
                          inst.bnd_t1, stride)
    got = solve(M, ctx, inst, M.FP64, stride)
    err = max(np.max(np.abs(got["mean_x"] - want[0])), np.max(np.abs(got["mean_y"] - want[1])))
    serr = max(np.max(np.abs(got["se_x"] - want[2])), np.max(np.abs(got["se_y"] - want[3])))
    say("33x33 4x4 periodic-xi stride 4, FP64 vs oracle: max|d mean| %.2e, max|d se| %.2e" % (err, serr))
    assert err <= 1e-9 and serr <= 1e-9
    assert np.array_equal(np.isnan(got["exit_frac"]), ~m)
    assert np.max(np.abs(got["exit_frac"][m] - want[4][m])) <= 1e-12


def test_fp32_full_size_rotating_bump_stride4(M, ctx):
    """The bench workload (129x129, 4x4, N = 1e5, K = 500): stride 4 runs
    paths at a quarter of the line nodes (plus crossings), each equal to
    the full run's, and the rest equals the oracle's interpolation."""
    inst = W.config2()
    P = oracle.Problem(**inst.problem_kwargs())
    full = solve(M, ctx, inst, M.FP32, 0)
    sub = solve(M, ctx, inst, M.FP32, 4)
    m = check_against_full(P, full, sub, 4, inst.bnd_t1, inst.name + "_fp32")
    # the interpolation error against the full run's estimates at the other
    # nodes, in units of their standard error
    z = np.abs(sub["mean_x"][~m] - full["mean_x"][~m]) / full["se_x"][~m]
    say("129x129 stride 4: %d of %d nodes run paths, path kernel %.1f ms vs %.1f ms; interpolated minus "
        "estimated: median %.2f se, max %.2f se" % (int(m.sum()), len(m), sub["device_ms"], full["device_ms"],
                                                     float(np.median(z)), float(np.max(z))))
    assert sub["device_ms"] < 0.6 * full["device_ms"]


def test_serving_path_gives_the_blocking_result(M, ctx):
    inst = small_instance(33, (4, 4), 0, 0, N=3000)
    blocking = solve(M, ctx, inst, M.FP32, 4)
    h = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
    try:
        M.mesh_sdd_set_monitor(h, np.ascontiguousarray(inst.rho))
        m = M.mesh_sdd_num_interface_nodes(h)
        tk = M.mesh_sdd_submit(h, M.make_step(inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, paths_per_node=3000,
                                              interface_stride=4))
        arrs, res = M.host_result(m)
        M.mesh_sdd_wait(ctx, tk, res, 60000)
        served = M.result_dict(arrs, res, m)
    finally:
        M.mesh_sdd_destroy(h)
    for k in KEYS:
        assert np.array_equal(served[k], blocking[k], equal_nan=True), k


def test_invalid_strides_are_rejected(M, ctx):
    inst = small_instance(33, (2, 2), 0, 0, N=10)
    h = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
    try:
        M.mesh_sdd_set_monitor(h, np.ascontiguousarray(inst.rho))
        m = M.mesh_sdd_num_interface_nodes(h)
        arrs, res = M.host_result(m)
        for s in (3, 32, 7):
            with pytest.raises(M.MeshSddError) as e:
                M.mesh_sdd_solve_interfaces(h, M.make_step(inst.x, inst.y, inst.bnd_t0, inst.bnd_t1,
                                                           paths_per_node=10, interface_stride=s), res)
            assert e.value.code == M.E_INVAL
            say("stride %d rejected: %s" % (s, e.value))
        # 0 and 1 both mean every node; 16 leaves two segments per line
        r1 = {}
        for s in (0, 1, 16):
            M.mesh_sdd_solve_interfaces(h, M.make_step(inst.x, inst.y, inst.bnd_t0, inst.bnd_t1,
                                                       paths_per_node=10, interface_stride=s), res)
            r1[s] = {k: np.array(v) for k, v in M.result_dict(arrs, res, m).items() if k in KEYS}
        assert all(np.array_equal(r1[0][k], r1[1][k]) for k in KEYS)
        assert np.isnan(r1[16]["exit_frac"]).any()
    finally:
        M.mesh_sdd_destroy(h)


def test_fp64_mesh_step_with_subsampling_matches_oracle(M, ctx):
    """One FP64 mesh step (edge generator, subsampled interface estimate,
    subdomain solves) against the oracle's same sequence."""
    n, tau, K, N, stride = 17, 0.01, 20, 500, 4
    x, y = W.uniform_mesh(n, n)
    rho = 1.0 + 0.5 * np.sin(np.pi * x) ** 2 * np.sin(np.pi * y)
    b = W.boundary_from_mesh(x, y)
    h = M.mesh_sdd_create(ctx, M.make_desc(n, n, 2, 2, K=K, tau=tau, precision=M.FP64))
    try:
        M.mesh_sdd_set_monitor(h, rho)
        m = M.mesh_sdd_num_interface_nodes(h)
        arrs, res = M.host_result(m)
        xn, yn, bn = np.empty_like(x), np.empty_like(y), np.empty_like(b)
        M.mesh_sdd_mp_step(h, M.make_step(x, y, b, b, paths_per_node=N, interface_stride=stride), xn, yn, bn, res)
        got = M.result_dict(arrs, res, m)
    finally:
        M.mesh_sdd_destroy(h)
    b1 = mp_oracle.edge_generate(rho, b, tau)
    P = oracle.Problem(n, n, 2, 2, tau=tau, K=K)
    sm = ss.sampled(P, stride)
    ranks = np.nonzero(sm)[0]
    est = oracle.solve(P, rho, x, y, b, b1, N, nodes=ranks, threads=THREADS)
    full = {k: np.zeros(len(sm)) for k in KEYS}
    for k in KEYS:
        full[k][ranks] = est[k]
    ix, iy, _, _, _ = ss.interpolate(P, full["mean_x"], full["mean_y"], full["se_x"], full["se_y"],
                                     full["exit_frac"], b1, stride)
    wx, wy = mp_oracle.subdomain_solve(rho, x, y, b1, ix, iy, tau, 2, 2)
    err = float(max(np.max(np.abs(xn - wx)), np.max(np.abs(yn - wy))))
    ierr = float(max(np.max(np.abs(got["mean_x"] - ix)), np.max(np.abs(got["mean_y"] - iy))))
    say("17x17 2x2 FP64 mesh step, stride 4 (%d of %d interface nodes run paths): mesh max|d| %.2e, "
        "interface max|d| %.2e" % (len(ranks), len(sm), err, ierr))
    assert err <= 1e-11 and ierr <= 1e-11 and np.max(np.abs(bn - b1)) <= 1e-13
