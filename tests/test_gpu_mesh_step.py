"""The mesh step on the GPU (edge generator, subdomain solves, single-domain
reference, arc-length monitor, mesh quality, the whole MP step) against the
plain FP64 oracle of ``oracle/mp_oracle.py``, through the C-ABI.

Both sides compute the same IEEE operations in the same order (the kernels
are built without floating-point contraction), so the tolerances are a few
ulps of the mesh coordinates.  At the full 129x129 / 257x257 sizes, where
the oracle's plain loops are too slow, the checks are the exact discrete
mode decay (interfaces on the mode's nodal lines) and agreement of the two
independent solver kernels (LDS-resident subdomains vs whole-grid sweeps)."""
import math

import numpy as np
import pytest

import oracle
from oracle import mp_oracle as mp
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


def grid(nx, ny):
    return np.meshgrid(np.arange(nx) / (nx - 1), np.arange(ny) / (ny - 1))


def case_inputs(nx, ny, px, py, Lx=1.0, Ly=1.0, seed=0, amp=0.01):
    """Smooth monitor, a perturbed (quasi-periodic where periodic) mesh and
    its boundary arrays."""
    rng = np.random.default_rng(seed)
    XI, ETA = grid(nx, ny)
    a, b, c = rng.uniform(0.5, 1.5, 3)
    rho = 1.0 + 0.6 * np.sin(2 * np.pi * XI + a) ** 2 * np.cos(2 * np.pi * ETA + b) ** 2 + 0.3 * c
    bump_x = np.sin(np.pi * XI) if not px else np.sin(2 * np.pi * XI)
    bump_y = np.sin(np.pi * ETA) if not py else np.sin(2 * np.pi * ETA)
    m = bump_x * bump_y
    x = Lx * XI + amp * m * rng.uniform(0.5, 1.0)
    y = Ly * ETA - amp * m * rng.uniform(0.5, 1.0)
    return rho, x, y, W.boundary_from_mesh(x, y)


def make_inst(M, ctx, nx, ny, sx, sy, px, py, Lx=1.0, Ly=1.0, tau=0.01, K=40, prec=None, rho=None):
    d = M.make_desc(nx, ny, sx, sy, px, py, K=K, Lx=Lx, Ly=Ly, tau=tau,
                    precision=M.FP64 if prec is None else prec)
    h = M.mesh_sdd_create(ctx, d)
    if rho is not None:
        M.mesh_sdd_set_monitor(h, rho)
    return h


CASES = [
    # name, nx, ny, sub_xi, sub_eta, per_xi, per_eta, Lx, Ly
    ("dir33_4x4", 33, 33, 4, 4, 0, 0, 1.0, 1.0),
    ("ragged31x13_3x4", 31, 13, 3, 4, 0, 0, 1.5, 0.7),
    ("perx33x17_2x2", 33, 17, 2, 2, 1, 0, 2.0, 1.0),
    ("pery17x21_2x4", 17, 21, 2, 4, 0, 1, 1.0, 2.0),
    ("perxy17_2x2", 17, 17, 2, 2, 1, 1, 2.0, 2.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_edge_generator_matches_oracle(M, ctx, case):
    name, nx, ny, sx, sy, px, py, Lx, Ly = case
    rho, x, y, b0 = case_inputs(nx, ny, px, py, Lx, Ly, seed=1)
    h = make_inst(M, ctx, nx, ny, sx, sy, px, py, Lx, Ly, rho=rho)
    try:
        got = np.empty_like(b0)
        M.mesh_sdd_edge_generate(h, b0, got)
        want = mp.edge_generate(rho, b0, 0.01, px, py, Lx, Ly)
        err = float(np.max(np.abs(got - want)))
        say("%s edge generator: max |gpu - oracle| = %.3e, moved %.3e" % (name, err, np.max(np.abs(want - b0))))
        assert err <= 1e-13
    finally:
        M.mesh_sdd_destroy(h)


@pytest.mark.parametrize("solver", [0, 2], ids=["lds", "sweep"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_subdomain_solve_matches_oracle(M, ctx, case, solver):
    name, nx, ny, sx, sy, px, py, Lx, Ly = case
    rho, x, y, b0 = case_inputs(nx, ny, px, py, Lx, Ly, seed=2)
    h = make_inst(M, ctx, nx, ny, sx, sy, px, py, Lx, Ly, rho=rho)
    try:
        b1 = mp.edge_generate(rho, b0, 0.01, px, py, Lx, Ly)
        I, J = M.mesh_sdd_interface_nodes(h)
        rng = np.random.default_rng(3)
        ix = x[J, I] + 1e-3 * rng.standard_normal(len(I))
        iy = y[J, I] + 1e-3 * rng.standard_normal(len(I))
        gx, gy = np.empty_like(x), np.empty_like(y)
        M.mesh_sdd_subdomain_solve(h, x, y, b1, ix, iy, gx, gy, M.make_mp_opts(solver=solver))
        wx, wy = mp.subdomain_solve(rho, x, y, b1, ix, iy, 0.01, sx, sy, px, py, Lx, Ly)
        err = max(float(np.max(np.abs(gx - wx))), float(np.max(np.abs(gy - wy))))
        say("%s subdomain solve (%s): max |gpu - oracle| = %.3e" % (name, ["auto", "", "sweep"][solver], err))
        assert err <= 1e-13
    finally:
        M.mesh_sdd_destroy(h)


@pytest.mark.parametrize("case", [c for c in CASES if c[0] != "ragged31x13_3x4"], ids=lambda c: c[0])
def test_single_domain_matches_oracle(M, ctx, case):
    name, nx, ny, sx, sy, px, py, Lx, Ly = case
    rho, x, y, b0 = case_inputs(nx, ny, px, py, Lx, Ly, seed=4)
    h = make_inst(M, ctx, nx, ny, sx, sy, px, py, Lx, Ly, rho=rho)
    try:
        gx, gy = np.empty_like(x), np.empty_like(y)
        M.mesh_sdd_single_domain_solve(h, x, y, b0, gx, gy)
        wx, wy = mp.single_domain_solve(rho, x, y, b0, 0.01, px, py, Lx, Ly)
        err = max(float(np.max(np.abs(gx - wx))), float(np.max(np.abs(gy - wy))))
        say("%s single domain: max |gpu - oracle| = %.3e" % (name, err))
        assert err <= 1e-13
    finally:
        M.mesh_sdd_destroy(h)


@pytest.mark.parametrize("normalize", [False, True])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_arclength_monitor_matches_oracle(M, ctx, case, normalize):
    name, nx, ny, sx, sy, px, py, Lx, Ly = case
    rho, x, y, _ = case_inputs(nx, ny, px, py, Lx, Ly, seed=5, amp=0.02)
    # a solution that is periodic where the axis is
    XI, ETA = grid(nx, ny)
    u = np.tanh(4.0 * (np.sin(2 * np.pi * XI) * np.cos(2 * np.pi * ETA))) + 0.3 * (0 if py else ETA)
    h = make_inst(M, ctx, nx, ny, sx, sy, px, py, Lx, Ly)
    try:
        M.mesh_sdd_set_monitor_arclength(h, u, x, y, 3.0, normalize)
        got = np.empty_like(u)
        M.mesh_sdd_get_monitor(h, got)
        want = mp.arclength_monitor(u, x, y, 3.0, normalize, px, py, Lx, Ly)
        err = float(np.max(np.abs(got - want) / want))
        say("%s arc-length monitor (normalize=%s): max rel diff %.3e" % (name, normalize, err))
        assert err <= 1e-14
    finally:
        M.mesh_sdd_destroy(h)


def test_mesh_quality_matches_oracle(M, ctx):
    for seed, (nx, ny) in enumerate(((33, 33), (31, 13), (129, 129))):
        _, xs, ys, _ = case_inputs(nx, ny, 0, 0, seed=10 + seed, amp=0.02)
        _, xd, yd, _ = case_inputs(nx, ny, 0, 0, seed=20 + seed, amp=0.02)
        h = make_inst(M, ctx, nx, ny, 2 if (nx - 1) % 2 == 0 else 3, 2 if (ny - 1) % 2 == 0 else 3, 0, 0)
        try:
            r = np.empty((ny - 1, nx - 1))
            rmax, rmean = M.mesh_sdd_mesh_quality(h, xs, ys, xd, yd, r)
            wr, wmax, wmean = mp.quality_ratio(xs, ys, xd, yd)
            say("quality %dx%d: R_max %.6f R_mean %.6f (oracle %.6f %.6f)" % (nx, ny, rmax, rmean, wmax, wmean))
            assert np.max(np.abs(r - wr)) <= 1e-14
            assert abs(rmax - wmax) <= 1e-14 and abs(rmean - wmean) <= 1e-14
            assert M.mesh_sdd_mesh_quality(h, xs, ys, xs, ys) == (1.0, 1.0)
        finally:
            M.mesh_sdd_destroy(h)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mp_step_matches_oracle_composition(M, ctx, prec):
    """edge generator -> interface estimate -> subdomain solves, against the
    oracle's edge generator, Monte-Carlo estimate and subdomain solves."""
    nx, ny, sx, sy, tau, K, N = 33, 33, 2, 2, 0.01, 40, 2000
    rho, x, y, b0 = case_inputs(nx, ny, 0, 0, seed=7)
    P = M.FP64 if prec == "fp64" else M.FP32
    h = make_inst(M, ctx, nx, ny, sx, sy, 0, 0, tau=tau, K=K, prec=P, rho=rho)
    try:
        m = M.mesh_sdd_num_interface_nodes(h)
        arrs, res = M.host_result(m)
        xn, yn, bn = np.empty_like(x), np.empty_like(y), np.empty_like(b0)
        step = M.make_step(x, y, b0, b0, paths_per_node=N, mesh_step=3)
        M.mesh_sdd_mp_step(h, step, xn, yn, bn, res)
        b1 = mp.edge_generate(rho, b0, tau)
        prob = oracle.Problem(nx, ny, sx, sy, tau=tau, K=K, mesh_step=3)
        o = oracle.solve(prob, rho, x, y, b0, b1, N)
        wx, wy = mp.subdomain_solve(rho, x, y, b1, o["mean_x"], o["mean_y"], tau, sx, sy)
        e_b = float(np.max(np.abs(bn - b1)))
        e_i = float(np.max(np.abs(arrs[0][:m] - o["mean_x"])))
        e_m = max(float(np.max(np.abs(xn - wx))), float(np.max(np.abs(yn - wy))))
        say("mp step %s: boundary %.3e, interface mean_x %.3e, mesh %.3e, executed %d path-steps"
            % (prec, e_b, e_i, e_m, res.executed_path_steps))
        assert e_b <= 1e-13
        if prec == "fp64":
            assert e_i <= 1e-12 and e_m <= 1e-12
        else:
            assert e_i <= 1e-5 and e_m <= 1e-5
    finally:
        M.mesh_sdd_destroy(h)


@pytest.mark.parametrize("n,sub", [(129, 4), (257, 8)])
def test_full_size_mode_decay_and_solver_agreement(M, ctx, n, sub):
    """Headline grid sizes: the mode sin(k pi xi) sin(k pi eta) with k = the
    number of subdomains has nodal lines on every interface, so the
    decomposed solve must multiply it by exactly (1 - dt lambda)^L; both
    solver kernels must agree bitwise."""
    import torch
    tau = 0.01 if n == 129 else 0.005
    XI, ETA = grid(n, n)
    mode = np.sin(sub * np.pi * XI) * np.sin(sub * np.pi * ETA)
    x0, y0 = XI + 0.002 * mode, ETA - 0.003 * mode
    bnd = W.boundary_from_mesh(XI, ETA)
    h = make_inst(M, ctx, n, n, sub, sub, 0, 0, tau=tau, rho=np.ones((n, n)))
    try:
        I, J = M.mesh_sdd_interface_nodes(h)
        dev = torch.device("cuda:0")
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        args = [T(x0), T(y0), T(bnd), T(XI[J, I]), T(ETA[J, I])]
        outs = {}
        for solver in (1, 2):
            gx, gy = torch.empty_like(args[0]), torch.empty_like(args[1])
            M.mesh_sdd_subdomain_solve(h, *args, gx, gy, M.make_mp_opts(solver=solver))
            torch.cuda.synchronize()
            outs[solver] = (gx.cpu().numpy(), gy.cpu().numpy())
        L = mp.fe_substeps_2d(tau, n, n)
        lam = 2.0 * 4.0 * (n - 1) ** 2 * math.sin(sub * math.pi / (2 * (n - 1))) ** 2
        f = (1.0 - tau / L * lam) ** L
        ex = max(float(np.max(np.abs(outs[1][0] - (XI + 0.002 * f * mode)))),
                 float(np.max(np.abs(outs[1][1] - (ETA - 0.003 * f * mode)))))
        same = np.array_equal(outs[1][0], outs[2][0]) and np.array_equal(outs[1][1], outs[2][1])
        say("%dx%d %dx%d: L=%d, decay factor %.6f, max |gpu - closed form| %.3e, lds == sweep: %s"
            % (n, n, sub, sub, L, f, ex, same))
        assert ex <= 1e-13
        assert same
    finally:
        M.mesh_sdd_destroy(h)


def test_mesh_step_error_paths(M, ctx):
    n = 17
    rho, x, y, b0 = case_inputs(n, n, 0, 0)
    h = make_inst(M, ctx, n, n, 2, 2, 0, 0)
    try:
        out = np.empty_like(b0)
        with pytest.raises(M.MeshSddError) as e:                 # before set_monitor
            M.mesh_sdd_edge_generate(h, b0, out)
        assert e.value.code == M.E_STATE
        M.mesh_sdd_set_monitor(h, rho)
        bad = M.make_mp_opts(solver=3)
        with pytest.raises(M.MeshSddError) as e:
            M.mesh_sdd_edge_generate(h, b0, out, bad)
        assert e.value.code == M.E_INVAL
        bad = M.make_mp_opts(fe_cfl=1.5)
        gx, gy = np.empty_like(x), np.empty_like(y)
        I, J = M.mesh_sdd_interface_nodes(h)
        with pytest.raises(M.MeshSddError) as e:
            M.mesh_sdd_subdomain_solve(h, x, y, b0, x[J, I], y[J, I], gx, gy, bad)
        assert e.value.code == M.E_INVAL
        with pytest.raises(M.MeshSddError) as e:                 # output aliases input
            M.mesh_sdd_subdomain_solve(h, x, y, b0, x[J, I], y[J, I], x, gy)
        assert e.value.code == M.E_INVAL
        # a degenerate mesh has no finite monitor
        with pytest.raises(M.MeshSddError) as e:
            M.mesh_sdd_set_monitor_arclength(h, x, np.zeros_like(x), y, 1.0)
        assert e.value.code == M.E_INVAL
    finally:
        M.mesh_sdd_destroy(h)
    # a 129x129 subdomain (2x2 of 257) does not fit in LDS
    n = 257
    h = make_inst(M, ctx, n, n, 2, 2, 0, 0, tau=0.0005, rho=np.ones((n, n)))
    try:
        XI, ETA = grid(n, n)
        I, J = M.mesh_sdd_interface_nodes(h)
        gx, gy = np.empty_like(XI), np.empty_like(ETA)
        bnd = W.boundary_from_mesh(XI, ETA)
        with pytest.raises(M.MeshSddError) as e:
            M.mesh_sdd_subdomain_solve(h, XI, ETA, bnd, XI[J, I], ETA[J, I], gx, gy, M.make_mp_opts(solver=1))
        assert e.value.code == M.E_INVAL
        M.mesh_sdd_subdomain_solve(h, XI, ETA, bnd, XI[J, I], ETA[J, I], gx, gy)   # automatic: sweeps
        assert np.max(np.abs(gx - XI)) < 1e-13 and np.max(np.abs(gy - ETA)) < 1e-13
    finally:
        M.mesh_sdd_destroy(h)


def test_mp_step_edge_cases(M, ctx):
    """No interface node at all (1x1 Dirichlet: the step is the edge generator
    plus one subdomain = the whole grid); a periodic axis with one subdomain
    (the seam alone is the interface); device arrays in and out; the edge
    generator in place; K not a multiple of 4."""
    import torch
    dev = torch.device("cuda:0")
    # 1x1 Dirichlet: M = 0, the mesh step equals edge generator + single domain
    n, tau = 21, 0.01
    rho, x, y, b0 = case_inputs(n, n, 0, 0, seed=31)
    h = make_inst(M, ctx, n, n, 1, 1, 0, 0, tau=tau, K=30, rho=rho)
    try:
        assert M.mesh_sdd_num_interface_nodes(h) == 0
        arrs, res = M.host_result(0)
        xn, yn, bn = np.empty_like(x), np.empty_like(y), np.empty_like(b0)
        M.mesh_sdd_mp_step(h, M.make_step(x, y, b0, b0, paths_per_node=100), xn, yn, bn, res)
        assert res.executed_path_steps == 0
        b1 = mp.edge_generate(rho, b0, tau)
        wx, wy = mp.single_domain_solve(rho, x, y, b1, tau)
        e = max(float(np.max(np.abs(xn - wx))), float(np.max(np.abs(yn - wy))), float(np.max(np.abs(bn - b1))))
        say("1x1 Dirichlet mesh step (no interface node): max |gpu - oracle| %.3e" % e)
        assert e <= 1e-13
    finally:
        M.mesh_sdd_destroy(h)
    # xi periodic with one subdomain: interface = the seam; device arrays; K = 30
    nx, ny, Lx = 25, 17, 2.0
    rho, x, y, b0 = case_inputs(nx, ny, 1, 0, Lx, 1.0, seed=32)
    h = make_inst(M, ctx, nx, ny, 1, 2, 1, 0, Lx, 1.0, tau=tau, K=30, rho=rho)
    try:
        m = M.mesh_sdd_num_interface_nodes(h)
        I, J = M.mesh_sdd_interface_nodes(h)
        assert np.all((I == 0) | (J == (ny - 1) // 2))
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        outs = [torch.empty(m, dtype=torch.float64, device=dev) for _ in range(5)]
        res = M.make_result(*outs)
        xn, yn, bn = T(np.zeros_like(x)), T(np.zeros_like(y)), T(np.zeros_like(b0))
        step = M.make_step(T(x), T(y), T(b0), T(b0), paths_per_node=700, mesh_step=5)
        M.mesh_sdd_mp_step(h, step, xn, yn, bn, res)
        torch.cuda.synchronize()
        b1 = mp.edge_generate(rho, b0, tau, 1, 0, Lx, 1.0)
        est = oracle.solve(oracle.Problem(nx, ny, 1, 2, 1, 0, Lx, 1.0, tau=tau, K=30, mesh_step=5), rho, x, y, b0,
                           b1, 700, threads=8)
        wx, wy = mp.subdomain_solve(rho, x, y, b1, est["mean_x"], est["mean_y"], tau, 1, 2, 1, 0, Lx, 1.0)
        gx, gy, gb = xn.cpu().numpy(), yn.cpu().numpy(), bn.cpu().numpy()
        e = max(float(np.max(np.abs(gx - wx))), float(np.max(np.abs(gy - wy))), float(np.max(np.abs(gb - b1))))
        say("seam-only periodic mesh step on device arrays (M=%d, K=30): max |gpu - oracle| %.3e" % (m, e))
        assert e <= 1e-12
        # the edge generator in place on a device array
        bd = T(b0)
        M.mesh_sdd_edge_generate(h, bd, bd)
        torch.cuda.synchronize()
        assert np.max(np.abs(bd.cpu().numpy() - b1)) <= 1e-14
    finally:
        M.mesh_sdd_destroy(h)
