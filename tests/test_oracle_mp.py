"""Pins of the mesh-step oracle (edge generator, subdomain solves, monitor,
mesh quality) against closed forms that do not come from the oracle itself.

Centred differences with forward Euler act on a Fourier mode as a scalar:
the discrete Laplacian of sin(k pi s) on a grid of spacing h is
-(4/h^2) sin^2(k pi h / 2) sin(k pi s), so after L steps of size dt the mode
is multiplied by exactly (1 - dt lambda)^L.  Interface lines placed on the
mode's nodal lines carry zero perturbation, so the decomposed solve must
reproduce the same factor.  A mesh linear in (xi, eta) under a monitor
exp(k xi + q eta) drifts uniformly at (sinh(k h_xi)/h_xi, sinh(q h_eta)/h_eta),
which forward Euler integrates exactly when the Dirichlet data move linearly
in time.  Steady states of the 1-D generator equidistribute 1/rho, and the
monitor and quality formulas are exact on linear, quadratic and bilinear
data."""
import math

import numpy as np
import pytest

import oracle
from oracle import mp_oracle as mp
from paper_1504_00084_amd import workloads as W


def lam1(k, h):
    return 4.0 / h ** 2 * math.sin(k * math.pi * h / 2.0) ** 2


def grid(n_xi, n_eta):
    xi = np.arange(n_xi) / (n_xi - 1)
    eta = np.arange(n_eta) / (n_eta - 1)
    return np.meshgrid(xi, eta)


# ---------------------------------------------------------------------------
# 1-D generator along a side
# ---------------------------------------------------------------------------
def test_edge_generator_dirichlet_mode_decay():
    n, tau, A = 17, 0.004, 0.03
    x, y = W.uniform_mesh(n, n)
    s = np.arange(n) / (n - 1)
    x[0, :] = s + A * np.sin(np.pi * s)          # tangential component on eta = 0
    b0 = W.boundary_from_mesh(x, y)
    rho = np.full((n, n), 2.5)
    L = mp.fe_substeps_1d(tau, n)
    out = mp.edge_generate(rho, b0, tau)
    got = out[mp._side_slice(n, n, 2, 0)]
    h = 1.0 / (n - 1)
    want = s + A * (1.0 - tau / L * lam1(1, h)) ** L * np.sin(np.pi * s)
    assert np.max(np.abs(got - want)) < 1e-14
    # the other sides and the normal components are untouched
    for side in (0, 1, 3):
        for comp in (0, 1):
            sl = mp._side_slice(n, n, side, comp)
            assert np.array_equal(out[sl], b0[sl])
    assert np.array_equal(out[mp._side_slice(n, n, 2, 1)], b0[mp._side_slice(n, n, 2, 1)])


def test_edge_generator_periodic_mode_and_winding():
    n, tau, A, Lx, L = 21, 0.002, 0.02, 2.0, 9
    s = np.arange(n) / (n - 1)
    v = -1.0 + Lx * s + A * np.sin(2 * np.pi * s)
    got = mp.generator_1d(v, np.zeros(n), tau, 1, Lx, L)
    h = 1.0 / (n - 1)
    want = -1.0 + Lx * s + A * (1.0 - tau / L * lam1(2, h)) ** L * np.sin(2 * np.pi * s)
    assert np.max(np.abs(got - want)) < 1e-14
    assert abs(got[-1] - got[0] - Lx) < 1e-15


@pytest.mark.parametrize("n", [17, 33])
def test_edge_generator_steady_state_equidistributes(n):
    # steady state of v_t = (rho_s / rho) v_s + v_ss = (rho v_s)_s / rho with
    # v(0) = 0, v(1) = 1 is v = int_0^s 1/rho / int_0^1 1/rho
    s = np.arange(n) / (n - 1)
    rho1 = 1.0 + 0.6 * np.sin(np.pi * s) ** 2
    rho = np.tile(rho1, (n, 1))
    x, y = W.uniform_mesh(n, n)
    b0 = W.boundary_from_mesh(x, y)
    out = mp.edge_generate(rho, b0, 3.0)
    got = out[mp._side_slice(n, n, 2, 0)]
    fine = np.linspace(0.0, 1.0, 200001)
    inv = 1.0 / (1.0 + 0.6 * np.sin(np.pi * fine) ** 2)
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (inv[1:] + inv[:-1]) * np.diff(fine))])
    want = np.interp(s, fine, cum / cum[-1])
    err = np.max(np.abs(got - want))
    assert err < 6.0 / (n - 1) ** 2          # second-order discretisation error
    # the drift moves nodes towards large rho (equidistribution), not away
    mid = n // 2
    assert got[mid // 2] > s[mid // 2]


def test_periodic_edge_steady_state_equidistributes():
    # periodic: rho v_s = C with v(s + 1) = v(s) + L, so v - v(0) is L times
    # the normalised cumulative integral of 1/rho (the offset is free)
    n, Lx = 33, 2.0
    s = np.arange(n) / (n - 1)
    rho1 = 1.0 + 0.5 * np.sin(2 * np.pi * s) ** 2 + 0.3 * np.sin(2 * np.pi * s)
    rho = np.tile(rho1[:, None], (1, n))            # varies along eta
    x, y = W.uniform_mesh(n, n, 1.0, Lx)
    b0 = W.boundary_from_mesh(x, y)
    out = mp.edge_generate(rho, b0, 3.0, periodic_xi=0, periodic_eta=1, Lx=1.0, Ly=Lx)
    got = out[mp._side_slice(n, n, 0, 1)]           # y along the side xi = 0
    fine = np.linspace(0.0, 1.0, 200001)
    inv = 1.0 / (1.0 + 0.5 * np.sin(2 * np.pi * fine) ** 2 + 0.3 * np.sin(2 * np.pi * fine))
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (inv[1:] + inv[:-1]) * np.diff(fine))])
    want = Lx * np.interp(s, fine, cum / cum[-1])
    assert np.max(np.abs((got - got[0]) - want)) < 6.0 * Lx / (n - 1) ** 2
    assert abs(got[-1] - got[0] - Lx) < 1e-13


def test_fe_step_count_is_smallest_stable_count():
    for tau in (1e-4, 5e-4, 0.002, 0.01, 0.05):
        for nx, ny in ((9, 9), (17, 33), (41, 41), (129, 129)):
            dt_max = 1.0 / (2.0 * (nx - 1) ** 2 + 2.0 * (ny - 1) ** 2)
            L = mp.fe_substeps_2d(tau, nx, ny, 0.9)
            assert tau / L <= 0.9 * dt_max * (1 + 1e-12)
            assert L == 1 or tau / (L - 1) > 0.9 * dt_max
            L1 = mp.fe_substeps_1d(tau, nx, 0.9)
            assert tau / L1 <= 0.9 * 0.5 / (nx - 1) ** 2 * (1 + 1e-12)
            assert L1 == 1 or tau / (L1 - 1) > 0.9 * 0.5 / (nx - 1) ** 2
    assert mp.fe_substeps_2d(0.002, 17, 17) == 3 and mp.fe_substeps_1d(0.004, 17) == 3


# ---------------------------------------------------------------------------
# subdomain solves
# ---------------------------------------------------------------------------
def mode_mesh(n_xi, n_eta, kx, ky, A, B, Lx=1.0, Ly=1.0, ox=0.0, oy=0.0):
    XI, ETA = grid(n_xi, n_eta)
    m = np.sin(kx * np.pi * XI) * np.sin(ky * np.pi * ETA)
    return ox + Lx * XI + A * m, oy + Ly * ETA + B * m, m


def test_single_subdomain_mode_decay_rectangular_grid():
    nx, ny, tau = 13, 17, 0.003
    x, y, m = mode_mesh(nx, ny, 1, 1, 0.02, -0.015)
    xu, yu = W.uniform_mesh(nx, ny)
    bnd = W.boundary_from_mesh(xu, yu)
    rho = np.full((ny, nx), 1.7)
    L = mp.fe_substeps_2d(tau, nx, ny)
    gx, gy = mp.subdomain_solve(rho, x, y, bnd, [], [], tau, 1, 1)
    f = (1.0 - tau / L * (lam1(1, 1.0 / (nx - 1)) + lam1(1, 1.0 / (ny - 1)))) ** L
    assert np.max(np.abs(gx - (xu + 0.02 * f * m))) < 1e-14
    assert np.max(np.abs(gy - (yu - 0.015 * f * m))) < 1e-14


@pytest.mark.parametrize("sub", [2, 4])
def test_decomposed_mode_decay_with_interfaces_on_nodal_lines(sub):
    n, tau = 17, 0.002
    x, y, m = mode_mesh(n, n, sub, sub, 0.01, 0.012)
    xu, yu = W.uniform_mesh(n, n)
    bnd = W.boundary_from_mesh(xu, yu)
    prob = oracle.Problem(n, n, sub, sub)
    I, J = oracle.interface_nodes(prob)
    ix, iy = xu[J, I], yu[J, I]           # zero perturbation on the nodal lines
    rho = np.ones((n, n))
    L = mp.fe_substeps_2d(tau, n, n)
    gx, gy = mp.subdomain_solve(rho, x, y, bnd, ix, iy, tau, sub, sub)
    h = 1.0 / (n - 1)
    f = (1.0 - tau / L * 2.0 * lam1(sub, h)) ** L
    assert np.max(np.abs(gx - (xu + 0.01 * f * m))) < 1e-14
    assert np.max(np.abs(gy - (yu + 0.012 * f * m))) < 1e-14


def test_drift_with_linear_in_time_dirichlet_data_is_exact():
    # rho = exp(k xi): the monitor table gives b = sinh(k h)/h at interior
    # nodes; x = xi + b t solves the semi-discrete problem exactly and
    # forward Euler follows it, given Dirichlet data linear in time
    nx, ny, tau, k, q, sub = 17, 13, 0.01, 1.3, -0.8, 4
    XI, ETA = grid(nx, ny)
    rho = np.exp(k * XI + q * ETA)
    hx, hy = 1.0 / (nx - 1), 1.0 / (ny - 1)
    bx, by = math.sinh(k * hx) / hx, math.sinh(q * hy) / hy
    x0, y0 = XI.copy(), ETA.copy()
    x1, y1 = XI + bx * tau, ETA + by * tau
    bnd1 = W.boundary_from_mesh(x1, y1)
    prob = oracle.Problem(nx, ny, sub, 3)
    I, J = oracle.interface_nodes(prob)
    gx, gy = mp.subdomain_solve(rho, x0, y0, bnd1, x1[J, I], y1[J, I], tau, sub, 3)
    assert np.max(np.abs(gx - x1)) < 1e-13
    assert np.max(np.abs(gy - y1)) < 1e-13
    # the wrong drift sign would move the mesh the other way
    assert np.all(gx[1:-1, 1:-1] > x0[1:-1, 1:-1]) and np.all(gy[1:-1, 1:-1] < y0[1:-1, 1:-1])


def test_periodic_single_domain_wraps():
    nx, ny, tau, Lx = 21, 13, 0.002, 2.0
    XI, ETA = grid(nx, ny)
    m = np.sin(2 * np.pi * XI) * np.sin(np.pi * ETA)
    x0 = -1.0 + Lx * XI + 0.02 * m
    y0 = ETA.copy()
    bnd = W.boundary_from_mesh(-1.0 + Lx * XI, ETA)
    rho = np.full((ny, nx), 3.0)
    L = mp.fe_substeps_2d(tau, nx, ny)
    gx, gy = mp.single_domain_solve(rho, x0, y0, bnd, tau, 1, 0, Lx, 1.0)
    f = (1.0 - tau / L * (lam1(2, 1.0 / (nx - 1)) + lam1(1, 1.0 / (ny - 1)))) ** L
    assert np.max(np.abs(gx - (-1.0 + Lx * XI + 0.02 * f * m))) < 1e-14
    assert np.max(np.abs(gy - ETA)) < 1e-15
    assert np.max(np.abs(gx[:, -1] - gx[:, 0] - Lx)) < 1e-14


def test_doubly_periodic_single_and_decomposed():
    n, tau, L2 = 17, 0.002, 2.0
    XI, ETA = grid(n, n)
    m = np.sin(2 * np.pi * XI) * np.sin(2 * np.pi * ETA)
    x0 = -1.0 + L2 * XI + 0.01 * m
    y0 = -1.0 + L2 * ETA - 0.01 * m
    xu, yu = -1.0 + L2 * XI, -1.0 + L2 * ETA
    bnd = W.boundary_from_mesh(xu, yu)
    rho = np.ones((n, n))
    L = mp.fe_substeps_2d(tau, n, n)
    f = (1.0 - tau / L * 2.0 * lam1(2, 1.0 / (n - 1))) ** L
    sx, sy = mp.single_domain_solve(rho, x0, y0, bnd, tau, 1, 1, L2, L2)
    assert np.max(np.abs(sx - (xu + 0.01 * f * m))) < 1e-14
    assert np.max(np.abs(sy - (yu - 0.01 * f * m))) < 1e-14
    # 2x2 with the seam as an interface: every interface lies on a nodal line
    prob = oracle.Problem(n, n, 2, 2, 1, 1, L2, L2)
    I, J = oracle.interface_nodes(prob)
    dx, dy = mp.subdomain_solve(rho, x0, y0, bnd, xu[J, I], yu[J, I], tau, 2, 2, 1, 1, L2, L2)
    assert np.max(np.abs(dx - sx)) < 1e-14 and np.max(np.abs(dy - sy)) < 1e-14


# ---------------------------------------------------------------------------
# monitor on the new mesh
# ---------------------------------------------------------------------------
def test_arclength_monitor_exact_for_linear_u_on_curved_mesh():
    n, a, b, alpha = 19, 0.7, -1.9, 3.0
    x, y, _ = mode_mesh(n, n, 1, 2, 0.04, 0.03)
    u = a * x + b * y
    rho = mp.arclength_monitor(u, x, y, alpha)
    assert np.max(np.abs(rho - math.sqrt(1.0 + alpha * (a * a + b * b)))) < 1e-12
    rn = mp.arclength_monitor(u, x, y, alpha, normalize=True)
    assert np.max(np.abs(rn - math.sqrt(1.0 + alpha))) < 1e-12


def test_arclength_monitor_periodic_wrap():
    nx, ny, Lx, c = 21, 15, 2.0, 1.4
    XI, ETA = grid(nx, ny)
    x = -1.0 + Lx * XI + 0.03 * np.sin(2 * np.pi * XI) * np.sin(np.pi * ETA)
    y = ETA + 0.02 * np.sin(2 * np.pi * XI) * np.sin(np.pi * ETA)
    u = c * y                                  # periodic in xi (y does not wind)
    rho = mp.arclength_monitor(u, x, y, 2.0, periodic_xi=1, Lx=Lx)
    assert np.max(np.abs(rho - math.sqrt(1.0 + 2.0 * c * c))) < 1e-12


def test_arclength_monitor_quadratic_on_uniform_mesh():
    n, alpha = 11, 0.5
    x, y = W.uniform_mesh(n, n)
    u = x * x + 3.0 * y * y
    rho = mp.arclength_monitor(u, x, y, alpha)
    want = np.sqrt(1.0 + alpha * (4 * x * x + 36 * y * y))
    assert np.max(np.abs(rho - want)) < 1e-12


# ---------------------------------------------------------------------------
# mesh quality
# ---------------------------------------------------------------------------
def test_quality_closed_forms():
    n = 9
    x, y = W.uniform_mesh(n, n)
    assert np.max(np.abs(mp.cell_quality(x, y) - 1.0)) < 1e-14
    s = 0.35
    q = mp.cell_quality(x + s * y, y)
    assert np.max(np.abs(q - (2.0 + s * s) / 2.0)) < 1e-13
    a, b = 2.0, 0.5
    q = mp.cell_quality(a * x, b * y)
    assert np.max(np.abs(q - (a * a + b * b) / (2 * a * b))) < 1e-13
    # rotation leaves Q unchanged
    c, sn = math.cos(0.4), math.sin(0.4)
    q = mp.cell_quality(c * x - sn * y, sn * x + c * y)
    assert np.max(np.abs(q - 1.0)) < 1e-13
    # bilinear map x = xi + c xi eta: on every cell the averaged edge
    # differences are the exact derivatives at the cell centre
    c = 0.8
    q = mp.cell_quality(x + c * x * y, y)
    xc = (np.arange(n - 1) + 0.5) / (n - 1)
    XC, EC = np.meshgrid(xc, xc)
    a11, a12 = 1.0 + c * EC, c * XC
    want = 0.5 * (a11 ** 2 + a12 ** 2 + 1.0) / np.abs(a11)
    assert np.max(np.abs(q - want)) < 1e-13
    r, rmax, rmean = mp.quality_ratio(a * x, b * y, a * x, b * y)
    assert rmax == 1.0 and rmean == 1.0


# ---------------------------------------------------------------------------
# the five-ring test of section 4.2, as the paper runs it (one substep)
# ---------------------------------------------------------------------------
@pytest.mark.slow
def test_five_ring_one_substep_matches_single_domain():
    """Section 4.2 reports single-domain and decomposed meshes of equal
    quality on the five-ring monitor with one path substep per mesh step.
    Read with the computational square the same [-1, 1[^2 as the physical
    domain (a step of 5e-4 there is 1.25e-4 in unit-square time), the
    decomposed 2x2 mesh after all 100 steps has R = Q_SD / Q_SDD within a
    few percent of 1 in every cell; read in unit-square time the single
    Euler-Maruyama substep crosses the steep rings in one jump and the
    decomposed mesh folds."""
    def run(comp_side):
        L = W.five_ring_loop(2, n_paths=2000, comp_side=comp_side)
        out = []
        for decomposed in (False, True):
            x, y, _ = mp.mp_loop(L.u, L.x0, L.y0, L.steps, L.tau, L.K, L.n_paths, L.sub_xi, L.sub_eta,
                                 L.periodic_xi, L.periodic_eta, L.Lx, L.Ly, L.alpha, L.normalize,
                                 decomposed=decomposed, threads=8)
            out.append((x, y))
        return out

    (xs, ys), (xd, yd) = run(2.0)
    r, rmax, rmean = mp.quality_ratio(xs, ys, xd, yd)
    assert float(r.min()) > 0.9 and rmax < 1.1 and abs(rmean - 1.0) < 0.005, (float(r.min()), rmax, rmean)
    (xs, ys), (xd, yd) = run(1.0)
    dx_xi, dy_xi = np.diff(xd, axis=1)[:-1], np.diff(yd, axis=1)[:-1]
    dx_eta, dy_eta = np.diff(xd, axis=0)[:, :-1], np.diff(yd, axis=0)[:, :-1]
    assert float(np.min(dx_xi * dy_eta - dx_eta * dy_xi)) < 0.0   # a folded cell: negative orientation
