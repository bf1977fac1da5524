"""Pins of the MᵏP / (MP)ˡ oracle: the piecewise-linear transfer (identity,
exact on linear fields including points a rounding error outside the mesh,
whole-cell shifts across periodic seams, the cell diagonal, second-order
convergence) and the loops (k = l = 1 reduce to the MP loop; MᵏP with a
monitor that the transfer reproduces exactly equals k MP steps of tau / k;
the time level and start mesh of the (MP)ˡ passes; the passes contract for
a mild monitor)."""
import numpy as np
import pytest

from oracle import mp_oracle as mp
from oracle import mp_variants as mv
from paper_1504_00084_amd import workloads as W


def curved_mesh(n, amp=0.03, periodic_xi=0, periodic_eta=0):
    x, y = W.uniform_mesh(n, n)
    xi, eta = x.copy(), y.copy()
    # displacement vanishing on Dirichlet sides and periodic on periodic axes
    fx = np.sin(2 * np.pi * eta) if periodic_eta else np.sin(np.pi * eta)
    fy = np.sin(2 * np.pi * xi) if periodic_xi else np.sin(np.pi * xi)
    gx = np.sin(2 * np.pi * xi) if periodic_xi else np.sin(np.pi * xi)
    gy = np.sin(2 * np.pi * eta) if periodic_eta else np.sin(np.pi * eta)
    return x + amp * gx * fx, y + amp * gy * fy


@pytest.mark.parametrize("per", [(0, 0), (1, 0), (1, 1)])
def test_transfer_onto_the_same_mesh_is_the_identity(per):
    x, y = curved_mesh(13, periodic_xi=per[0], periodic_eta=per[1])
    f = np.random.default_rng(1).uniform(1.0, 2.0, x.shape)
    g = mv.p1_transfer(x, y, f, x, y, *per)
    inner = (slice(None, -1 if per[1] else None), slice(None, -1 if per[0] else None))
    assert np.array_equal(g[inner], f[inner])


def test_linear_fields_are_exact_including_points_just_outside():
    x, y = curved_mesh(15, amp=0.04)
    f = 0.7 + 1.3 * x - 0.4 * y
    rng = np.random.default_rng(2)
    h = 1.0 / 14
    xn = x + rng.uniform(-0.3 * h, 0.3 * h, x.shape)
    yn = y + rng.uniform(-0.3 * h, 0.3 * h, y.shape)
    # boundary nodes slide along their sides, a rounding error outside
    xn[:, 0], xn[:, -1] = -1e-15, 1.0 + 1e-15
    yn[0, :], yn[-1, :] = -1e-15, 1.0 + 1e-15
    g = mv.p1_transfer(x, y, f, xn, yn)
    assert np.max(np.abs(g - (0.7 + 1.3 * xn - 0.4 * yn))) < 1e-13


def test_linear_in_y_field_across_a_periodic_xi_seam():
    Lx = 2.0
    x, y = curved_mesh(17, periodic_xi=1)
    x = x * Lx
    f = 1.0 + 0.5 * y
    xn = x - 0.37 * Lx / 16          # every node moves left; column 0 crosses the seam
    g = mv.p1_transfer(x, y, f, xn, y, 1, 0, Lx, 1.0)
    assert np.max(np.abs(g - f)) < 1e-13


def test_whole_cell_shift_across_both_seams_is_a_permutation():
    n, Lx, Ly = 17, 2.0, 3.0
    x, y = W.uniform_mesh(n, n, Lx, Ly)
    f = np.random.default_rng(3).uniform(size=x.shape)
    f[:, -1], f[-1, :] = f[:, 0], f[0, :]
    xn, yn = x + Lx / (n - 1), y + 2 * Ly / (n - 1)
    g = mv.p1_transfer(x, y, f, xn, yn, 1, 1, Lx, Ly)
    m = n - 1
    want = f[np.ix_((np.arange(n) + 2) % m, (np.arange(n) + 1) % m)]
    assert np.max(np.abs(g[:-1, :-1] - want[:-1, :-1])) < 1e-13


def test_cell_centres_lie_on_the_i_j_to_i1_j1_diagonal():
    n = 9
    x, y = W.uniform_mesh(n, n)
    f = x * y
    c = (np.arange(n - 1) + 0.5) / (n - 1)
    xc, yc = np.meshgrid(c, c)
    g = mv.p1_transfer(x, y, f, xc, yc)
    h = 1.0 / (n - 1)
    along = ((xc - h / 2) * (yc - h / 2) + (xc + h / 2) * (yc + h / 2)) / 2
    across = ((xc + h / 2) * (yc - h / 2) + (xc - h / 2) * (yc + h / 2)) / 2
    assert np.max(np.abs(g - along)) < 1e-15 and np.min(np.abs(g - across)) > 1e-3


def test_second_order_convergence():
    rng = np.random.default_rng(4)
    px, py = rng.uniform(size=(2, 20, 20))
    fun = lambda a, b: np.sin(3 * a) * np.cos(2 * b)
    errs = []
    for n in (9, 17, 33):
        x, y = W.uniform_mesh(n, n)
        errs.append(np.max(np.abs(mv.p1_transfer(x, y, fun(x, y), px, py) - fun(px, py))))
    h = 1.0 / 8
    assert errs[0] < h * h * (9 + 6 + 4)
    assert 3.0 < errs[0] / errs[1] < 5.5 and 3.0 < errs[1] / errs[2] < 5.5


def bump(x, y, t):
    return np.exp(-((x - 0.5 - 0.2 * t) ** 2 + (y - 0.5) ** 2) / 0.02)


@pytest.mark.parametrize("decomposed", [False, True])
def test_k1_l1_reduce_to_the_mp_loop(decomposed):
    n, tau, K, N = 17, 0.01, 8, 64
    x, y = W.uniform_mesh(n, n)
    kw = dict(tau=tau, K=K, n_paths=N, sub_xi=2, sub_eta=2, alpha=5.0, decomposed=decomposed, threads=4)
    a = mv.variant_loop(2, x, y, u_of=bump, **kw)
    b = mp.mp_loop(bump, x, y, 2, tau, K, N, 2, 2, alpha=5.0, decomposed=decomposed, threads=4)
    for p, q in zip(a, b):
        assert np.array_equal(p, q)


@pytest.mark.parametrize("decomposed", [False, True])
def test_mkp_with_an_exactly_transferred_monitor_equals_k_mp_steps(decomposed):
    """rho linear in the physical position: the transferred monitor is the
    monitor evaluated on the sub-mesh, so two MᵏP sub-steps are two MP steps
    of tau / 2 with the monitor evaluated there (same streams: n k + s)."""
    n, tau, K, N = 17, 0.02, 8, 64
    x, y = curved_mesh(n, amp=0.02)
    rho = lambda xm, ym, t: 1.0 + 2.0 * xm + 0.5 * ym
    kw = dict(n_paths=N, sub_xi=2, sub_eta=2, monitor_of=rho, decomposed=decomposed, threads=4)
    a = mv.variant_loop(1, x, y, tau=tau, K=K, k_sub=2, **kw)
    b = mv.variant_loop(2, x, y, tau=tau / 2, K=K // 2, **kw)
    moved = np.max(np.abs(a[0] - x))
    assert moved > 1e-4
    for p, q in zip(a, b):
        assert np.max(np.abs(p - q)) < 1e-12


def test_mpl_second_pass_uses_t_n_plus_1_from_the_old_mesh():
    """rho constant at t^n (pass 1 leaves the uniform mesh unchanged) and
    1 + 0.5 x at t^{n+1}: pass 2 is one MP step from the old mesh with that
    monitor."""
    n, tau = 17, 0.02
    x, y = W.uniform_mesh(n, n)
    rho = lambda xm, ym, t: 1.0 + (t / tau) * 0.5 * xm
    kw = dict(tau=tau, K=4, n_paths=16, sub_xi=1, sub_eta=1, decomposed=False)
    one = mv.variant_loop(1, x, y, monitor_of=rho, l_iter=1, **kw)
    assert np.max(np.abs(one[0] - x)) < 1e-15
    two = mv.variant_loop(1, x, y, monitor_of=rho, l_iter=2, **kw)
    ref = mv.variant_loop(1, x, y, monitor_of=lambda xm, ym, t: 1.0 + 0.5 * xm, **kw)
    assert np.max(np.abs(two[0] - x)) > 1e-4
    for p, q in zip(two, ref):
        assert np.array_equal(p, q)


def test_mpl_passes_contract_for_a_mild_monitor():
    """With alpha = 0.5 the passes are iterates of a contraction (with
    alpha >= 2 on this bump they stall: the iteration need not converge)."""
    n, tau = 17, 0.02
    x, y = W.uniform_mesh(n, n)
    kw = dict(tau=tau, K=4, n_paths=16, sub_xi=1, sub_eta=1, u_of=bump, alpha=0.5, decomposed=False)
    meshes = [mv.variant_loop(1, x, y, l_iter=l, **kw)[0] for l in range(1, 6)]
    d = [np.max(np.abs(meshes[k + 1] - meshes[k])) for k in range(4)]
    assert d[0] > 1e-3
    assert all(d[k + 1] < 0.5 * d[k] for k in range(3))


def test_combined_variants_are_rejected():
    x, y = W.uniform_mesh(9, 9)
    with pytest.raises(ValueError):
        mv.variant_loop(1, x, y, 0.01, 4, 8, 1, 1, u_of=bump, k_sub=2, l_iter=2)
    with pytest.raises(ValueError):
        mv.variant_loop(1, x, y, 0.01, 5, 8, 1, 1, u_of=bump, k_sub=2)
