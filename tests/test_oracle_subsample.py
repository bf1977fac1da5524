"""Pins of the interface-subsampling oracle: which nodes are estimated,
exactness of the Keys interpolation along interface lines (quadratics with
Keys' end rule at Dirichlet sides, linear data wrapped across a periodic
seam), and the propagated standard error against an empirical spread."""
import numpy as np
import pytest

import oracle
from oracle import subsample as ss


def layout(prob):
    I, J = oracle.interface_nodes(prob)
    return I, J, I / (prob.n_xi - 1), J / (prob.n_eta - 1)


def bnd_of(prob, fx, fy):
    """Boundary arrays (C-ABI layout) of the functions fx, fy of (xi, eta)."""
    nx, ny = prob.n_xi, prob.n_eta
    xi, eta = np.arange(nx) / (nx - 1), np.arange(ny) / (ny - 1)
    parts = [fx(0 * eta, eta), fy(0 * eta, eta), fx(0 * eta + 1, eta), fy(0 * eta + 1, eta),
             fx(xi, 0 * xi), fy(xi, 0 * xi), fx(xi, 0 * xi + 1), fy(xi, 0 * xi + 1)]
    return np.concatenate(parts)


def test_sampled_set():
    p = oracle.Problem(33, 33, 2, 2)
    I, J, _, _ = layout(p)
    assert ss.sampled(p, 1).all()
    m = ss.sampled(p, 4)
    # crossings always; elsewhere every 4th node along the line
    assert m[(I == 16) & (J == 16)].all()
    assert m[(I == 16) & (J % 4 == 0)].all() and not m[(I == 16) & (J % 4 != 0)].any()
    assert m.sum() == 2 * 7 - 1                    # 7 per line, one shared crossing


def test_stride_validation():
    ss.check_stride(oracle.Problem(17, 17, 2, 2), 8)          # two segments per line: allowed
    with pytest.raises(ValueError):
        ss.sampled(oracle.Problem(33, 33, 2, 2), 3)            # does not divide 16
    with pytest.raises(ValueError):
        ss.sampled(oracle.Problem(33, 25, 2, 3), 16)           # does not divide 8
    with pytest.raises(ValueError):
        ss.check_stride(oracle.Problem(17, 17, 1, 1, 1, 1), 16)  # one segment per line
    with pytest.raises(ValueError):
        ss.check_stride(oracle.Problem(17, 17, 2, 2), 0)


@pytest.mark.parametrize("n,sub,stride", [(33, (2, 4), 2), (33, (2, 4), 4), (33, (2, 4), 8), (17, (2, 2), 8)])
def test_quadratics_are_exact_along_dirichlet_lines(n, sub, stride):
    p = oracle.Problem(n, n, sub[0], sub[1])
    I, J, xi, eta = layout(p)
    fx = lambda a, b: 0.3 + a + 0.7 * a * a - 0.4 * b * b + 0.2 * a * b
    fy = lambda a, b: b - 0.5 * b * b + 0.3 * a * a + 0.1 * a * b
    mx, my = fx(xi, eta), fy(xi, eta)
    m = ss.sampled(p, stride)
    garbage = np.where(m, 1.0, np.nan)
    gx, gy, sx, sy, ef = ss.interpolate(p, mx * garbage, my * garbage, np.zeros(len(I)), np.zeros(len(I)),
                                        np.zeros(len(I)), bnd_of(p, fx, fy), stride)
    assert np.max(np.abs(gx - mx)) < 1e-13 and np.max(np.abs(gy - my)) < 1e-13
    assert np.isnan(ef[~m]).all() and (ef[m] == 0).all()
    assert (sx == 0).all()


def test_linear_data_wrap_across_a_periodic_seam():
    Lx, Ly = 2.0, 3.0
    p = oracle.Problem(33, 25, 4, 2, 1, 1, Lx, Ly)
    I, J, xi, eta = layout(p)
    # x winds along xi and is periodic in eta, y the other way round
    fx = lambda a, b: -1.0 + Lx * a + 0.0 * b
    fy = lambda a, b: 0.5 + Ly * b + 0.0 * a
    mx, my = fx(xi, eta), fy(xi, eta)
    m = ss.sampled(p, 4)
    gx, gy, _, _, _ = ss.interpolate(p, np.where(m, mx, 9.0), np.where(m, my, 9.0), np.zeros(len(I)),
                                     np.zeros(len(I)), np.zeros(len(I)), np.zeros(4 * 25 + 4 * 33), 4)
    assert np.max(np.abs(gx - mx)) < 1e-13 and np.max(np.abs(gy - my)) < 1e-13


def test_propagated_se_matches_empirical_spread():
    p = oracle.Problem(33, 33, 2, 1, 0, 1, 1.0, 1.0)     # xi Dirichlet, eta periodic: vertical line wraps
    I, J, xi, eta = layout(p)
    m = ss.sampled(p, 4)
    rng = np.random.default_rng(5)
    se = np.where(m, rng.uniform(0.5, 2.0, len(I)), 0.0)
    base = xi.copy()
    bnd = bnd_of(p, lambda a, b: a, lambda a, b: b)
    _, _, sx, _, _ = ss.interpolate(p, base, base, se, se, np.zeros(len(I)), bnd, 4)
    reps = 400
    out = np.empty((reps, len(I)))
    for k in range(reps):
        noisy = base + se * rng.standard_normal(len(I))
        out[k], _, _, _, _ = ss.interpolate(p, noisy, noisy, se, se, np.zeros(len(I)), bnd, 4)
    emp = out.std(axis=0, ddof=1)
    interp = ~m
    rel = np.abs(emp[interp] / sx[interp] - 1.0)
    # std of a 400-sample standard deviation estimate is ~3.5 %; allow 5 sigma
    assert np.max(rel) < 0.18 and np.mean(rel) < 0.06
