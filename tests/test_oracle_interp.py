"""Pins of the oracle's deterministic pieces: finite-difference gradient,
bilinear and Keys-bicubic interpolation (section 3.4 with readings R1-R3,
R6), bridge probability (reading R4) and the interface-node enumeration
(section 3.5, reading R7)."""
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def quad(xi, eta):
    return 0.3 + 1.7 * xi - 0.9 * eta + 2.1 * xi * xi - 1.3 * xi * eta + 0.8 * eta * eta


def quad_dxi(xi, eta):
    return 1.7 + 4.2 * xi - 1.3 * eta


def quad_deta(xi, eta):
    return -0.9 - 1.3 * xi + 1.6 * eta


def grid(n_xi, n_eta):
    xi = np.arange(n_xi) / (n_xi - 1)
    eta = np.arange(n_eta) / (n_eta - 1)
    return np.meshgrid(xi, eta)


@pytest.mark.parametrize("n_xi,n_eta", [(9, 9), (17, 5), (5, 33)])
def test_fd_exact_on_quadratics(oracle_lib, n_xi, n_eta):
    XI, ETA = grid(n_xi, n_eta)
    rx, ry = oracle_lib.monitor_gradient(quad(XI, ETA))
    assert np.max(np.abs(rx - quad_dxi(XI, ETA))) < 1e-11
    assert np.max(np.abs(ry - quad_deta(XI, ETA))) < 1e-11


def test_fd_periodic_closed_form(oracle_lib):
    # central difference of sin(2 pi xi) over the n-1 distinct nodes:
    # cos(2 pi xi) sin(2 pi h) / h, also across the seam.
    n = 17
    XI, ETA = grid(n, n)
    f = np.sin(2 * np.pi * XI) + quad(0 * XI, ETA)
    rx, ry = oracle_lib.monitor_gradient(f, periodic_xi=1)
    h = 1.0 / (n - 1)
    want = np.cos(2 * np.pi * XI) * np.sin(2 * np.pi * h) / h
    assert np.max(np.abs(rx - want)) < 1e-11
    assert np.max(np.abs(ry - quad_deta(0 * XI, ETA))) < 1e-11
    # doubly periodic: eta too
    g = np.sin(2 * np.pi * XI) * np.cos(2 * np.pi * ETA)
    rx, ry = oracle_lib.monitor_gradient(g, 1, 1)
    assert np.max(np.abs(ry + np.sin(2 * np.pi * XI) * np.sin(2 * np.pi * ETA) * np.sin(2 * np.pi * h) / h)) < 1e-11


def test_bilinear_exact_on_bilinear(oracle_lib):
    n_xi, n_eta = 9, 13
    XI, ETA = grid(n_xi, n_eta)
    fs = [lambda a, b, c=c: c[0] + c[1] * a + c[2] * b + c[3] * a * b
          for c in ([1.0, 2.0, 3.0, 4.0], [-2.0, 0.5, 0.0, 1.5], [0.1, 0.0, -3.0, 2.0])]
    tabs = [f(XI, ETA) for f in fs]
    rng = np.random.default_rng(3)
    pts = list(rng.random((200, 2))) + [(0.0, 0.0), (1.0, 1.0), (1.0, 0.0), (0.0, 1.0), (0.5, 1.0)]
    for (a, b) in pts:
        out = oracle_lib.bilinear(*tabs, a, b)
        for k in range(3):
            assert abs(out[k] - fs[k](a, b)) < 1e-12


def test_bilinear_periodic_seam(oracle_lib):
    # in the last periodic cell the far corner is node 0
    n = 9
    XI, ETA = grid(n, n)
    t = np.cos(2 * np.pi * XI) + ETA
    h = 1.0 / (n - 1)
    a, b = 1.0 - 0.25 * h, 0.3
    out = oracle_lib.bilinear(t, t, t, a, b, periodic_xi=1)
    want = 0.25 * math.cos(2 * math.pi * (1 - h)) + 0.75 * 1.0 + b
    assert abs(out[0] - want) < 1e-12


def test_keys_kernel_midpoint_weights(oracle_lib):
    # Keys (a = -1/2) halfway between nodes weights the 4 neighbours by
    # (-1/16, 9/16, 9/16, -1/16); test on a spike well inside the grid.
    n = 16
    for k, w in [(6, -1 / 16), (7, 9 / 16), (8, 9 / 16), (9, -1 / 16), (10, 0.0)]:
        f = np.zeros((n, n))
        f[:, k] = 1.0
        xi = (7.5) / (n - 1)
        assert abs(oracle_lib.keys_bicubic(f, xi, 0.4) - w) < 1e-14


def test_keys_exact_on_quadratics(oracle_lib):
    n_xi, n_eta = 11, 7
    XI, ETA = grid(n_xi, n_eta)
    F = quad(XI, ETA)
    rng = np.random.default_rng(5)
    pts = list(rng.random((300, 2))) + [(0.0, 0.0), (1.0, 1.0), (0.01, 0.99), (0.999, 0.002)]
    for (a, b) in pts:
        assert abs(oracle_lib.keys_bicubic(F, a, b) - quad(a, b)) < 1e-12


def test_keys_not_exact_on_cubics(oracle_lib):
    # the kernel is third-order, so a cubic is not reproduced (guards
    # against silently using another interpolant)
    n = 11
    XI, ETA = grid(n, n)
    F = XI ** 3
    a = 0.53   # off the midpoint, where the 4-point weights happen to be cubic-exact
    err = abs(oracle_lib.keys_bicubic(F, a, 0.5) - a ** 3)
    assert 1e-6 < err < 1e-2


def test_keys_periodic_offsets(oracle_lib):
    # x = Lx xi + 0.1 cos(2 pi eta) + 0.05 sin(2 pi xi): quasi-periodic in xi
    n = 33
    Lx = 2.5
    XI, ETA = grid(n, n)
    F = Lx * XI + 0.1 * ETA ** 2 + 0.05 * np.sin(2 * np.pi * XI)
    rng = np.random.default_rng(9)
    h = 1.0 / (n - 1)
    for (a, b) in rng.random((200, 2)):
        want = Lx * a + 0.1 * b * b + 0.05 * math.sin(2 * math.pi * a)
        got = oracle_lib.keys_bicubic(F, a, b, periodic_xi=1, off_xi=Lx)
        assert abs(got - want) < 0.05 * (2 * math.pi * h) ** 3  # O(h^3) sine error only
    # exact when the periodic part vanishes, including the seam cells
    G = Lx * XI + 0.1 * ETA ** 2
    for a in [0.0, 0.5 * h, 1.0 - 0.5 * h, 1.0 - 1e-9]:
        assert abs(oracle_lib.keys_bicubic(G, a, 0.3, periodic_xi=1, off_xi=Lx) - (Lx * a + 0.009)) < 1e-12


def test_bridge_probability_values(oracle_lib):
    assert oracle_lib.bridge_probability(0.0, 0.3, 1e-4) == 1.0
    assert abs(oracle_lib.bridge_probability(0.01, 0.01, 1e-4) - math.exp(-1.0)) < 1e-15


def test_bridge_probability_brute_force(oracle_lib):
    """Crossing frequency of a fine-step Brownian bridge of variance 2 dt
    (the SDE's diffusion sqrt(2) dW over one substep), extrapolated in the
    monitoring step, against exp(-d0 d1 / dt)."""
    rng = np.random.default_rng(11)
    dt = 1e-4
    for d0, d1 in [(0.01, 0.01), (0.005, 0.02), (0.02, 0.015)]:
        freqs = []
        for m in (400, 1600):
            n_br = 40_000
            hits = 0
            for chunk in range(4):
                nb = n_br // 4
                inc = rng.standard_normal((nb, m)) * math.sqrt(2 * dt / m)
                w = np.cumsum(inc, axis=1)
                s = np.arange(1, m + 1) / m
                bridge = d0 + w - s * (w[:, -1:] - (d1 - d0))   # pinned to d0 -> d1
                hits += int(np.sum(bridge.min(axis=1) <= 0.0))
            freqs.append(hits / n_br)
        # discrete monitoring misses crossings at rate ~ sqrt(step): Richardson in sqrt
        est = (2.0 * freqs[1] - freqs[0]) / (2.0 - 1.0)
        p = oracle_lib.bridge_probability(d0, d1, dt)
        assert abs(est - p) < 5.0 * math.sqrt(p * (1 - p) / 10_000) + 0.01, (d0, d1, est, p, freqs)
        # and the factor in the exponent is right: exp(-2 d0 d1/dt) is far off
        assert abs(est - math.exp(-2 * d0 * d1 / dt)) > 0.03


def _brute_interface(n_xi, n_eta, s_xi, s_eta, per_xi, per_eta):
    """Nodes on the boundary of some subdomain rectangle that are not on
    the physical boundary, found by walking the rectangles."""
    P_xi, P_eta = (n_xi - 1) // s_xi, (n_eta - 1) // s_eta
    nodes = set()
    for a in range(s_xi):
        for b in range(s_eta):
            i0, i1, j0, j1 = a * P_xi, (a + 1) * P_xi, b * P_eta, (b + 1) * P_eta
            for i in range(i0, i1 + 1):
                for j in range(j0, j1 + 1):
                    if i in (i0, i1) or j in (j0, j1):
                        ii = i % (n_xi - 1) if per_xi else i
                        jj = j % (n_eta - 1) if per_eta else j
                        nodes.add((ii, jj))
    keep = []
    for (i, j) in nodes:
        if not per_xi and i in (0, n_xi - 1):
            continue
        if not per_eta and j in (0, n_eta - 1):
            continue
        keep.append((j, i))
    keep.sort()
    return [(i, j) for (j, i) in keep]


def test_interface_counts_golden(oracle_lib):
    rows = [ln.split() for ln in open(os.path.join(HERE, "golden", "interface_counts.txt"))
            if ln.strip() and not ln.startswith("#")]
    for r in rows:
        n_xi, n_eta, s_xi, s_eta, px, pe, count = (int(v) for v in r[:7])
        P = oracle_lib.Problem(n_xi=n_xi, n_eta=n_eta, sub_xi=s_xi, sub_eta=s_eta, periodic_xi=px, periodic_eta=pe)
        i, j = oracle_lib.interface_nodes(P)
        assert len(i) == count, r
        if n_xi <= 257:
            brute = _brute_interface(n_xi, n_eta, s_xi, s_eta, px, pe)
            assert list(zip(i.tolist(), j.tolist())) == brute


@pytest.mark.parametrize("n_xi,n_eta,s_xi,s_eta,px,pe", [(17, 9, 4, 2, 0, 0), (17, 9, 4, 2, 1, 0), (9, 17, 2, 4, 0, 1),
                                                        (9, 9, 1, 1, 1, 1), (9, 9, 1, 1, 0, 0), (13, 13, 3, 4, 0, 0)])
def test_interface_brute_force(oracle_lib, n_xi, n_eta, s_xi, s_eta, px, pe):
    P = oracle_lib.Problem(n_xi=n_xi, n_eta=n_eta, sub_xi=s_xi, sub_eta=s_eta, periodic_xi=px, periodic_eta=pe)
    i, j = oracle_lib.interface_nodes(P)
    assert list(zip(i.tolist(), j.tolist())) == _brute_interface(n_xi, n_eta, s_xi, s_eta, px, pe)
