"""Plain FP64 reference of the MᵏP and (MP)ˡ variants of the moving-mesh step.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).

Paper: Bihlo, Haynes & Walsh, arXiv:1504.00084, section 5 (conclusion):
- MᵏP: the mesh at t^{n+1} is reached through k sub-meshes, each obtained
  from the previous one by a step of tau / k of the linearised generator;
  the monitor of every sub-step is the piecewise-linear interpolant of the
  values (x^n, rho^n) at the nodes of the current sub-mesh;
- (MP)ˡ: the mesh and the physical solution are updated alternately l times
  per time step, reducing the lag between the two.

Readings (each also listed in the design notes):
- the piecewise-linear interpolant lives on the triangles of the old mesh,
  every cell (i, j)-(i+1, j+1) split along its diagonal from node (i, j) to
  node (i+1, j+1); a point takes the linear interpolant of the triangle
  containing it; a point outside the old mesh (a boundary node a rounding
  error outside) takes the linear extension of the triangle whose smallest
  barycentric coordinate is largest; periodic axes extend the old mesh by
  its images (x + Lx along xi, y + Ly along eta, the field unchanged);
- a sub-step of MᵏP runs K / k path substeps (the substep dt unchanged) and
  the random streams of mesh step n, sub-step s use the mesh-step counter
  n k + s;
- (MP)ˡ without a physical solver: pass 1 is the MP step from x^n with the
  monitor of u(., t^n) on x^n; pass m > 1 repeats the step from x^n with the
  monitor of u(., t^{n+1}) on the mesh of pass m - 1 (the physical solution
  "solved" on that mesh is the given u evaluated there); every pass uses the
  same random streams (mesh-step counter n), so the passes are iterates of
  one deterministic map;
- the two variants are separate (as in the paper): k > 1 with l > 1 is
  rejected.

Pinned by ``tests/test_oracle_variants.py``.
"""
from __future__ import annotations

import numpy as np

from . import Problem
from . import mp_oracle as mp


def _triangles(x, y, f, periodic_xi: int, periodic_eta: int, Lx: float, Ly: float):
    """Vertex coordinates [T, 3, 2] and values [T, 3] of the old mesh's
    triangles, with the periodic images."""
    x = np.array(x, dtype=np.float64)
    y = np.array(y, dtype=np.float64)
    f = np.array(f, dtype=np.float64)
    if periodic_xi:      # node n-1 is the image of node 0
        x[:, -1] = x[:, 0] + Lx
        y[:, -1] = y[:, 0]
        f[:, -1] = f[:, 0]
    if periodic_eta:
        x[-1, :] = x[0, :]
        y[-1, :] = y[0, :] + Ly
        f[-1, :] = f[0, :]
    A = (slice(0, -1), slice(0, -1))
    B = (slice(0, -1), slice(1, None))
    C = (slice(1, None), slice(1, None))
    D = (slice(1, None), slice(0, -1))
    pts, vals = [], []
    for sy in ((-1, 0, 1) if periodic_eta else (0,)):
        for sx in ((-1, 0, 1) if periodic_xi else (0,)):
            for tri in ((A, B, C), (A, C, D)):
                pts.append(np.stack([np.stack([x[v].ravel() + sx * Lx, y[v].ravel() + sy * Ly], axis=-1)
                                     for v in tri], axis=1))
                vals.append(np.stack([f[v].ravel() for v in tri], axis=1))
    return np.concatenate(pts), np.concatenate(vals)


def p1_transfer(x_old, y_old, f_old, x_new, y_new, periodic_xi: int = 0, periodic_eta: int = 0,
                Lx: float = 1.0, Ly: float = 1.0):
    """f at the nodes of (x_new, y_new): the piecewise-linear interpolant of
    the nodal values f_old on the old mesh's triangles (brute force over all
    triangles).  The image nodes of periodic axes copy node 0's value."""
    P, V = _triangles(x_old, y_old, f_old, periodic_xi, periodic_eta, Lx, Ly)
    a, b, c = P[:, 0], P[:, 1], P[:, 2]
    e1, e2 = b - a, c - a
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    xn = np.asarray(x_new, dtype=np.float64)
    yn = np.asarray(y_new, dtype=np.float64)
    out = np.empty(xn.size)
    px_all, py_all = xn.ravel(), yn.ravel()
    for s in range(0, xn.size, 32):
        px = px_all[s:s + 32, None]
        py = py_all[s:s + 32, None]
        dx, dy = px - a[None, :, 0], py - a[None, :, 1]
        lb = (dx * e2[None, :, 1] - dy * e2[None, :, 0]) / det[None, :]
        lc = (e1[None, :, 0] * dy - e1[None, :, 1] * dx) / det[None, :]
        la = 1.0 - lb - lc
        best = np.argmax(np.minimum(np.minimum(la, lb), lc), axis=1)
        r = np.arange(len(best))
        out[s:s + 32] = la[r, best] * V[best, 0] + lb[r, best] * V[best, 1] + lc[r, best] * V[best, 2]
    out = out.reshape(xn.shape)
    if periodic_xi:
        out[:, -1] = out[:, 0]
    if periodic_eta:
        out[-1, :] = out[0, :]
    return out


def variant_loop(steps: int, x0, y0, tau: float, K: int, n_paths: int, sub_xi: int, sub_eta: int,
                 periodic_xi: int = 0, periodic_eta: int = 0, Lx: float = 1.0, Ly: float = 1.0,
                 u_of=None, alpha: float = 1.0, normalize: bool = False, monitor_of=None,
                 k_sub: int = 1, l_iter: int = 1, decomposed: bool = True, seed: int = 0,
                 instance_id: int = 0, threads: int | None = None):
    """Mesh after `steps` time steps of MᵏP (k_sub sub-steps) inside (MP)ˡ
    (l_iter passes).  The monitor at a mesh and time is either the
    arc-length monitor of u_of(x, y, t) (with alpha, normalize) or, when
    monitor_of is given, monitor_of(x, y, t) at the nodes."""
    from . import solve as mc_solve
    if K % k_sub:
        raise ValueError("K must be a multiple of k_sub")
    if k_sub > 1 and l_iter > 1:
        raise ValueError("MᵏP and (MP)ˡ are separate variants: k_sub > 1 needs l_iter = 1")
    x = np.array(x0, dtype=np.float64)
    y = np.array(y0, dtype=np.float64)
    n_eta, n_xi = x.shape
    h = tau / k_sub

    def monitor(xm, ym, t):
        if monitor_of is not None:
            return np.asarray(monitor_of(xm, ym, t), dtype=np.float64)
        return mp.arclength_monitor(u_of(xm, ym, t), xm, ym, alpha, normalize, periodic_xi, periodic_eta, Lx, Ly)

    def one_step(rho_n, xs, ys, bs, n):
        """k_sub sub-steps from (xs, ys, bs) with monitors transferred from (xs, ys, rho_n)."""
        xa, ya, ba = xs, ys, bs
        for s in range(k_sub):
            rho = rho_n if s == 0 else p1_transfer(xs, ys, rho_n, xa, ya, periodic_xi, periodic_eta, Lx, Ly)
            b1 = mp.edge_generate(rho, ba, h, periodic_xi, periodic_eta, Lx, Ly)
            if decomposed:
                prob = Problem(n_xi=n_xi, n_eta=n_eta, sub_xi=sub_xi, sub_eta=sub_eta, periodic_xi=periodic_xi,
                               periodic_eta=periodic_eta, Lx=Lx, Ly=Ly, tau=h, K=K // k_sub, seed=seed,
                               instance_id=instance_id, mesh_step=n * k_sub + s)
                est = mc_solve(prob, rho, xa, ya, ba, b1, n_paths, threads=threads)
                xa, ya = mp.subdomain_solve(rho, xa, ya, b1, est["mean_x"], est["mean_y"], h, sub_xi, sub_eta,
                                            periodic_xi, periodic_eta, Lx, Ly)
            else:
                xa, ya = mp.single_domain_solve(rho, xa, ya, b1, h, periodic_xi, periodic_eta, Lx, Ly)
            ba = b1
        return xa, ya, ba

    b = mp.boundary_arrays(x, y)
    for n in range(steps):
        xn, yn, bn = one_step(monitor(x, y, n * tau), x, y, b, n)
        for _ in range(1, l_iter):
            xn, yn, bn = one_step(monitor(xn, yn, (n + 1) * tau), x, y, b, n)
        x, y, b = xn, yn, bn
    return x, y, b
