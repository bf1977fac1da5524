"""Deterministic single-domain finite-difference solve of the mesh generator.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  It gives an
independent, non-random reference for the Monte-Carlo estimate when the
monitor is not constant: the paper's subdomain solver discretisation
(section 3.5: centred differences in space, forward Euler in time) applied
on one domain, on a grid refined r times, to

    x_t = b . grad x + lap x,   b = (rho_xi / rho, rho_eta / rho)

(eq. Gen with rho frozen, section 3.2), where b is the SAME coefficient field
the estimator samples: the finite-difference table of the oracle,
interpolated bilinearly (three fields, then divided).  Dirichlet sides take
the boundary arrays, linear in time between t^n and t^{n+1}; periodic axes
wrap (with the quasi-periodic offset for the coordinate that winds).

The initial mesh is evaluated on the refined grid with the oracle's Keys
bicubic (exact for the uniform meshes used in the tests).
"""
from __future__ import annotations

import numpy as np

from . import keys_bicubic, monitor_gradient


def _bilinear_grid(f, per_xi, per_eta, XI, ETA):
    """Bilinear interpolation of a node table at points (vectorised)."""
    n_eta, n_xi = f.shape
    sx = XI * (n_xi - 1)
    sy = ETA * (n_eta - 1)
    cx = np.floor(sx).astype(np.int64)
    cy = np.floor(sy).astype(np.int64)
    if not per_xi:
        cx = np.clip(cx, 0, n_xi - 2)
    if not per_eta:
        cy = np.clip(cy, 0, n_eta - 2)
    tx = sx - cx
    ty = sy - cy
    mx, my = n_xi - 1, n_eta - 1

    def node(i, j):
        if per_xi:
            i = np.mod(i, mx)
        if per_eta:
            j = np.mod(j, my)
        return f[j, i]

    return ((1 - tx) * (1 - ty) * node(cx, cy) + tx * (1 - ty) * node(cx + 1, cy)
            + (1 - tx) * ty * node(cx, cy + 1) + tx * ty * node(cx + 1, cy + 1))


def _boundary_side(bnd, n_xi, n_eta, side, comp):
    if side < 2:
        o = (side * 2 + comp) * n_eta
        return bnd[o:o + n_eta]
    o = 4 * n_eta + ((side - 2) * 2 + comp) * n_xi
    return bnd[o:o + n_xi]


def solve(rho, x0, y0, bnd_t0, bnd_t1, tau, periodic_xi=0, periodic_eta=0, Lx=1.0, Ly=1.0,
          refine=4, cfl=0.2):
    """Return (x, y) at t^{n+1} on the ORIGINAL grid nodes.

    refine: fine-grid factor r (fine spacing H = h / r); cfl: dt = cfl*H^2.
    """
    rho = np.asarray(rho, dtype=np.float64)
    n_eta, n_xi = rho.shape
    rx, ry = monitor_gradient(rho, periodic_xi, periodic_eta)
    m_xi = refine * (n_xi - 1) + 1
    m_eta = refine * (n_eta - 1) + 1
    Hx, Hy = 1.0 / (m_xi - 1), 1.0 / (m_eta - 1)
    XI, ETA = np.meshgrid(np.arange(m_xi) * Hx, np.arange(m_eta) * Hy)
    r = _bilinear_grid(rho, periodic_xi, periodic_eta, XI, ETA)
    bx = _bilinear_grid(rx, periodic_xi, periodic_eta, XI, ETA) / r
    by = _bilinear_grid(ry, periodic_xi, periodic_eta, XI, ETA) / r

    def initial(f, off_xi, off_eta):
        out = np.empty((m_eta, m_xi))
        for j in range(m_eta):
            for i in range(m_xi):
                out[j, i] = keys_bicubic(f, XI[j, i], ETA[j, i], periodic_xi, periodic_eta, off_xi, off_eta)
        return out

    fields = [initial(x0, Lx, 0.0), initial(y0, 0.0, Ly)]
    offs = [(Lx if periodic_xi else 0.0, 0.0), (0.0, Ly if periodic_eta else 0.0)]

    h = min(Hx, Hy)
    n_steps = int(np.ceil(tau / (cfl * h * h)))
    dt = tau / n_steps

    fine_xi = np.arange(m_xi) * Hx
    fine_eta = np.arange(m_eta) * Hy

    def side_values(bnd, side, comp):
        arr = _boundary_side(bnd, n_xi, n_eta, side, comp)
        coarse = np.arange(len(arr)) / (len(arr) - 1)
        return np.interp(fine_eta if side < 2 else fine_xi, coarse, arr)

    sides = {}
    for comp in range(2):
        for side in range(4):
            sides[(side, comp)] = (side_values(bnd_t0, side, comp), side_values(bnd_t1, side, comp))

    def apply_bc(f, comp, t_frac):
        # t_frac: elapsed fraction of the step from t^n
        for side in range(4):
            if side < 2 and periodic_xi:
                continue
            if side >= 2 and periodic_eta:
                continue
            v0, v1 = sides[(side, comp)]
            v = (1.0 - t_frac) * v0 + t_frac * v1
            if side == 0:
                f[:, 0] = v
            elif side == 1:
                f[:, -1] = v
            elif side == 2:
                f[0, :] = v
            else:
                f[-1, :] = v

    def shifted(f, comp, di, dj):
        """f at (i+di, j+dj) with periodic wrap (and quasi-periodic offsets)."""
        g = f
        if di != 0:
            if periodic_xi:
                core = f[:, :-1]
                g = np.roll(core, -di, axis=1)
                if di > 0:
                    g[:, -di:] += offs[comp][0]
                else:
                    g[:, :-di] -= offs[comp][0]
                g = np.concatenate([g, g[:, :1] + offs[comp][0]], axis=1)
            else:
                g = np.zeros_like(f)
                if di > 0:
                    g[:, :-di] = f[:, di:]
                else:
                    g[:, -di:] = f[:, :di]
        if dj != 0:
            base = g
            if periodic_eta:
                core = base[:-1, :]
                g2 = np.roll(core, -dj, axis=0)
                if dj > 0:
                    g2[-dj:, :] += offs[comp][1]
                else:
                    g2[:-dj, :] -= offs[comp][1]
                g = np.concatenate([g2, g2[:1, :] + offs[comp][1]], axis=0)
            else:
                g = np.zeros_like(base)
                if dj > 0:
                    g[:-dj, :] = base[dj:, :]
                else:
                    g[-dj:, :] = base[:dj, :]
        return g

    for comp in range(2):
        apply_bc(fields[comp], comp, 0.0)
    for step in range(n_steps):
        for comp in range(2):
            f = fields[comp]
            fe, fw = shifted(f, comp, 1, 0), shifted(f, comp, -1, 0)
            fn, fs = shifted(f, comp, 0, 1), shifted(f, comp, 0, -1)
            rhs = (bx * (fe - fw) / (2 * Hx) + by * (fn - fs) / (2 * Hy)
                   + (fe - 2 * f + fw) / (Hx * Hx) + (fn - 2 * f + fs) / (Hy * Hy))
            f = f + dt * rhs
            if periodic_xi:
                f[:, -1] = f[:, 0] + offs[comp][0]
            if periodic_eta:
                f[-1, :] = f[0, :] + offs[comp][1]
            apply_bc(f, comp, (step + 1) / n_steps)
            fields[comp] = f
    x1 = fields[0][::refine, ::refine]
    y1 = fields[1][::refine, ::refine]
    return x1, y1
