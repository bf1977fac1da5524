"""Plain FP64 reference of the mesh step around the interface estimate.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): only the tests, the
smoke check and the CPU baseline leg of the benchmark may import it.  It is
written from the paper, in numpy, node by node where that is the clearest
form, and shares no code with the GPU library.

Paper: Bihlo, Haynes & Walsh, arXiv:1504.00084.
- section 2, eq. (Gen): the parabolic generator x_t = (grad rho / rho) . grad x
  + lap x (same for y) on the unit computational square; x = 0 / Lx on the
  sides xi = 0 / 1 and y = 0 / Ly on eta = 0 / 1; the tangential component
  along each physical side follows the one-dimensional form of (Gen).
- section 3.5 (local subdomain problem): once the interface values are
  known, every subdomain is a Dirichlet problem of (Gen), discretised by
  centred differences in space and forward Euler in time.
- section 3.6: the new mesh is assembled from the subdomain solves, then the
  monitor is evaluated on it.
- section 3.7, eq. (Q): geometric quality Q(K) = tr(J^T J) / (2 sqrt(det J^T J))
  per cell, and the ratio R = Q_SD / Q_SDD against a single-domain mesh.

Readings where the paper is silent (each also listed in the design notes):
- forward-Euler step count L = ceil(tau / (cfl * dt_max)) with the
  stability limit dt_max = 1 / (2/h_xi^2 + 2/h_eta^2) (1-D: h^2 / 2);
- Dirichlet data of a subdomain (interface and physical-boundary nodes) move
  linearly in time from the mesh at t^n to the values at t^{n+1};
- drift coefficients at the nodes: the finite-difference monitor table
  (central inside, second-order one-sided at Dirichlet edges, wrapped on
  periodic axes) divided by rho at the node;
- arc-length monitor rho = sqrt(1 + alpha |grad u|^2) from nodal u, with the
  physical gradient from centred computational differences through the
  inverse mesh Jacobian (one-sided second order at Dirichlet edges; wrapped,
  with the period added to the winding coordinate, on periodic axes);
- the Jacobian of a cell for Q: average of the two edge differences along
  each computational direction, divided by the computational spacing.

Every function is pinned by ``tests/test_oracle_mp.py`` (exact discrete mode
decay, steady equidistribution, exactness on linear and quadratic data,
closed-form Q of sheared and stretched meshes).
"""
from __future__ import annotations

import math

import numpy as np

from . import Problem, interface_nodes, monitor_gradient


# ---------------------------------------------------------------------------
# forward-Euler step count
# ---------------------------------------------------------------------------
def fe_substeps_2d(tau: float, n_xi: int, n_eta: int, cfl: float = 0.9) -> int:
    h_xi, h_eta = 1.0 / (n_xi - 1), 1.0 / (n_eta - 1)
    dt_max = 1.0 / (2.0 / h_xi ** 2 + 2.0 / h_eta ** 2)
    return max(1, int(math.ceil(tau / (cfl * dt_max) - 1e-12)))


def fe_substeps_1d(tau: float, n: int, cfl: float = 0.9) -> int:
    h = 1.0 / (n - 1)
    return max(1, int(math.ceil(tau / (cfl * 0.5 * h * h) - 1e-12)))


# ---------------------------------------------------------------------------
# one-dimensional generator along a physical side (section 2)
# ---------------------------------------------------------------------------
def generator_1d(v, b, tau: float, periodic: int, period: float, substeps: int):
    """Forward Euler on v_t = b v_s + v_ss over [0, tau] with `substeps` steps.

    Dirichlet: the end values stay fixed.  Periodic: nodes 0..n-2 are the
    distinct ones, node n-1 is node 0 shifted by `period` (and node -1 is node
    n-2 shifted by -period).
    """
    v = np.array(v, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = len(v)
    h = 1.0 / (n - 1)
    dt = tau / substeps
    for _ in range(substeps):
        new = v.copy()
        if periodic:
            for i in range(n - 1):
                left = v[i - 1] if i > 0 else v[n - 2] - period
                right = v[i + 1]            # i + 1 <= n - 1, node n-1 is the image
                new[i] = v[i] + dt * (b[i] * (right - left) / (2 * h) + (right - 2 * v[i] + left) / (h * h))
            new[n - 1] = new[0] + period
        else:
            for i in range(1, n - 1):
                new[i] = v[i] + dt * (b[i] * (v[i + 1] - v[i - 1]) / (2 * h)
                                      + (v[i + 1] - 2 * v[i] + v[i - 1]) / (h * h))
        v = new
    return v


def _side_slice(n_xi: int, n_eta: int, side: int, comp: int):
    """Offsets of one component of one side in the boundary-array layout:
    sides 0 (xi = 0) and 1 (xi = 1) hold n_eta values per component, sides 2
    (eta = 0) and 3 (eta = 1) n_xi values, as (side, comp) blocks in order."""
    if side < 2:
        o = (side * 2 + comp) * n_eta
        return slice(o, o + n_eta)
    o = 4 * n_eta + ((side - 2) * 2 + comp) * n_xi
    return slice(o, o + n_xi)


def edge_generate(rho, bnd_t0, tau: float, periodic_xi: int = 0, periodic_eta: int = 0,
                  Lx: float = 1.0, Ly: float = 1.0, cfl: float = 0.9, substeps: int = 0):
    """Boundary arrays at t^{n+1}: the tangential component of each physical
    side advanced by the 1-D generator with the monitor frozen at t^n; the
    normal component is unchanged.  Sides of periodic axes are copied."""
    rho = np.asarray(rho, dtype=np.float64)
    n_eta, n_xi = rho.shape
    rx, ry = monitor_gradient(rho, periodic_xi, periodic_eta)
    out = np.array(bnd_t0, dtype=np.float64)
    if not periodic_xi:            # sides xi = 0, 1: y runs along eta
        L = substeps or fe_substeps_1d(tau, n_eta, cfl)
        for side, i in ((0, 0), (1, n_xi - 1)):
            s = _side_slice(n_xi, n_eta, side, 1)
            out[s] = generator_1d(out[s], ry[:, i] / rho[:, i], tau, periodic_eta, Ly, L)
    if not periodic_eta:           # sides eta = 0, 1: x runs along xi
        L = substeps or fe_substeps_1d(tau, n_xi, cfl)
        for side, j in ((2, 0), (3, n_eta - 1)):
            s = _side_slice(n_xi, n_eta, side, 0)
            out[s] = generator_1d(out[s], rx[j, :] / rho[j, :], tau, periodic_xi, Lx, L)
    return out


# ---------------------------------------------------------------------------
# subdomain solves (section 3.5) and the single-domain reference
# ---------------------------------------------------------------------------
def dirichlet_targets(n_xi: int, n_eta: int, sub_xi: int, sub_eta: int, periodic_xi: int, periodic_eta: int,
                      Lx: float, Ly: float, bnd_t1, iface_x, iface_y, with_interfaces: bool = True):
    """Mask of the Dirichlet nodes of the decomposed problem and their
    values at t^{n+1}: physical-boundary nodes from the boundary arrays,
    interface nodes from the interface estimate, and on periodic axes the
    image row/column (node n-1) as node 0 shifted by the period."""
    mask = np.zeros((n_eta, n_xi), dtype=bool)
    X1 = np.zeros((n_eta, n_xi))
    Y1 = np.zeros((n_eta, n_xi))
    bnd_t1 = np.asarray(bnd_t1, dtype=np.float64)
    if with_interfaces:
        prob = Problem(n_xi=n_xi, n_eta=n_eta, sub_xi=sub_xi, sub_eta=sub_eta, periodic_xi=periodic_xi,
                       periodic_eta=periodic_eta, Lx=Lx, Ly=Ly)
        I, J = interface_nodes(prob)
        for r, (i, j) in enumerate(zip(I, J)):
            mask[j, i] = True
            X1[j, i] = iface_x[r]
            Y1[j, i] = iface_y[r]
    if not periodic_xi:
        for side, i in ((0, 0), (1, n_xi - 1)):
            mask[:, i] = True
            X1[:, i] = bnd_t1[_side_slice(n_xi, n_eta, side, 0)]
            Y1[:, i] = bnd_t1[_side_slice(n_xi, n_eta, side, 1)]
    if not periodic_eta:
        for side, j in ((2, 0), (3, n_eta - 1)):
            mask[j, :] = True
            X1[j, :] = bnd_t1[_side_slice(n_xi, n_eta, side, 0)]
            Y1[j, :] = bnd_t1[_side_slice(n_xi, n_eta, side, 1)]
    return mask, X1, Y1


def fe_solve(rho, x0, y0, mask, X1, Y1, tau: float, periodic_xi: int, periodic_eta: int,
             Lx: float, Ly: float, substeps: int):
    """Forward Euler with centred differences for (Gen) on the whole grid:
    nodes in `mask` follow their Dirichlet data linearly in time from the
    mesh at t^n to (X1, Y1); every other node is updated by the stencil.
    On a periodic axis the image node n-1 is node 0 plus the period; when it
    is not Dirichlet (single-domain reference) the stencil wraps."""
    rho = np.asarray(rho, dtype=np.float64)
    n_eta, n_xi = rho.shape
    rx, ry = monitor_gradient(rho, periodic_xi, periodic_eta)
    bx, by = rx / rho, ry / rho
    hx, hy = 1.0 / (n_xi - 1), 1.0 / (n_eta - 1)
    dt = tau / substeps
    x = np.array(x0, dtype=np.float64)
    y = np.array(y0, dtype=np.float64)
    X0, Y0 = x.copy(), y.copy()

    def nb(f, j, i, L_xi, L_eta):
        """Value at (j, i), indices possibly one outside on a periodic axis."""
        off = 0.0
        if periodic_xi:
            if i < 0:
                i += n_xi - 1
                off -= L_xi
            elif i > n_xi - 1:
                i -= n_xi - 1
                off += L_xi
        if periodic_eta:
            if j < 0:
                j += n_eta - 1
                off -= L_eta
            elif j > n_eta - 1:
                j -= n_eta - 1
                off += L_eta
        return f[j, i] + off

    for l in range(substeps):
        th1 = (l + 1) / substeps
        nx, ny = x.copy(), y.copy()
        for j in range(n_eta):
            for i in range(n_xi):
                if mask[j, i]:
                    nx[j, i] = (1.0 - th1) * X0[j, i] + th1 * X1[j, i]
                    ny[j, i] = (1.0 - th1) * Y0[j, i] + th1 * Y1[j, i]
                    continue
                if (periodic_xi and i == n_xi - 1) or (periodic_eta and j == n_eta - 1):
                    continue            # image node: set from node 0 below
                for f, out, Lxi, Leta in ((x, nx, Lx, 0.0), (y, ny, 0.0, Ly)):
                    c = f[j, i]
                    e, w = nb(f, j, i + 1, Lxi, Leta), nb(f, j, i - 1, Lxi, Leta)
                    n_, s_ = nb(f, j + 1, i, Lxi, Leta), nb(f, j - 1, i, Lxi, Leta)
                    out[j, i] = c + dt * (bx[j, i] * (e - w) / (2 * hx) + by[j, i] * (n_ - s_) / (2 * hy)
                                          + (e - 2 * c + w) / (hx * hx) + (n_ - 2 * c + s_) / (hy * hy))
        # images of non-Dirichlet nodes on periodic axes
        if periodic_xi:
            for j in range(n_eta):
                if not mask[j, n_xi - 1]:
                    nx[j, n_xi - 1] = nx[j, 0] + Lx
                    ny[j, n_xi - 1] = ny[j, 0]
        if periodic_eta:
            for i in range(n_xi):
                if not mask[n_eta - 1, i]:
                    nx[n_eta - 1, i] = nx[0, i]
                    ny[n_eta - 1, i] = ny[0, i] + Ly
        x, y = nx, ny
    return x, y


def subdomain_solve(rho, x0, y0, bnd_t1, iface_x, iface_y, tau: float, sub_xi: int, sub_eta: int,
                    periodic_xi: int = 0, periodic_eta: int = 0, Lx: float = 1.0, Ly: float = 1.0,
                    cfl: float = 0.9, substeps: int = 0):
    """New mesh from the decomposed problem (section 3.5)."""
    n_eta, n_xi = np.shape(rho)
    mask, X1, Y1 = dirichlet_targets(n_xi, n_eta, sub_xi, sub_eta, periodic_xi, periodic_eta, Lx, Ly,
                                     bnd_t1, iface_x, iface_y, True)
    # image nodes of Dirichlet nodes on periodic axes follow their originals
    if periodic_xi:
        mask[:, n_xi - 1] = mask[:, 0]
        X1[:, n_xi - 1] = X1[:, 0] + Lx
        Y1[:, n_xi - 1] = Y1[:, 0]
    if periodic_eta:
        mask[n_eta - 1, :] = mask[0, :]
        X1[n_eta - 1, :] = X1[0, :]
        Y1[n_eta - 1, :] = Y1[0, :] + Ly
    L = substeps or fe_substeps_2d(tau, n_xi, n_eta, cfl)
    return fe_solve(rho, x0, y0, mask, X1, Y1, tau, periodic_xi, periodic_eta, Lx, Ly, L)


def single_domain_solve(rho, x0, y0, bnd_t1, tau: float, periodic_xi: int = 0, periodic_eta: int = 0,
                        Lx: float = 1.0, Ly: float = 1.0, cfl: float = 0.9, substeps: int = 0):
    """Reference mesh of the undecomposed problem (section 3.7): Dirichlet
    data on the physical boundary only, periodic axes wrap."""
    n_eta, n_xi = np.shape(rho)
    mask, X1, Y1 = dirichlet_targets(n_xi, n_eta, 1, 1, periodic_xi, periodic_eta, Lx, Ly, bnd_t1,
                                     None, None, False)
    L = substeps or fe_substeps_2d(tau, n_xi, n_eta, cfl)
    return fe_solve(rho, x0, y0, mask, X1, Y1, tau, periodic_xi, periodic_eta, Lx, Ly, L)


# ---------------------------------------------------------------------------
# monitor from nodal u on the new mesh (section 3.6)
# ---------------------------------------------------------------------------
def _d_xi(f, periodic: int, period: float):
    """Centred difference along xi (axis 1) in units of the node index;
    one-sided second order at Dirichlet ends; wrapped (plus the period of a
    winding coordinate) on a periodic axis."""
    n = f.shape[1]
    d = np.empty_like(f)
    for i in range(n):
        if periodic:
            if i == 0 or i == n - 1:
                left = f[:, n - 2] - period
                right = f[:, 1]
            else:
                left, right = f[:, i - 1], f[:, i + 1]
            d[:, i] = 0.5 * (right - left)
        elif i == 0:
            d[:, i] = 0.5 * (-3 * f[:, 0] + 4 * f[:, 1] - f[:, 2])
        elif i == n - 1:
            d[:, i] = 0.5 * (3 * f[:, n - 1] - 4 * f[:, n - 2] + f[:, n - 3])
        else:
            d[:, i] = 0.5 * (f[:, i + 1] - f[:, i - 1])
    return d


def arclength_monitor(u, x, y, alpha: float, normalize: bool = False, periodic_xi: int = 0,
                      periodic_eta: int = 0, Lx: float = 1.0, Ly: float = 1.0):
    """rho = sqrt(1 + a |grad u|^2) at the nodes; a = alpha, or
    alpha / max |grad u|^2 when `normalize` (the Burgers setting)."""
    u = np.asarray(u, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n_eta, n_xi = u.shape
    hx, hy = 1.0 / (n_xi - 1), 1.0 / (n_eta - 1)
    u_xi = _d_xi(u, periodic_xi, 0.0) / hx
    x_xi = _d_xi(x, periodic_xi, Lx) / hx
    y_xi = _d_xi(y, periodic_xi, 0.0) / hx
    u_eta = _d_xi(u.T, periodic_eta, 0.0).T / hy
    x_eta = _d_xi(x.T, periodic_eta, 0.0).T / hy
    y_eta = _d_xi(y.T, periodic_eta, Ly).T / hy
    jac = x_xi * y_eta - x_eta * y_xi
    ux = (u_xi * y_eta - u_eta * y_xi) / jac
    uy = (u_eta * x_xi - u_xi * x_eta) / jac
    g = ux * ux + uy * uy
    a = alpha
    if normalize:
        gmax = float(np.max(g))
        a = alpha / gmax if gmax > 0.0 else 0.0
    return np.sqrt(1.0 + a * g)


# ---------------------------------------------------------------------------
# mesh quality (section 3.7)
# ---------------------------------------------------------------------------
def cell_quality(x, y):
    """Q(K) per cell [n_eta-1, n_xi-1]; the cell Jacobian averages the two
    edge differences along each computational direction."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n_eta, n_xi = x.shape
    hx, hy = 1.0 / (n_xi - 1), 1.0 / (n_eta - 1)
    q = np.empty((n_eta - 1, n_xi - 1))
    for j in range(n_eta - 1):
        for i in range(n_xi - 1):
            x_xi = 0.5 * ((x[j, i + 1] - x[j, i]) + (x[j + 1, i + 1] - x[j + 1, i])) / hx
            y_xi = 0.5 * ((y[j, i + 1] - y[j, i]) + (y[j + 1, i + 1] - y[j + 1, i])) / hx
            x_eta = 0.5 * ((x[j + 1, i] - x[j, i]) + (x[j + 1, i + 1] - x[j, i + 1])) / hy
            y_eta = 0.5 * ((y[j + 1, i] - y[j, i]) + (y[j + 1, i + 1] - y[j, i + 1])) / hy
            tr = x_xi ** 2 + y_xi ** 2 + x_eta ** 2 + y_eta ** 2
            det = abs(x_xi * y_eta - x_eta * y_xi)
            q[j, i] = 0.5 * tr / det
    return q


def quality_ratio(x_sd, y_sd, x_dd, y_dd):
    """R(K) = Q_SD / Q_SDD per cell, with its maximum and mean."""
    r = cell_quality(x_sd, y_sd) / cell_quality(x_dd, y_dd)
    return r, float(np.max(r)), float(np.mean(r))


# ---------------------------------------------------------------------------
# the moving-mesh loop (section 3.2 MP procedure, sections 3.4-3.6)
# ---------------------------------------------------------------------------
def boundary_arrays(x, y):
    """Boundary arrays of a mesh in the layout of ``_side_slice``."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return np.concatenate([x[:, 0], y[:, 0], x[:, -1], y[:, -1], x[0, :], y[0, :], x[-1, :], y[-1, :]])


def mp_loop(u_of, x0, y0, steps: int, tau: float, K: int, n_paths: int, sub_xi: int, sub_eta: int,
            periodic_xi: int = 0, periodic_eta: int = 0, Lx: float = 1.0, Ly: float = 1.0, alpha: float = 1.0,
            normalize: bool = False, decomposed: bool = True, seed: int = 0, instance_id: int = 0,
            threads: int | None = None):
    """Mesh after `steps` MP steps.  Each step n: u = u_of(x, y, n tau) at the
    nodes, the arc-length monitor on the current mesh, the boundary arrays at
    t^{n+1} from the edge generator, then either the interface estimate
    (Monte Carlo, mesh_step = n) and the subdomain solves, or the
    single-domain solve."""
    from . import solve as mc_solve
    x = np.array(x0, dtype=np.float64)
    y = np.array(y0, dtype=np.float64)
    n_eta, n_xi = x.shape
    b = boundary_arrays(x, y)
    for n in range(steps):
        u = u_of(x, y, n * tau)
        rho = arclength_monitor(u, x, y, alpha, normalize, periodic_xi, periodic_eta, Lx, Ly)
        b1 = edge_generate(rho, b, tau, periodic_xi, periodic_eta, Lx, Ly)
        if decomposed:
            prob = Problem(n_xi=n_xi, n_eta=n_eta, sub_xi=sub_xi, sub_eta=sub_eta, periodic_xi=periodic_xi,
                           periodic_eta=periodic_eta, Lx=Lx, Ly=Ly, tau=tau, K=K, seed=seed,
                           instance_id=instance_id, mesh_step=n)
            est = mc_solve(prob, rho, x, y, b, b1, n_paths, threads=threads)
            x, y = subdomain_solve(rho, x, y, b1, est["mean_x"], est["mean_y"], tau, sub_xi, sub_eta,
                                   periodic_xi, periodic_eta, Lx, Ly)
        else:
            x, y = single_domain_solve(rho, x, y, b1, tau, periodic_xi, periodic_eta, Lx, Ly)
        b = b1
    return x, y, b
