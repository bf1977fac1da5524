"""Seeded synthetic inputs for the interface solve.

This module builds inputs only: grids, meshes, boundary arrays and frozen
monitor tables rho on the grid.  It holds none of the estimator's arithmetic
(no random paths, no interpolation, no finite differences), so the GPU path
and the CPU oracle can both consume what it produces.

The monitor is the arc-length density rho = sqrt(1 + alpha |grad u|^2) of
section 1 / section 4 of the paper, evaluated with the analytic gradient of a
synthetic physical field u at the current mesh positions.  Two families of u
stand in for the paper's physical solutions (no dataset is involved):

* Gaussian bump ``u = exp(-|x - c|^2 / w)`` on a Dirichlet unit square;
* moving front ``u = tanh(d / w)`` with the nearest-image signed distance
  ``d = ((x - 0.3 sin(2 pi y) - 0.2 t) + L/2 mod L) - L/2``, periodic in x.

Boundary arrays use the layout of the C-ABI: side 0 (xi=0) and side 1
(xi=1) carry n_eta values per component, side 2 (eta=0) and side 3 (eta=1)
carry n_xi values, ordered [s0 x][s0 y][s1 x][s1 y][s2 x][s2 y][s3 x][s3 y].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np


@dataclass
class Instance:
    """One interface-solve problem with all of its inputs."""
    name: str
    n_xi: int
    n_eta: int
    sub_xi: int
    sub_eta: int
    periodic_xi: int
    periodic_eta: int
    Lx: float
    Ly: float
    tau: float
    K: int
    n_paths: int
    rho: np.ndarray          # [n_eta, n_xi] frozen monitor at t^n
    x: np.ndarray            # [n_eta, n_xi] mesh at t^n
    y: np.ndarray
    bnd_t0: np.ndarray       # boundary arrays at t^n
    bnd_t1: np.ndarray       # boundary arrays at t^{n+1}
    bridge: int = 1
    seed: int = 0
    instance_id: int = 0
    mesh_step: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def dt(self) -> float:
        return self.tau / self.K

    def with_paths(self, n_paths: int) -> "Instance":
        return replace(self, n_paths=int(n_paths))

    def problem_kwargs(self) -> dict:
        """Scalar fields shared by the C-ABI descriptor and the oracle."""
        return dict(n_xi=self.n_xi, n_eta=self.n_eta, sub_xi=self.sub_xi, sub_eta=self.sub_eta,
                    periodic_xi=self.periodic_xi, periodic_eta=self.periodic_eta, Lx=self.Lx,
                    Ly=self.Ly, tau=self.tau, K=self.K, bridge=self.bridge, seed=self.seed,
                    instance_id=self.instance_id, mesh_step=self.mesh_step)


# --------------------------------------------------------------------------
# meshes and boundary arrays
# --------------------------------------------------------------------------
def uniform_mesh(n_xi: int, n_eta: int, Lx: float = 1.0, Ly: float = 1.0):
    """x0 = Lx xi, y0 = Ly eta on the uniform computational grid (eq. Gen)."""
    xi = np.arange(n_xi, dtype=np.float64) / (n_xi - 1)
    eta = np.arange(n_eta, dtype=np.float64) / (n_eta - 1)
    x = np.broadcast_to(Lx * xi[None, :], (n_eta, n_xi)).copy()
    y = np.broadcast_to(Ly * eta[:, None], (n_eta, n_xi)).copy()
    return x, y


def boundary_from_mesh(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Pack the boundary rows/columns of a mesh into the C-ABI layout."""
    n_eta, n_xi = x.shape
    parts = [x[:, 0], y[:, 0], x[:, -1], y[:, -1], x[0, :], y[0, :], x[-1, :], y[-1, :]]
    return np.ascontiguousarray(np.concatenate(parts), dtype=np.float64)


def boundary_size(n_xi: int, n_eta: int) -> int:
    return 4 * n_eta + 4 * n_xi


def constant_boundary(n_xi: int, n_eta: int, value_x: float, value_y: float) -> np.ndarray:
    b = np.empty(boundary_size(n_xi, n_eta))
    o = 0
    for side in range(4):
        n = n_eta if side < 2 else n_xi
        b[o:o + n] = value_x
        b[o + n:o + 2 * n] = value_y
        o += 2 * n
    return b


# --------------------------------------------------------------------------
# monitors (arc-length density of a synthetic physical field)
# --------------------------------------------------------------------------
def arc_length_monitor(ux: np.ndarray, uy: np.ndarray, alpha: float) -> np.ndarray:
    return np.sqrt(1.0 + alpha * (ux * ux + uy * uy))


def gaussian_bump_grad(x, y, cx: float, cy: float, w: float):
    """Gradient of u = exp(-((x-cx)^2 + (y-cy)^2) / w)."""
    u = np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / w)
    return -2.0 * (x - cx) / w * u, -2.0 * (y - cy) / w * u


def tanh_front_grad(x, y, t: float, w: float, Lx: float = 1.0, phase: float = 0.0):
    """Gradient of u = tanh(d / w), d the nearest-image signed distance to
    the curve x = phase + 0.3 sin(2 pi y) + 0.2 t (period Lx in x)."""
    raw = x - phase - 0.3 * np.sin(2.0 * np.pi * y) - 0.2 * t
    d = np.mod(raw + 0.5 * Lx, Lx) - 0.5 * Lx
    sech2 = 1.0 / np.cosh(np.clip(d / w, -350.0, 350.0)) ** 2
    ux = sech2 / w
    uy = sech2 / w * (-0.3 * 2.0 * np.pi * np.cos(2.0 * np.pi * y))
    return ux, uy


# --------------------------------------------------------------------------
# the benchmark configurations
# --------------------------------------------------------------------------
def config1(n_paths: int = 10_000) -> Instance:
    """33x33 Dirichlet unit square, 2 subdomains split by one vertical
    interface (31 nodes), Gaussian bump exp(-r^2/0.01), alpha = 10,
    tau = 0.05, dt = 1e-4 (K = 500), 1e4 paths per node, seed 0."""
    n = 33
    x, y = uniform_mesh(n, n)
    ux, uy = gaussian_bump_grad(x, y, 0.5, 0.5, 0.01)
    rho = arc_length_monitor(ux, uy, 10.0)
    b = boundary_from_mesh(x, y)
    return Instance("bump33_2x1", n, n, 2, 1, 0, 0, 1.0, 1.0, 0.05, 500, n_paths,
                    rho, x, y, b, b.copy())


def rotating_bump_centre(t: float):
    return 0.5 + 0.25 * math.cos(t), 0.5 + 0.25 * math.sin(t)


def config2(n_paths: int = 100_000, t: float = 0.0, mesh=None, mesh_step: int = 0) -> Instance:
    """129x129 Dirichlet, 4x4 subdomains (753 nodes), rotating Gaussian
    bump exp(-|x-c(t)|^2/0.005), c(t) = 0.5 + 0.25 (cos t, sin t),
    alpha = 10, tau = 0.01, dt = 2e-5 (K = 500), 1e5 paths per node."""
    n = 129
    if mesh is None:
        x, y = uniform_mesh(n, n)
    else:
        x, y = mesh
    cx, cy = rotating_bump_centre(t)
    ux, uy = gaussian_bump_grad(x, y, cx, cy, 0.005)
    rho = arc_length_monitor(ux, uy, 10.0)
    b = boundary_from_mesh(x, y)
    return Instance("rotbump129_4x4", n, n, 4, 4, 0, 0, 1.0, 1.0, 0.01, 500, n_paths,
                    rho, x, y, b, b.copy(), mesh_step=mesh_step, meta={"t": t})


def config3(n_paths: int = 100_000) -> Instance:
    """257x257, periodic in xi, Dirichlet in eta, 8x8 subdomains (3776
    nodes with the periodic seam), tanh front of width 0.01 at t = 0,
    alpha = 1, tau = 0.005, dt = 1e-5 (K = 500), 1e5 paths per node."""
    n = 257
    x, y = uniform_mesh(n, n)
    ux, uy = tanh_front_grad(x, y, 0.0, 0.01)
    rho = arc_length_monitor(ux, uy, 1.0)
    b = boundary_from_mesh(x, y)
    return Instance("front257_8x8_perx", n, n, 8, 8, 1, 0, 1.0, 1.0, 0.005, 500, n_paths,
                    rho, x, y, b, b.copy())


def random_instance(rng: np.random.Generator, index: int, tau: float = 0.01, K: int = 500,
                    n_paths: int | None = None, sizes=(33, 65, 129, 257, 513),
                    subs=(2, 4, 8, 16)) -> Instance:
    """One instance of the batched mix: grid n in `sizes`, s x s subdomains,
    Gaussian bump (Dirichlet, alpha = 10) or tanh front (xi periodic,
    alpha = 1), centre and width random, paths log-uniform in [1e4, 1e6]
    rounded to a multiple of 64."""
    n = int(rng.choice(sizes))
    s = int(rng.choice(subs))
    kind = "bump" if rng.random() < 0.5 else "front"
    w = float(rng.uniform(0.005, 0.05))
    N = int(round(math.exp(rng.uniform(math.log(1e4), math.log(1e6))) / 64.0)) * 64
    if n_paths is not None:
        N = n_paths
    x, y = uniform_mesh(n, n)
    if kind == "bump":
        cx, cy = (float(v) for v in rng.uniform(0.25, 0.75, size=2))
        ux, uy = gaussian_bump_grad(x, y, cx, cy, w)
        rho = arc_length_monitor(ux, uy, 10.0)
        per_xi, meta = 0, {"kind": kind, "centre": (cx, cy), "w": w}
    else:
        ph = float(rng.uniform(0.0, 1.0))
        ux, uy = tanh_front_grad(x, y, 0.0, w, phase=ph)
        rho = arc_length_monitor(ux, uy, 1.0)
        per_xi, meta = 1, {"kind": kind, "phase": ph, "w": w}
    b = boundary_from_mesh(x, y)
    return Instance("mix%02d_%s%d_%dx%d" % (index, kind, n, s, s), n, n, s, s, per_xi, 0, 1.0, 1.0,
                    tau, K, N, rho, x, y, b, b.copy(), instance_id=index, meta=meta)


def config4(count: int = 64, seed: int = 0, n_paths: int | None = None, sizes=(33, 65, 129, 257, 513)):
    """The batched mix: `count` independent instances from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return [random_instance(rng, i, n_paths=n_paths, sizes=sizes) for i in range(count)]


def serving_stream(n_requests: int, rate_hz: float = 200.0, seed: int = 0, se_lo: float = 1e-4,
                   se_hi: float = 1e-3, max_paths: int = 1_000_000, sizes=(33, 65, 129, 257, 513)):
    """Poisson arrivals of interface-solve requests drawn from the batched
    mix.  The per-request standard-error target (log-uniform in
    [se_lo, se_hi]) sets N = min(max_paths, ceil(2 tau L^2 / SE^2)) a priori
    (sigma^2 of a displacement over one step is at most 2 tau L^2 per axis).
    Returns a list of (arrival_seconds, Instance, target_se)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += float(rng.exponential(1.0 / rate_hz))
        se = math.exp(rng.uniform(math.log(se_lo), math.log(se_hi)))
        inst = random_instance(rng, r % 65536, sizes=sizes)
        N = min(max_paths, int(math.ceil(2.0 * inst.tau * inst.Lx * inst.Lx / (se * se))))
        N = max(64, (N + 63) // 64 * 64)
        inst = replace(inst, n_paths=N, instance_id=r % 65536)
        out.append((t, inst, se))
    return out


# --------------------------------------------------------------------------
# solutions sampled at the nodes of a moving mesh (the MP loop)
# --------------------------------------------------------------------------
def rotating_bump_u(x, y, t: float, w: float = 0.005):
    """u = exp(-|x - c(t)|^2 / w) of the rotating-bump workload."""
    cx, cy = rotating_bump_centre(t)
    return np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / w)


def five_ring_u(x, y, R: float = 30.0):
    """The five-ring solution of the periodic mesh test (section 4.2): five
    tanh rings of squared radius 1/8 centred at (0, 0) and (+-1/2, +-1/2) on
    [-1, 1[^2, sharpness R."""
    u = np.zeros(np.broadcast(x, y).shape)
    for cx, cy in ((0.0, 0.0), (0.5, 0.5), (0.5, -0.5), (-0.5, 0.5), (-0.5, -0.5)):
        u = u + np.tanh(R * ((x - cx) ** 2 + (y - cy) ** 2 - 0.125))
    return u


@dataclass
class MeshLoop:
    """A moving-mesh run: grid, partition, step, the solution u(x, y, t)
    whose arc-length monitor drives the mesh, and the starting mesh."""
    name: str
    n_xi: int
    n_eta: int
    sub_xi: int
    sub_eta: int
    periodic_xi: int
    periodic_eta: int
    Lx: float
    Ly: float
    tau: float
    K: int
    n_paths: int
    steps: int
    alpha: float
    normalize: bool
    x0: np.ndarray
    y0: np.ndarray
    u: object                     # callable (x, y, t) -> u at the nodes

    def problem_kwargs(self, mesh_step: int = 0) -> dict:
        return dict(n_xi=self.n_xi, n_eta=self.n_eta, sub_xi=self.sub_xi, sub_eta=self.sub_eta,
                    periodic_xi=self.periodic_xi, periodic_eta=self.periodic_eta, Lx=self.Lx, Ly=self.Ly,
                    tau=self.tau, K=self.K, mesh_step=mesh_step)


def rotating_bump_loop(n_paths: int = 100_000, steps: int = 50) -> MeshLoop:
    """The 129x129, 4x4 rotating bump advanced over `steps` mesh steps of
    tau = 0.01 (K = 500): u re-evaluated on every new mesh, with the
    normalised arc-length monitor alpha = 10 / max |grad u|^2 of the paper's
    Dirichlet test (rho <= sqrt(11)).  Unnormalised alpha = 10 (rho up to 38)
    folds even the single-domain mesh within four such steps."""
    x, y = uniform_mesh(129, 129)
    return MeshLoop("mp_rotbump129_4x4", 129, 129, 4, 4, 0, 0, 1.0, 1.0, 0.01, 500, n_paths, steps, 10.0, True,
                    x, y, lambda xx, yy, t: rotating_bump_u(xx, yy, t))


def five_ring_loop(sub: int, n: int = 41, n_paths: int = 10_000, steps: int = 100, K: int = 1,
                   comp_side: float = 2.0) -> MeshLoop:
    """The five-ring periodic mesh test (section 4.2): [-1, 1[^2 periodic in
    both axes, n x n nodes (node n-1 is the image of node 0), sub x sub
    subdomains, R = 30, alpha = 0.2, time step 5e-4 with K substeps (the
    paper uses one), 1e4 paths, 100 steps to t = 0.05.

    The computational coordinates span a square of side `comp_side` (2: the
    same [-1, 1[^2 as the physical domain).  The generator's operator scales
    as 1 / side^2 under a change of that side, so a step of 5e-4 there is a
    step of 5e-4 / side^2 in the unit-square coordinates every solver here
    works in (comp_side = 1 reads the step in unit-square time instead)."""
    x, y = uniform_mesh(n, n, 2.0, 2.0)
    tau = 5e-4 / (comp_side * comp_side)
    return MeshLoop("five_ring%d_%dx%d_K%d" % (n, sub, sub, K) + ("" if comp_side == 2.0 else "_side%g" % comp_side),
                    n, n, sub, sub, 1, 1, 2.0, 2.0, tau, K, n_paths, steps, 0.2, False, x - 1.0, y - 1.0,
                    lambda xx, yy, t: five_ring_u(xx, yy))


# --------------------------------------------------------------------------
# small special-case inputs used by the closed-form checks
# --------------------------------------------------------------------------
def constant_problem(n: int, sub: int, periodic_xi: int, periodic_eta: int, tau: float, K: int,
                     n_paths: int, Lx: float = 1.0, Ly: float = 1.0, name: str = "const") -> Instance:
    """Constant monitor (rho = 1) on a uniform mesh: the heat-equation case."""
    x, y = uniform_mesh(n, n, Lx, Ly)
    rho = np.ones((n, n))
    b = boundary_from_mesh(x, y)
    return Instance(name, n, n, sub, sub, periodic_xi, periodic_eta, Lx, Ly, tau, K, n_paths,
                    rho, x, y, b, b.copy())
