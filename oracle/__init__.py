"""Plain FP64 CPU oracle for the interface-node Monte-Carlo estimate.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product library
never loads it, and it shares no code with the GPU path: the arithmetic lives
in ``mc_oracle.c`` (built with gcc), and this module only marshals numpy
arrays into it.

Paper: Bihlo, Haynes & Walsh, "Stochastic domain decomposition for time
dependent adaptive mesh generation", arXiv:1504.00084, section 3.2 (Dirichlet
representation), 3.3 (periodic representation) and 3.4 (Euler-Maruyama
discretisation, bilinear/bicubic interpolation, bridge test, mean over N).

Parity pins: every function here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against something other than itself (rocRAND's
open-source Philox header, exactness on polynomials, heat-equation closed
forms, a brute-force bridge simulation, a finite-difference solve).  The
MC estimator as a whole has no published per-node values, so agreement with
the paper's own runs is "parity unpinned" at that level (their Tables 1-3
need the full mesh + physics pipeline).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``mc_oracle.c`` into ``liboracle.so`` with gcc (FP64, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n_xi", ctypes.c_int32), ("n_eta", ctypes.c_int32),
        ("sub_xi", ctypes.c_int32), ("sub_eta", ctypes.c_int32),
        ("periodic_xi", ctypes.c_int32), ("periodic_eta", ctypes.c_int32),
        ("Lx", ctypes.c_double), ("Ly", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("K", ctypes.c_int32), ("bridge", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("instance_id", ctypes.c_uint32), ("mesh_step", ctypes.c_uint32),
    ]


@dataclass
class Problem:
    """One interface solve: grid, partition, step, RNG identity."""
    n_xi: int
    n_eta: int
    sub_xi: int
    sub_eta: int
    periodic_xi: int = 0
    periodic_eta: int = 0
    Lx: float = 1.0
    Ly: float = 1.0
    tau: float = 0.05
    K: int = 500
    bridge: int = 1
    seed: int = 0
    instance_id: int = 0
    mesh_step: int = 0

    def c(self) -> _Problem:
        return _Problem(self.n_xi, self.n_eta, self.sub_xi, self.sub_eta,
                        self.periodic_xi, self.periodic_eta, self.Lx, self.Ly,
                        self.tau, self.K, self.bridge, self.seed,
                        self.instance_id, self.mesh_step)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER
    d, i32, i64, u32 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    pd, pi32, pi64, pu32 = P(d), P(i32), P(i64), P(u32)
    lib.oracle_philox4x32_10.argtypes = [pu32, pu32, pu32]
    lib.oracle_uniform.argtypes = [u32]
    lib.oracle_uniform.restype = d
    lib.oracle_box_muller.argtypes = [u32, u32, pd, pd]
    lib.oracle_normals.argtypes = [P(_Problem), i32, i64, i32, pd, pd]
    lib.oracle_bridge_uniform.argtypes = [P(_Problem), i32, i64, i32]
    lib.oracle_bridge_uniform.restype = d
    lib.oracle_stream_word.argtypes = [P(_Problem), i32, i64, i64]
    lib.oracle_stream_word.restype = u32
    lib.oracle_monitor_gradient.argtypes = [i32, i32, i32, i32, pd, pd, pd]
    lib.oracle_interface_nodes.argtypes = [P(_Problem), pi32, pi32]
    lib.oracle_interface_nodes.restype = i32
    lib.oracle_bilinear.argtypes = [i32, i32, i32, i32, pd, pd, pd, d, d, pd]
    lib.oracle_keys_bicubic.argtypes = [i32, i32, i32, i32, pd, d, d, d, d]
    lib.oracle_keys_bicubic.restype = d
    lib.oracle_bridge_probability.argtypes = [d, d, d]
    lib.oracle_bridge_probability.restype = d
    lib.oracle_solve.argtypes = [P(_Problem), pd, pd, pd, pd, pd, i64, i32, pi32, i32,
                                 pd, pd, pd, pd, pd, pi64]
    lib.oracle_solve.restype = i32
    lib.oracle_paths.argtypes = [P(_Problem), pd, pd, pd, pd, pd, i32, i64, i64,
                                 pd, pd, pi32, pi32, pi32, pd]
    lib.oracle_paths.restype = i32
    lib.oracle_path_amplification.argtypes = [P(_Problem), pd, pd, pd, pd, pd, i32, i64, i64, pd]
    lib.oracle_path_amplification.restype = i32
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def philox4x32_10(ctr, key):
    """Philox4x32-10 block for counter (4 words) and key (2 words)."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib.oracle_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform(r: int) -> float:
    return float(_load().oracle_uniform(int(r) & 0xFFFFFFFF))


def box_muller(r0: int, r1: int):
    a, b = ctypes.c_double(), ctypes.c_double()
    _load().oracle_box_muller(int(r0) & 0xFFFFFFFF, int(r1) & 0xFFFFFFFF, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def normals(prob: Problem, node: int, path: int, k: int):
    a, b = ctypes.c_double(), ctypes.c_double()
    pc = prob.c()
    _load().oracle_normals(ctypes.byref(pc), node, path, k, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def stream_word(prob: Problem, node: int, path: int, q: int) -> int:
    """Word q of the random stream of one path."""
    pc = prob.c()
    return int(_load().oracle_stream_word(ctypes.byref(pc), node, path, q))


def bridge_uniform(prob: Problem, node: int, path: int, k: int) -> float:
    pc = prob.c()
    return float(_load().oracle_bridge_uniform(ctypes.byref(pc), node, path, k))


def monitor_gradient(rho, periodic_xi: int = 0, periodic_eta: int = 0):
    """Finite-difference (rho_xi, rho_eta) of a [n_eta, n_xi] monitor."""
    rho = _f64(rho)
    n_eta, n_xi = rho.shape
    rx = np.empty_like(rho)
    ry = np.empty_like(rho)
    _load().oracle_monitor_gradient(n_xi, n_eta, periodic_xi, periodic_eta,
                                    _ptr(rho, ctypes.c_double), _ptr(rx, ctypes.c_double),
                                    _ptr(ry, ctypes.c_double))
    return rx, ry


def interface_nodes(prob: Problem):
    """Interface nodes as (i, j) int32 arrays in row-major (j, i) order."""
    lib = _load()
    pc = prob.c()
    n = lib.oracle_interface_nodes(ctypes.byref(pc), None, None)
    i = np.empty(max(n, 1), dtype=np.int32)
    j = np.empty(max(n, 1), dtype=np.int32)
    lib.oracle_interface_nodes(ctypes.byref(pc), _ptr(i, ctypes.c_int32), _ptr(j, ctypes.c_int32))
    return i[:n], j[:n]


def bilinear(rho, rho_xi, rho_eta, xi: float, eta: float, periodic_xi: int = 0, periodic_eta: int = 0):
    rho, rho_xi, rho_eta = _f64(rho), _f64(rho_xi), _f64(rho_eta)
    n_eta, n_xi = rho.shape
    out = np.empty(3)
    _load().oracle_bilinear(n_xi, n_eta, periodic_xi, periodic_eta, _ptr(rho, ctypes.c_double),
                            _ptr(rho_xi, ctypes.c_double), _ptr(rho_eta, ctypes.c_double),
                            float(xi), float(eta), _ptr(out, ctypes.c_double))
    return out


def keys_bicubic(f, xi: float, eta: float, periodic_xi: int = 0, periodic_eta: int = 0,
                 off_xi: float = 0.0, off_eta: float = 0.0) -> float:
    f = _f64(f)
    n_eta, n_xi = f.shape
    return float(_load().oracle_keys_bicubic(n_xi, n_eta, periodic_xi, periodic_eta,
                                             _ptr(f, ctypes.c_double), off_xi, off_eta,
                                             float(xi), float(eta)))


def bridge_probability(d0: float, d1: float, dt: float) -> float:
    return float(_load().oracle_bridge_probability(d0, d1, dt))


def solve(prob: Problem, rho, x_cur, y_cur, bnd_t0, bnd_t1, n_paths: int,
          nodes=None, threads: int | None = None) -> dict:
    """Per-node estimate at the interface nodes.

    ``nodes``: ranks into the interface enumeration (None: all).  Returns a
    dict of numpy arrays mean_x, mean_y, se_x, se_y, exit_frac, steps and
    the ranks solved.
    """
    lib = _load()
    pc = prob.c()
    rho, x_cur, y_cur = _f64(rho), _f64(x_cur), _f64(y_cur)
    bnd_t0, bnd_t1 = _f64(bnd_t0), _f64(bnd_t1)
    if nodes is None:
        ranks = np.arange(lib.oracle_interface_nodes(ctypes.byref(pc), None, None), dtype=np.int32)
    else:
        ranks = np.ascontiguousarray(nodes, dtype=np.int32)
    m = len(ranks)
    outs = {k: np.empty(max(m, 1)) for k in ("mean_x", "mean_y", "se_x", "se_y", "exit_frac")}
    steps = np.empty(max(m, 1), dtype=np.int64)
    if threads is None:
        threads = os.cpu_count() or 1
    rc = lib.oracle_solve(ctypes.byref(pc), _ptr(rho, ctypes.c_double), _ptr(x_cur, ctypes.c_double),
                          _ptr(y_cur, ctypes.c_double), _ptr(bnd_t0, ctypes.c_double),
                          _ptr(bnd_t1, ctypes.c_double), int(n_paths), m,
                          _ptr(ranks, ctypes.c_int32), int(threads),
                          _ptr(outs["mean_x"], ctypes.c_double), _ptr(outs["mean_y"], ctypes.c_double),
                          _ptr(outs["se_x"], ctypes.c_double), _ptr(outs["se_y"], ctypes.c_double),
                          _ptr(outs["exit_frac"], ctypes.c_double), _ptr(steps, ctypes.c_int64))
    if rc != 0:
        raise ValueError("oracle_solve rejected its arguments")
    res = {k: v[:m] for k, v in outs.items()}
    res["steps"] = steps[:m]
    res["nodes"] = ranks
    return res


def path_amplification(prob: Problem, rho, x_cur, y_cur, bnd_t0, bnd_t1, node: int, p_begin: int,
                       p_end: int):
    """Per path, how much it amplifies rounding (linearised, not an
    estimate): the standard deviation of its end point in (xi, eta) per unit
    standard deviation of independent perturbations of each coordinate
    after every substep; sqrt(substeps) where there is no drift."""
    lib = _load()
    pc = prob.c()
    rho, x_cur, y_cur = _f64(rho), _f64(x_cur), _f64(y_cur)
    bnd_t0, bnd_t1 = _f64(bnd_t0), _f64(bnd_t1)
    n = p_end - p_begin
    amp = np.empty(max(n, 1))
    rc = lib.oracle_path_amplification(ctypes.byref(pc), _ptr(rho, ctypes.c_double), _ptr(x_cur, ctypes.c_double),
                                       _ptr(y_cur, ctypes.c_double), _ptr(bnd_t0, ctypes.c_double),
                                       _ptr(bnd_t1, ctypes.c_double), node, p_begin, p_end,
                                       _ptr(amp, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_path_amplification rejected its arguments")
    return amp[:n]


def paths(prob: Problem, rho, x_cur, y_cur, bnd_t0, bnd_t1, node: int, p_begin: int, p_end: int,
          trace: bool = False) -> dict:
    """Per-path outcomes of one node (values, exit flag/side, steps, trace)."""
    lib = _load()
    pc = prob.c()
    rho, x_cur, y_cur = _f64(rho), _f64(x_cur), _f64(y_cur)
    bnd_t0, bnd_t1 = _f64(bnd_t0), _f64(bnd_t1)
    n = p_end - p_begin
    vx, vy = np.empty(max(n, 1)), np.empty(max(n, 1))
    ex, sd, st = (np.empty(max(n, 1), dtype=np.int32) for _ in range(3))
    tr = np.full((max(n, 1), prob.K, 4), np.nan) if trace else None
    rc = lib.oracle_paths(ctypes.byref(pc), _ptr(rho, ctypes.c_double), _ptr(x_cur, ctypes.c_double),
                          _ptr(y_cur, ctypes.c_double), _ptr(bnd_t0, ctypes.c_double),
                          _ptr(bnd_t1, ctypes.c_double), node, p_begin, p_end,
                          _ptr(vx, ctypes.c_double), _ptr(vy, ctypes.c_double),
                          _ptr(ex, ctypes.c_int32), _ptr(sd, ctypes.c_int32), _ptr(st, ctypes.c_int32),
                          _ptr(tr, ctypes.c_double) if trace else None)
    if rc != 0:
        raise ValueError("oracle_paths rejected its arguments")
    out = {"vx": vx[:n], "vy": vy[:n], "exited": ex[:n], "side": sd[:n], "steps": st[:n]}
    if trace:
        out["trace"] = tr[:n]
    return out
