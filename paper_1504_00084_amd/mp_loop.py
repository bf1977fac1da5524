"""Moving-mesh (MP) loop through the C-ABI (sections 3.2 and 3.4-3.6).

Each mesh step: the solution u is sampled at the nodes of the current mesh,
the library turns it into the frozen arc-length monitor on the GPU
(``mesh_sdd_set_monitor_arclength``), and ``mesh_sdd_mp_step`` advances the
mesh by the edge generator, the interface estimate and the subdomain
solves.  The single-domain reference of section 3.7 runs the same loop with
``mesh_sdd_single_domain_solve`` in place of the decomposed step.  This
module only sequences calls and moves arrays; every numerical step runs in
the library's kernels.
"""
from __future__ import annotations

import time

import numpy as np

from . import mesh_sdd as M
from . import workloads as W


def _desc(loop: W.MeshLoop, precision: int, seed: int, instance_id: int):
    return M.make_desc(loop.n_xi, loop.n_eta, loop.sub_xi, loop.sub_eta, loop.periodic_xi, loop.periodic_eta,
                       K=loop.K, Lx=loop.Lx, Ly=loop.Ly, tau=loop.tau, precision=precision, seed=seed,
                       instance_id=instance_id)


def run(ctx, loop: W.MeshLoop, precision: int = M.FP32, decomposed: bool = True, steps: int | None = None,
        opts: M.MpOpts | None = None, seed: int = 0, instance_id: int = 0, log=None, stride: int = 0) -> dict:
    """Advance loop.x0, loop.y0 over `steps` (default loop.steps) mesh steps.
    stride > 1 estimates every stride-th node of each interface line and
    interpolates the others (section 3.6).

    Returns the final mesh and boundary arrays, the executed path-steps and
    the per-step wall and device times."""
    steps = loop.steps if steps is None else steps
    h = M.mesh_sdd_create(ctx, _desc(loop, precision, seed, instance_id))
    try:
        m = M.mesh_sdd_num_interface_nodes(h)
        x = np.ascontiguousarray(loop.x0, dtype=np.float64)
        y = np.ascontiguousarray(loop.y0, dtype=np.float64)
        b = W.boundary_from_mesh(x, y)
        executed, wall, dev = 0, [], []
        has_sides = not (loop.periodic_xi and loop.periodic_eta)
        for n in range(steps):
            t0 = time.perf_counter()
            u = np.ascontiguousarray(loop.u(x, y, n * loop.tau), dtype=np.float64)
            M.mesh_sdd_set_monitor_arclength(h, u, x, y, loop.alpha, loop.normalize)
            xn, yn, bn = np.empty_like(x), np.empty_like(y), np.empty_like(b)
            if decomposed:
                arrs, res = M.host_result(m)
                step = M.make_step(x, y, b, b, paths_per_node=loop.n_paths, mesh_step=n, interface_stride=stride)
                M.mesh_sdd_mp_step(h, step, xn, yn, bn, res, opts)
                executed += int(res.executed_path_steps)
                dev.append(float(res.device_ms))
            else:
                if has_sides:
                    M.mesh_sdd_edge_generate(h, b, bn, opts)
                else:
                    bn[:] = b
                M.mesh_sdd_single_domain_solve(h, x, y, bn, xn, yn, opts)
            x, y, b = xn, yn, bn
            wall.append(time.perf_counter() - t0)
            if log is not None and (n + 1) % max(1, steps // 10) == 0:
                log("%s %s: step %d/%d, %.1f ms" % (loop.name, "SDD" if decomposed else "SD", n + 1, steps,
                                                   1e3 * wall[-1]))
        return {"x": x, "y": y, "bnd": b, "executed_path_steps": executed, "wall_s": wall, "device_ms": dev,
                "interface_nodes": m}
    finally:
        M.mesh_sdd_destroy(h)


def quality(ctx, loop: W.MeshLoop, sd: dict, sdd: dict):
    """(R_max, R_mean, R per cell) of the decomposed mesh against the
    single-domain one (section 3.7, eq. Q)."""
    h = M.mesh_sdd_create(ctx, _desc(loop, M.FP64, 0, 0))
    try:
        r = np.empty((loop.n_eta - 1, loop.n_xi - 1))
        rmax, rmean = M.mesh_sdd_mesh_quality(h, sd["x"], sd["y"], sdd["x"], sdd["y"], r)
        return rmax, rmean, r
    finally:
        M.mesh_sdd_destroy(h)
