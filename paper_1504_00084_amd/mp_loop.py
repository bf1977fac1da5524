"""Moving-mesh (MP) loop through the C-ABI (sections 3.2 and 3.4-3.6).

Each mesh step: the solution u is sampled at the nodes of the current mesh,
the library turns it into the frozen arc-length monitor on the GPU
(``mesh_sdd_set_monitor_arclength``), and ``mesh_sdd_mp_step`` advances the
mesh by the edge generator, the interface estimate and the subdomain
solves.  The single-domain reference of section 3.7 runs the same loop with
``mesh_sdd_single_domain_solve`` in place of the decomposed step.  This
module only sequences calls and moves arrays; every numerical step runs in
the library's kernels.  The MᵏP and (MP)ˡ variants of section 5 are
sequences of the same calls plus the monitor transfer
(``mesh_sdd_transfer_field``).
"""
from __future__ import annotations

import time

import numpy as np

from . import mesh_sdd as M
from . import workloads as W


def _desc(loop: W.MeshLoop, precision: int, seed: int, instance_id: int, k_sub: int = 1):
    return M.make_desc(loop.n_xi, loop.n_eta, loop.sub_xi, loop.sub_eta, loop.periodic_xi, loop.periodic_eta,
                       K=loop.K // k_sub, Lx=loop.Lx, Ly=loop.Ly, tau=loop.tau / k_sub, precision=precision,
                       seed=seed, instance_id=instance_id)


def run(ctx, loop: W.MeshLoop, precision: int = M.FP32, decomposed: bool = True, steps: int | None = None,
        opts: M.MpOpts | None = None, seed: int = 0, instance_id: int = 0, log=None, stride: int = 0,
        k_sub: int = 1, l_iter: int = 1, monitor_of=None) -> dict:
    """Advance loop.x0, loop.y0 over `steps` (default loop.steps) mesh steps.

    stride > 1 estimates every stride-th node of each interface line and
    interpolates the others (section 3.6).  k_sub > 1 runs the MᵏP variant
    (section 5): k_sub sub-steps of tau / k_sub (K / k_sub path substeps
    each, random streams of mesh-step counter n k_sub + s), the monitor of
    sub-step s > 0 being the piecewise-linear transfer of (x^n, rho^n) onto
    the current sub-mesh.  l_iter > 1 runs (MP)ˡ: pass m > 1 repeats the step
    from x^n with the monitor of u(., t^{n+1}) on the mesh of pass m - 1,
    on the same random streams.  monitor_of(x, y, t), when given, replaces
    the arc-length monitor of loop.u.

    Returns the final mesh and boundary arrays, the executed path-steps and
    the per-step wall and device times."""
    if k_sub < 1 or l_iter < 1 or loop.K % k_sub:
        raise ValueError("k_sub must divide K; k_sub, l_iter >= 1")
    if k_sub > 1 and l_iter > 1:
        raise ValueError("MᵏP and (MP)ˡ are separate variants")
    steps = loop.steps if steps is None else steps
    h = M.mesh_sdd_create(ctx, _desc(loop, precision, seed, instance_id, k_sub))
    try:
        m = M.mesh_sdd_num_interface_nodes(h)
        x = np.ascontiguousarray(loop.x0, dtype=np.float64)
        y = np.ascontiguousarray(loop.y0, dtype=np.float64)
        b = W.boundary_from_mesh(x, y)
        executed, wall, dev = 0, [], []
        has_sides = not (loop.periodic_xi and loop.periodic_eta)

        def install(xm, ym, t):
            if monitor_of is not None:
                M.mesh_sdd_set_monitor(h, np.ascontiguousarray(monitor_of(xm, ym, t), dtype=np.float64))
            else:
                u = np.ascontiguousarray(loop.u(xm, ym, t), dtype=np.float64)
                M.mesh_sdd_set_monitor_arclength(h, u, xm, ym, loop.alpha, loop.normalize)

        def advance(xa, ya, ba, counter):
            nonlocal executed
            xn, yn, bn = np.empty_like(xa), np.empty_like(ya), np.empty_like(ba)
            if decomposed:
                arrs, res = M.host_result(m)
                step = M.make_step(xa, ya, ba, ba, paths_per_node=loop.n_paths, mesh_step=counter,
                                   interface_stride=stride)
                M.mesh_sdd_mp_step(h, step, xn, yn, bn, res, opts)
                executed += int(res.executed_path_steps)
                dev.append(float(res.device_ms))
            else:
                if has_sides:
                    M.mesh_sdd_edge_generate(h, ba, bn, opts)
                else:
                    bn[:] = ba
                M.mesh_sdd_single_domain_solve(h, xa, ya, bn, xn, yn, opts)
            return xn, yn, bn

        rho_n, rho_s = np.empty_like(x), np.empty_like(x)
        for n in range(steps):
            t0 = time.perf_counter()
            install(x, y, n * loop.tau)
            xs, ys, bs = x, y, b
            if k_sub > 1:
                M.mesh_sdd_get_monitor(h, rho_n)
            for s in range(k_sub):
                if s > 0:
                    M.mesh_sdd_transfer_field(h, x, y, rho_n, xs, ys, rho_s)
                    M.mesh_sdd_set_monitor(h, rho_s)
                xs, ys, bs = advance(xs, ys, bs, n * k_sub + s)
            for _ in range(1, l_iter):
                install(xs, ys, (n + 1) * loop.tau)
                xs, ys, bs = advance(x, y, b, n)
            x, y, b = xs, ys, bs
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
