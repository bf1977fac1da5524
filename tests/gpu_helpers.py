"""Shared helpers of the GPU tests: run an instance through the C-ABI and
through the oracle on the same inputs and streams."""
import os
import sys

import numpy as np

THREADS = min(16, os.cpu_count() or 1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_solve(oracle_lib, inst, nodes=None, n_paths=None):
    P = oracle_lib.Problem(**inst.problem_kwargs())
    return oracle_lib.solve(P, inst.rho, inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, n_paths or inst.n_paths,
                            nodes=nodes, threads=THREADS)


def gpu_solve(M, ctx, inst, precision, n_paths=None):
    return M.solve_instance(ctx, inst, precision, n_paths=n_paths)


def compare(gpu, ora, nodes=None, tol=1e-5, label=""):
    """Per-node absolute differences of mean and SE; returns a summary."""
    idx = np.arange(len(ora["mean_x"])) if nodes is None else np.asarray(nodes)
    g = {k: np.asarray(gpu[k])[idx] for k in ("mean_x", "mean_y", "se_x", "se_y", "exit_frac")}
    err = max(np.max(np.abs(g["mean_x"] - ora["mean_x"])), np.max(np.abs(g["mean_y"] - ora["mean_y"])))
    se_err = max(np.max(np.abs(g["se_x"] - ora["se_x"])), np.max(np.abs(g["se_y"] - ora["se_y"])))
    n = gpu["paths_per_node"]
    flips = int(np.max(np.abs(g["exit_frac"] - ora["exit_frac"])) * n + 0.5)
    sig = np.concatenate([ora["se_x"], ora["se_y"]])
    z = np.concatenate([np.abs(g["mean_x"] - ora["mean_x"]) / np.maximum(ora["se_x"], 1e-300),
                        np.abs(g["mean_y"] - ora["mean_y"]) / np.maximum(ora["se_y"], 1e-300)])
    say("%s: max|dmean| = %.3e  max|dse| = %.3e  max exit-count diff = %d  max z = %.3e  (median se %.2e)"
        % (label, err, se_err, flips, np.max(z), np.median(sig)))
    return {"err": err, "se_err": se_err, "flips": flips, "zmax": float(np.max(z))}
