"""Benchmark of the interface-node Monte-Carlo solve on one MI355X.

One step = one pass of the whole hot path over one mesh step of the
rotating-bump workload (129x129 grid, 4x4 subdomains, 753 interface nodes,
1e5 paths per node, K = 500 substeps): freeze the monitor (finite-difference
table on the device), then estimate (x, y) at every interface node with the
batched FP32 kernel.  Inputs are resident in HBM before the timed region.

Prints ONE JSON line: throughput in executed path-steps per second, the
FP64 plain kernel on the same inputs and path count (equal standard error),
the roofline of the dominant kernel and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU issue peak of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (one
# non-packed VALU lane-operation per lane per clock).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic VALU issue slots per executed path-step (see the design notes:
# Philox 0.75 blocks, Box-Muller, bilinear of three fields, drift, EM, exit
# test), weighted by the measured issue cost of each instruction class.
W_SLOTS_PER_STEP = 120.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--paths", type=int, default=100_000)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true", help="use the default launch shape")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU work of the oracle sample")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1504_00084_amd import mesh_sdd as M
    from paper_1504_00084_amd import workloads as W

    M.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    inst = W.config2(n_paths=args.paths)
    log("workload %s: grid %dx%d, %dx%d subdomains, N=%d, K=%d, tau=%g"
        % (inst.name, inst.n_xi, inst.n_eta, inst.sub_xi, inst.sub_eta, inst.n_paths, inst.K, inst.tau))

    with torch.cuda.stream(stream):
        rho = torch.from_numpy(inst.rho).to(dev)
        x = torch.from_numpy(inst.x).to(dev)
        y = torch.from_numpy(inst.y).to(dev)
        b0 = torch.from_numpy(inst.bnd_t0).to(dev)
        b1 = torch.from_numpy(inst.bnd_t1).to(dev)
    stream.synchronize()
    ctx = M.mesh_sdd_ctx_create(0, 0, stream.cuda_stream)
    h32 = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
    m = M.mesh_sdd_num_interface_nodes(h32)
    outs = [torch.empty(m, dtype=torch.float64, device=dev) for _ in range(5)]
    res = M.make_result(*outs)
    step = M.make_step(x, y, b0, b1, paths_per_node=inst.n_paths, mesh_step=0)

    M.mesh_sdd_set_monitor(h32, rho)
    if not args.no_tune:
        t = time.time()
        lo = M.mesh_sdd_autotune(h32, step)
        log("autotune: block %d, waves/SIMD %d, chunk %d (%.1f s)" % (lo.block, lo.waves_per_simd, lo.chunk_paths,
                                                                      time.time() - t))
    lo = M.mesh_sdd_get_launch(h32)

    def one_step():
        M.mesh_sdd_set_monitor(h32, rho)        # a0: table of the frozen monitor
        M.mesh_sdd_solve_interfaces(h32, step, res)
        return int(res.executed_path_steps), float(res.device_ms)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    executed, kernel_ms = 0, []
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        e, k = one_step()
        executed += e
        kernel_ms.append(k)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stream_ms = ev0.elapsed_time(ev1)
    rate = executed / wall
    ms_per_step = 1e3 * wall / args.steps
    nominal = m * inst.n_paths * inst.K
    se_max = float(torch.max(torch.maximum(outs[2], outs[3])).item())
    log("fp32 batched: %.3e path-steps/s (%.1f ms/step, kernel %.1f ms avg, stream %.1f ms), executed %.3e of "
        "nominal %.3e per step, max SE %.2e" % (rate, ms_per_step, sum(kernel_ms) / len(kernel_ms), stream_ms,
                                                executed / args.steps, nominal, se_max))

    # FP64 plain kernel, one instance per launch, same inputs and N (equal SE)
    fp64 = None
    if not args.no_fp64:
        h64 = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP64))
        M.mesh_sdd_set_monitor(h64, rho)
        outs64 = [torch.empty(m, dtype=torch.float64, device=dev) for _ in range(5)]
        res64 = M.make_result(*outs64)
        torch.cuda.synchronize()
        t = time.perf_counter()
        M.mesh_sdd_solve_interfaces(h64, step, res64)
        torch.cuda.synchronize()
        w64 = time.perf_counter() - t
        fp64 = {"value": res64.executed_path_steps / w64, "ms_per_step": 1e3 * w64,
                "kernel_ms": res64.device_ms, "max_abs_diff_vs_fp32": float(torch.max(torch.abs(outs64[0] - outs[0])).item())}
        log("fp64 plain: %.3e path-steps/s (%.1f ms), fp32 vs fp64 max |dmean_x| %.2e"
            % (fp64["value"], fp64["ms_per_step"], fp64["max_abs_diff_vs_fp32"]))
        M.mesh_sdd_destroy(h64)

    kern_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    per_launch = executed / args.steps
    achieved = W_SLOTS_PER_STEP * per_launch / kern_s / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 3), "unit": "TOP/s",
                "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": None,
                "kernel": "paths_fp32", "kernel_ms": round(kern_s * 1e3, 3),
                "path_steps_per_launch": per_launch, "slots_per_path_step": W_SLOTS_PER_STEP}

    cpu = None
    if not args.no_cpu:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        P = oracle.Problem(**inst.problem_kwargs())
        # bounded sample: evenly spaced interface nodes at a reduced path count;
        # the rate in path-steps/s does not depend on N
        probe = oracle.solve(P, inst.rho, inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, 200,
                             nodes=np.arange(0, m, max(1, m // threads))[:threads], threads=threads)
        t = time.perf_counter()
        probe = oracle.solve(P, inst.rho, inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, 400,
                             nodes=np.arange(0, m, max(1, m // threads))[:threads], threads=threads)
        probe_rate = float(np.sum(probe["steps"])) / (time.perf_counter() - t)
        n_nodes = min(m, 4 * threads)
        nodes = np.linspace(0, m - 1, n_nodes).astype(np.int32)
        avg_len = float(np.sum(probe["steps"])) / (400 * len(probe["steps"]))
        n_cpu = int(max(64, args.cpu_seconds * probe_rate / (n_nodes * avg_len)))
        t = time.perf_counter()
        r = oracle.solve(P, inst.rho, inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, n_cpu, nodes=nodes, threads=threads)
        cw = time.perf_counter() - t
        cpu = {"value": float(np.sum(r["steps"])) / cw, "unit": "path-steps/s", "cores": threads, "kind": "oracle",
               "sample": "%d of %d interface nodes x %d paths x K=%d (%.1f s)" % (n_nodes, m, n_cpu, inst.K, cw)}
        log("cpu oracle: %.3e path-steps/s on %d threads (%s)" % (cpu["value"], threads, cpu["sample"]))

    line = {
        "metric": "interface-node path-steps/sec at 1 GPU (FP32 batched vs FP64 plain) at sigma<=1e-3; p99 latency",
        "value": rate, "unit": "path-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (paths) / f64 (sums)", "data": "synthetic",
        "config": {"workload": inst.name, "grid": [inst.n_xi, inst.n_eta], "subdomains": [inst.sub_xi, inst.sub_eta],
                   "interface_nodes": m, "paths_per_node": inst.n_paths, "K": inst.K, "tau": inst.tau,
                   "nominal_path_steps": nominal, "executed_path_steps_per_step": per_launch,
                   "max_se": se_max, "launch": {"block": lo.block, "waves_per_simd": lo.waves_per_simd,
                                                "chunk_paths": lo.chunk_paths}},
        "fp64_plain": fp64,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    M.mesh_sdd_destroy(h32)
    M.mesh_sdd_ctx_destroy(ctx)


if __name__ == "__main__":
    main()
