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
# Algorithmic VALU issue slots per executed path-step (Philox 0.75 blocks,
# two uniforms, Box-Muller, bilinear cell location and three fields, drift,
# EM, side distance, exit and bridge pre-tests, substep counter), weighted by
# the measured issue cost of each instruction class.
W_SLOTS_PER_STEP = 86.5

# HBM traffic of one paths_fp32 launch on the 129x129, 4x4 workload at the
# default launch (single instance: the LDS-table kernel at level 2, 1024
# threads per workgroup, one workgroup per CU, 128-path chunks), from two
# rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch), each scaled by what the counter reads for a 1 GiB device copy in
# the same run (FETCH_SIZE reads 524708 KiB: x2.0; WRITE_SIZE reads 1.0492e6
# KiB: x1.0).  Most of the writes are L2 write-backs of the waves' end-state
# buffers.  Valid only for the kernel code it was measured on
# (kernels_code_sha1: SHA-1 of csrc/kernels.hip without comments); reported
# as null otherwise.
TRAFFIC_RECORD = {"kernels_sha1": "a66ea9c138f2fd0073ad12e22fe7f2c9808fb4cc", "fetch_kib": 8889.0,
                  "write_kib": 247854.0, "fetch_scale": 2.0, "write_scale": 1.0}


def kernels_code_sha1():
    """SHA-1 of csrc/kernels.hip with its // comments and blank lines removed
    (an edit of a comment does not change the kernels)."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_1504_00084_amd", "csrc", "kernels.hip")
    lines = []
    with open(src, encoding="utf-8") as f:
        for line in f:
            line = re.sub(r"//.*$", "", line).rstrip()
            if line:
                lines.append(line)
    return hashlib.sha1("\n".join(lines).encode()).hexdigest()


def recorded_traffic():
    r = TRAFFIC_RECORD
    if kernels_code_sha1() != r["kernels_sha1"]:
        return None
    return 1024.0 * (r["fetch_kib"] * r["fetch_scale"] + r["write_kib"] * r["write_scale"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--paths", type=int, default=100_000)
    ap.add_argument("--workload", default="rotbump129", choices=["rotbump129", "front257"],
                    help="step mode: the rotating bump 129^2 4x4 (the metric's workload), or the periodic "
                         "tanh front 257^2 8x8 (windowed kernel)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving burst of the step mode")
    ap.add_argument("--tune", action="store_true",
                    help="run the library's autotuner first (default: the library's default launch shape, the "
                         "one the recorded HBM traffic was measured with)")
    ap.add_argument("--launch", default="", help="fixed launch shape BLOCK,WAVES_PER_SIMD,CHUNK")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU work of the oracle sample")
    ap.add_argument("--mode", default="step", choices=["step", "batch", "serve", "mp", "quality", "variants"],
                    help="step: the metric line (rotating bump 129^2); batch: the 64-instance mix in one "
                         "persistent launch; serve: Poisson request stream through submit/poll; mp: the "
                         "rotating-bump moving-mesh loop; quality: five-ring mesh quality R against the "
                         "single-domain mesh")
    ap.add_argument("--mp-steps", type=int, default=50, help="mesh steps of the mp mode")
    ap.add_argument("--quality-subs", default="2,3,4", help="subdomains per axis of the quality mode")
    ap.add_argument("--quality-K", default="1,10", help="path substeps per mesh step of the quality mode")
    ap.add_argument("--quality-stride", default="1,2",
                    help="interface sampling strides of the quality mode (skipped where a stride does not divide "
                         "the subdomain size)")
    ap.add_argument("--mp-stride", default="1,2,4", help="interface sampling strides of the mp mode")
    ap.add_argument("--variants", default="1x1,2x1,4x1,1x2,1x3",
                    help="kxl schedules of the variants mode: k MᵏP sub-steps, l (MP)ˡ passes")
    ap.add_argument("--variant-steps", type=int, default=20, help="mesh steps of the variants mode")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-scale", type=float, default=1.0, help="scale the mix's path counts (batch mode)")
    ap.add_argument("--batch-sizes", default="",
                    help="comma-separated grid sizes: keep only the mix's instances of these sizes (batch mode)")
    ap.add_argument("--requests", type=int, default=40, help="requests in serve mode")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="arrival rate in req/s for serve mode (0: 0.7 x the measured capacity)")
    ap.add_argument("--serve-sizes", default="33,65,129", help="grid sizes of the serving mix")
    ap.add_argument("--serve-max-paths", type=int, default=200_000, help="cap on a request's paths per node")
    ap.add_argument("--serve-precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--budget-mb", type=int, default=0, help="HBM budget of the serving context (0: 90%% free)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.mode == "batch":
        return run_batch(args)
    if args.mode == "serve":
        return run_serve(args)
    if args.mode == "mp":
        return run_mp(args)
    if args.mode == "quality":
        return run_quality(args)
    if args.mode == "variants":
        return run_variants(args)
    import numpy as np
    import torch

    from paper_1504_00084_amd import mesh_sdd as M
    from paper_1504_00084_amd import workloads as W

    M.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    inst = W.config2(n_paths=args.paths) if args.workload == "rotbump129" else W.config3(n_paths=args.paths)
    log("workload %s: grid %dx%d, %dx%d subdomains, N=%d, K=%d, tau=%g"
        % (inst.name, inst.n_xi, inst.n_eta, inst.sub_xi, inst.sub_eta, inst.n_paths, inst.K, inst.tau))

    with torch.cuda.stream(stream):
        rho = torch.from_numpy(inst.rho).to(dev)
        x = torch.from_numpy(inst.x).to(dev)
        y = torch.from_numpy(inst.y).to(dev)
        b0 = torch.from_numpy(inst.bnd_t0).to(dev)
        b1 = torch.from_numpy(inst.bnd_t1).to(dev)
    stream.synchronize()
    if args.copy_mb:
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("plain copy: %d MiB read, %d MiB written" % (args.copy_mb, args.copy_mb))
        del src, dst
    ctx = M.mesh_sdd_ctx_create(0, 0, stream.cuda_stream)
    h32 = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
    m = M.mesh_sdd_num_interface_nodes(h32)
    outs = [torch.empty(m, dtype=torch.float64, device=dev) for _ in range(5)]
    res = M.make_result(*outs)
    step = M.make_step(x, y, b0, b1, paths_per_node=inst.n_paths, mesh_step=0)

    M.mesh_sdd_set_monitor(h32, rho)
    if args.launch:
        b, w, c = (int(v) for v in args.launch.split(","))
        M.mesh_sdd_set_launch(ctx, M.make_launch(b, w, c))
    elif args.tune:
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
    # node tables the library stages in LDS for this single-instance launch
    tables = {0: None, 2: "rho + dt rho_xi", 3: "rho + dt rho_xi windows"}[lo.table_level]
    per_launch = executed / args.steps
    achieved = W_SLOTS_PER_STEP * per_launch / kern_s / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 3), "unit": "TOP/s",
                "frac": round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": recorded_traffic() if args.workload == "rotbump129" else None,
                "kernel": {0: "paths_fp32 (cell records)",
                           2: "paths_fp32 (LDS table: rho + dt rho_xi; 1024 threads x 1 workgroup per CU)",
                           3: "paths_fp32_win (LDS windows of rho + dt rho_xi; 1024 threads x 1 workgroup per CU)"}[
                               lo.table_level], "kernel_ms": round(kern_s * 1e3, 3),
                "path_steps_per_launch": per_launch, "slots_per_path_step": W_SLOTS_PER_STEP}

    # p50 / p99 of a short FP32 serving burst (0.7 x capacity) beside the throughput
    serving = None
    if not args.no_serve:
        serving = serve_measure(24, "fp32", [int(v) for v in args.serve_sizes.split(",")], args.serve_max_paths,
                                quiet=True)
        log("serving: %d requests at %.2f req/s: p50 %.1f ms, p99 %.1f ms"
            % (serving["requests"], serving["rate_req_s"], serving["p50_ms"], serving["p99_ms"]))

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
                   "max_se": se_max, "launch": {"block": 1024 if tables else lo.block,
                                                "waves_per_simd": 4 if tables else lo.waves_per_simd,
                                                "chunk_paths": lo.chunk_paths, "lds_tables": tables or "none (L2)"}},
        "fp64_plain": fp64,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving_fp32": serving,
    }
    print(json.dumps(line), flush=True)
    M.mesh_sdd_destroy(h32)
    M.mesh_sdd_ctx_destroy(ctx)


def run_batch(args):
    """The batched mix: independent instances (grids 33..513, 2x2..16x16
    subdomains, bump or periodic front, 1e4..1e6 paths) in ONE persistent
    FP32 launch through mesh_sdd_solve_batch."""
    import numpy as np
    import torch

    from paper_1504_00084_amd import mesh_sdd as M
    from paper_1504_00084_amd import workloads as W

    M.load()
    insts = W.config4(count=args.batch_count)
    if args.batch_sizes:
        keep = {int(v) for v in args.batch_sizes.split(",")}
        insts = [it for it in insts if it.n_xi in keep]
    if args.batch_scale != 1.0:
        for it in insts:
            it.n_paths = max(64, int(it.n_paths * args.batch_scale) // 64 * 64)
    ctx = M.mesh_sdd_ctx_create(0)
    hs, ms, steps, results, arrs = [], [], [], [], []
    for it in insts:
        h = M.mesh_sdd_create(ctx, M.desc_for(it, M.FP32))
        M.mesh_sdd_set_monitor(h, it.rho)
        m = M.mesh_sdd_num_interface_nodes(h)
        a, r = M.host_result(m)
        hs.append(h)
        ms.append(m)
        arrs.append(a)
        results.append(r)
        steps.append(M.make_step(it.x, it.y, it.bnd_t0, it.bnd_t1, paths_per_node=it.n_paths))
    if args.launch:
        b, w, c = (int(v) for v in args.launch.split(","))
        M.mesh_sdd_set_launch(ctx, M.make_launch(b, w, c))
    nominal = sum(m * it.n_paths * it.K for m, it in zip(ms, insts))
    log("batch: %d instances, %d interface nodes, nominal %.3e path-steps" % (len(insts), sum(ms), nominal))
    torch.cuda.synchronize()
    t = time.perf_counter()
    M.mesh_sdd_solve_batch(hs, steps, results)
    wall = time.perf_counter() - t
    executed = sum(int(r.executed_path_steps) for r in results)
    kernel_ms = results[0].device_ms
    se = max(float(np.max(np.maximum(a[2][:m], a[3][:m]))) for a, m in zip(arrs, ms) if m)
    line = {"metric": "batched mix path-steps/s (one persistent launch)", "value": executed / wall,
            "unit": "path-steps/s", "kernel_ms": kernel_ms, "wall_s": wall, "executed_path_steps": executed,
            "nominal_path_steps": nominal, "instances": len(insts), "interface_nodes": sum(ms), "max_se": se,
            "path_scale": args.batch_scale, "sizes": sorted({it.n_xi for it in insts}),
            "dtype": "f32 (paths) / f64 (sums)", "data": "synthetic",
            "roofline_frac": W_SLOTS_PER_STEP * executed / (kernel_ms / 1e3) / 1e12 / VALU_PEAK_TOPS}
    print(json.dumps(line), flush=True)
    for h in hs:
        M.mesh_sdd_destroy(h)
    M.mesh_sdd_ctx_destroy(ctx)


def serve_measure(requests: int, precision: str, sizes, max_paths: int, rate: float = 0.0, budget_mb: int = 0,
                  launch: str = "", quiet: bool = False) -> dict:
    """Poisson stream of interface-solve requests from the batched mix, with
    a per-request standard-error target setting N; requests are created,
    frozen and submitted at their arrival times by client threads and
    served by the library's continuous-batching scheduler.  p50 / p99 are
    the library's submit-to-completion latencies."""
    import threading

    import numpy as np

    from paper_1504_00084_amd import mesh_sdd as M
    from paper_1504_00084_amd import workloads as W

    M.load()
    prec = M.FP32 if precision == "fp32" else M.FP64
    stream = W.serving_stream(requests, rate_hz=1.0, sizes=tuple(sizes),   # unit rate, rescaled below
                              max_paths=max_paths)
    work = []
    for _, it, _ in stream:
        m = len(M.mesh_sdd_desc_interface_nodes(M.desc_for(it))[0])
        work.append(m * it.n_paths * it.K)
    if rate <= 0.0:
        # 0.7 x capacity, capacity from the measured single-GPU rates of the
        # two paths (executed path-steps are about 0.85 of nominal)
        cap = 2.5e11 if prec == M.FP32 else 6.0e10
        rate = 0.7 * cap * 0.85 / float(np.mean(work))
    arrivals = [t / rate for t, _, _ in stream]
    ctx = M.mesh_sdd_ctx_create(0, budget_mb << 20)
    if launch:
        b, w, c = (int(v) for v in launch.split(","))
        M.mesh_sdd_set_launch(ctx, M.make_launch(b, w, c))
    log("serve: %d requests at %.3f req/s (%s), mean nominal work %.3e path-steps"
        % (len(stream), rate, precision, float(np.mean(work))))
    done, e2e, rejected = [], [], []
    lock = threading.Lock()
    t0 = time.perf_counter()

    def client(k):
        ta = arrivals[k]
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        ts = time.perf_counter()
        _, it, _ = stream[k]
        h = M.mesh_sdd_create(ctx, M.desc_for(it, prec))
        try:
            M.mesh_sdd_set_monitor(h, it.rho)
            m = M.mesh_sdd_num_interface_nodes(h)
            a, r = M.host_result(m)
            try:
                tk = M.mesh_sdd_submit(h, M.make_step(it.x, it.y, it.bnd_t0, it.bnd_t1, paths_per_node=it.n_paths))
            except M.MeshSddError as e:
                if e.code != M.E_BUDGET:
                    raise
                with lock:   # the request alone needs more device memory than the whole budget
                    rejected.append(k)
                    if not quiet:
                        log("request %d rejected: %s" % (k, e))
                return
            M.mesh_sdd_wait(ctx, tk, r, -1)
        finally:
            M.mesh_sdd_destroy(h)
        with lock:
            done.append(int(r.executed_path_steps))
            e2e.append(time.perf_counter() - ts)
            if not quiet:
                log("request %d done (%d of %d): %.3e path-steps, %.1f ms"
                    % (k, len(done), len(stream), float(r.executed_path_steps), 1e3 * e2e[-1]))

    errors = []

    def guarded(k):
        try:
            client(k)
        except Exception as e:   # re-raised once every client has ended
            with lock:
                errors.append(e)

    threads = [threading.Thread(target=guarded, args=(k,)) for k in range(len(stream))]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    wall = time.perf_counter() - t0
    if errors:
        M.mesh_sdd_ctx_destroy(ctx)
        raise errors[0]
    st = M.mesh_sdd_ctx_stats(ctx)
    out = {"precision": precision, "requests": len(stream), "rate_req_s": rate, "completed": int(st.completed),
           "failed": int(st.failed), "rejected_over_budget": len(rejected), "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "mean_ms": st.mean_ms,
           "client_p50_ms": 1e3 * float(np.percentile(e2e, 50)) if e2e else None,
           "client_p99_ms": 1e3 * float(np.percentile(e2e, 99)) if e2e else None,
           "throughput_path_steps_s": sum(done) / wall, "busy_ms": st.busy_ms, "wall_s": wall,
           "ticks": int(st.ticks), "sizes": list(sizes), "max_paths": max_paths,
           "budget_mb": budget_mb or None}
    M.mesh_sdd_ctx_destroy(ctx)
    return out


def run_serve(args):
    sizes = [int(v) for v in args.serve_sizes.split(",")]
    line = {"metric": "serving p50/p99 latency and throughput"}
    line.update(serve_measure(args.requests, args.serve_precision, sizes, args.serve_max_paths, args.rate,
                              args.budget_mb, args.launch))
    line["data"] = "synthetic"
    print(json.dumps(line), flush=True)


def run_mp(args):
    """The rotating-bump moving-mesh loop (129x129, 4x4, tau = 0.01, K = 500):
    each step samples u on the current mesh, builds the arc-length monitor
    on the GPU and runs one MP step (edge generator, FP32 interface
    estimate, subdomain solves).  Reports path-steps/s of the whole loop and
    the time split of one step."""
    import numpy as np
    import torch

    from paper_1504_00084_amd import mesh_sdd as M
    from paper_1504_00084_amd import mp_loop
    from paper_1504_00084_amd import workloads as W

    M.load()
    loop = W.rotating_bump_loop(n_paths=args.paths, steps=args.mp_steps)
    ctx = M.mesh_sdd_ctx_create(0)
    sd = mp_loop.run(ctx, loop, M.FP32, decomposed=False, log=log)      # single-domain reference mesh
    strides = [int(v) for v in args.mp_stride.split(",")]
    if 1 not in strides:
        strides.insert(0, 1)
    by_stride = []
    for s in strides:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = mp_loop.run(ctx, loop, M.FP32, decomposed=True, log=log, stride=s)
        w = time.perf_counter() - t0
        q = mp_loop.quality(ctx, loop, sd, o)
        by_stride.append((s, o, w, q))
        log("mp loop stride %d: %.1f ms per mesh step, R_max %.4f R_mean %.4f" % (s, 1e3 * w / loop.steps, q[0], q[1]))
    _, out, wall, (rmax, rmean, r) = next(t for t in by_stride if t[0] == 1)
    # time split of one step on the final mesh
    h = M.mesh_sdd_create(ctx, M.make_desc(129, 129, 4, 4, K=loop.K, tau=loop.tau))
    x, y, b = out["x"], out["y"], out["bnd"]
    m = M.mesh_sdd_num_interface_nodes(h)
    split = {}

    def timed(name, fn):
        t = time.perf_counter()
        fn()
        split[name] = 1e3 * (time.perf_counter() - t)

    u = loop.u(x, y, loop.steps * loop.tau)
    timed("monitor_ms", lambda: M.mesh_sdd_set_monitor_arclength(h, u, x, y, loop.alpha))
    bn = np.empty_like(b)
    timed("edge_ms", lambda: M.mesh_sdd_edge_generate(h, b, bn))
    arrs, res = M.host_result(m)
    step = M.make_step(x, y, b, bn, paths_per_node=loop.n_paths, mesh_step=loop.steps)
    timed("interface_ms", lambda: M.mesh_sdd_solve_interfaces(h, step, res))
    xn, yn = np.empty_like(x), np.empty_like(y)
    timed("subdomain_ms", lambda: M.mesh_sdd_subdomain_solve(h, x, y, bn, arrs[0][:m], arrs[1][:m], xn, yn))
    split["interface_kernel_ms"] = float(res.device_ms)
    M.mesh_sdd_destroy(h)
    M.mesh_sdd_ctx_destroy(ctx)
    line = {"metric": "moving-mesh loop path-steps/s (rotating bump, edge generator + interface estimate + "
                      "subdomain solves + monitor per step)",
            "value": out["executed_path_steps"] / wall, "unit": "path-steps/s", "steps": loop.steps,
            "ms_per_mesh_step": 1e3 * wall / loop.steps, "executed_path_steps": out["executed_path_steps"],
            "split_of_one_step": split, "quality_vs_single_domain": {"R_max": rmax, "R_mean": rmean,
                                                                     "R_min": float(r.min())},
            "interface_subsampling": [{"stride": s, "ms_per_mesh_step": 1e3 * w / loop.steps,
                                       "path_steps_per_mesh_step": o["executed_path_steps"] / loop.steps,
                                       "R_max": q[0], "R_mean": q[1], "R_min": float(q[2].min())}
                                      for s, o, w, q in by_stride],
            "dtype": "f32 (paths) / f64 (mesh, sums)", "data": "synthetic",
            "config": {"workload": loop.name, "grid": [129, 129], "subdomains": [4, 4], "paths_per_node": loop.n_paths,
                       "K": loop.K, "tau": loop.tau, "alpha": "10 / max |grad u|^2"}}
    print(json.dumps(line), flush=True)


def equidistribution_cv(M, ctx, loop, x, y, t):
    """Spread of rho * cell area over the cells (coefficient of variation):
    0 for a mesh that equidistributes the monitor of u(., t) exactly.  The
    monitor comes from the library on the given mesh; the cell sums are a
    benchmark-side diagnostic."""
    import numpy as np
    h = M.mesh_sdd_create(ctx, M.make_desc(loop.n_xi, loop.n_eta, 1, 1, loop.periodic_xi, loop.periodic_eta,
                                           K=loop.K, Lx=loop.Lx, Ly=loop.Ly, tau=loop.tau, precision=M.FP64))
    try:
        u = np.ascontiguousarray(loop.u(x, y, t))
        M.mesh_sdd_set_monitor_arclength(h, u, x, y, loop.alpha, loop.normalize)
        rho = np.empty_like(x)
        M.mesh_sdd_get_monitor(h, rho)
    finally:
        M.mesh_sdd_destroy(h)
    rc = 0.25 * (rho[:-1, :-1] + rho[:-1, 1:] + rho[1:, :-1] + rho[1:, 1:])
    area = 0.5 * np.abs((x[1:, 1:] - x[:-1, :-1]) * (y[1:, :-1] - y[:-1, 1:])
                        - (x[1:, :-1] - x[:-1, 1:]) * (y[1:, 1:] - y[:-1, :-1]))
    m = rc * area
    return float(np.std(m) / np.mean(m))


def run_variants(args):
    """The MᵏP and (MP)ˡ schedules (section 5) on the rotating-bump loop
    (129x129, 4x4, N = 1e5, K = 500, tau = 0.01): per schedule, the time per
    mesh step of the decomposed loop, R against the single-domain loop of
    the same schedule, and how evenly the final meshes distribute the
    monitor (coefficient of variation of rho * cell area)."""
    import torch

    from paper_1504_00084_amd import mesh_sdd as M
    from paper_1504_00084_amd import mp_loop
    from paper_1504_00084_amd import workloads as W

    M.load()
    loop = W.rotating_bump_loop(n_paths=args.paths, steps=args.variant_steps)
    ctx = M.mesh_sdd_ctx_create(0)
    rows = []
    t_end = loop.steps * loop.tau
    for v in args.variants.split(","):
        k, l = (int(a) for a in v.split("x"))
        sd = mp_loop.run(ctx, loop, M.FP32, decomposed=False, k_sub=k, l_iter=l)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sdd = mp_loop.run(ctx, loop, M.FP32, decomposed=True, k_sub=k, l_iter=l, log=log)
        wall = time.perf_counter() - t0
        rmax, rmean, r = mp_loop.quality(ctx, loop, sd, sdd)
        row = {"k_sub": k, "l_iter": l, "ms_per_mesh_step": 1e3 * wall / loop.steps,
               "path_steps_per_s": sdd["executed_path_steps"] / wall, "R_max": rmax, "R_mean": rmean,
               "R_min": float(r.min()), "equidistribution_cv_sdd": equidistribution_cv(M, ctx, loop, sdd["x"],
                                                                                        sdd["y"], t_end),
               "equidistribution_cv_sd": equidistribution_cv(M, ctx, loop, sd["x"], sd["y"], t_end)}
        rows.append(row)
        log("variant k=%d l=%d: %.1f ms per mesh step, R_max %.4f R_mean %.4f, equidistribution CV %.4f (SD %.4f)"
            % (k, l, row["ms_per_mesh_step"], rmax, rmean, row["equidistribution_cv_sdd"],
               row["equidistribution_cv_sd"]))
    M.mesh_sdd_ctx_destroy(ctx)
    print(json.dumps({"metric": "MᵏP / (MP)ˡ schedules on the rotating-bump loop: time per mesh step, R = Q_SD / "
                                "Q_SDD, equidistribution spread at the final time",
                      "results": rows, "steps": loop.steps, "dtype": "f32 (paths) / f64 (mesh)",
                      "data": "synthetic", "config": {"workload": loop.name, "grid": [129, 129], "subdomains": [4, 4],
                                                      "paths_per_node": loop.n_paths, "K": loop.K, "tau": loop.tau}}),
          flush=True)


def run_quality(args):
    """Five-ring periodic mesh test: 100 steps of dt = 5e-4 (K = 1), 1e4 paths,
    alpha = 0.2, R = 30, on [-1, 1[^2; the decomposed mesh against the
    single-domain mesh, R_max and R_mean of R = Q_SD / Q_SDD.  41 nodes per
    axis (40 distinct) for 2x2 and 4x4; 43 for 3x3 (40 is not a multiple
    of 3)."""
    from paper_1504_00084_amd import mesh_sdd as M
    from paper_1504_00084_amd import mp_loop
    from paper_1504_00084_amd import workloads as W

    M.load()
    ctx = M.mesh_sdd_ctx_create(0)
    rows = []
    strides = [int(v) for v in args.quality_stride.split(",")]
    for K in (int(v) for v in args.quality_K.split(",")):
        for sub in (int(v) for v in args.quality_subs.split(",")):
            n = 41 if 40 % sub == 0 else next(k for k in range(41, 200) if (k - 1) % sub == 0)
            loop = W.five_ring_loop(sub, n=n, K=K)
            sd = mp_loop.run(ctx, loop, M.FP32, decomposed=False, log=log)
            for s in strides:
                if s > 1 and ((n - 1) // sub) % s:
                    continue
                t = time.perf_counter()
                sdd = mp_loop.run(ctx, loop, M.FP32, decomposed=True, log=log, stride=s)
                rmax, rmean, r = mp_loop.quality(ctx, loop, sd, sdd)
                rows.append({"subdomains": sub, "n": n, "K": K, "interface_stride": s,
                             "interface_nodes": sdd["interface_nodes"], "R_max": rmax, "R_mean": rmean,
                             "R_min": float(r.min()), "steps": loop.steps, "wall_s": time.perf_counter() - t})
                log("five ring %dx%d (n=%d, K=%d, stride %d): R_max %.4f R_mean %.4f R_min %.4f"
                    % (sub, sub, n, K, s, rmax, rmean, r.min()))
    M.mesh_sdd_ctx_destroy(ctx)
    print(json.dumps({"metric": "five-ring mesh quality R = Q_SD / Q_SDD (max, mean over cells) at t = 0.05",
                      "results": rows, "paper": "R_max = R_mean = 1 at 2x2, 3x3 and 4x4",
                      "dtype": "f32 (paths) / f64 (mesh)", "data": "synthetic (analytic u)"}), flush=True)


if __name__ == "__main__":
    main()
