"""Benchmark of the interface-node Monte-Carlo solve on one MI355X.

One step = one pass of the whole hot path over one mesh step of the periodic
moving-front workload (257x257 grid, xi periodic, 8x8 subdomains, 3776
interface nodes, 1e5 paths per node, K = 500 substeps, tau = 0.005): freeze
the monitor (finite-difference table on the device), then estimate (x, y) at
every interface node with the batched FP32 kernel.  Inputs are resident in
HBM before the timed region.  It is the largest single-instance workload on
which every node reaches a standard error of 1e-3.

Prints ONE JSON line: throughput in executed path-steps per second; the FP64
plain kernel on the same inputs and path count (equal standard error) with
the FP32-FP64 difference of every node; the 64-instance batched mix in one
persistent launch; a short serving run of the mix (FP32 and FP64 plain); the
roofline of the dominant kernel; the CPU oracle on a bounded sample of every
workload, with the per-node GPU-oracle differences on that sample.
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


def w_slots(per_xi: int, per_eta: int) -> float:
    """Algorithmic VALU issue slots of one executed path-step: Philox
    (0.75 blocks: 15 32x32->64 multiplies at 1.3 slots, 15 three-input
    XORs), two uniforms, Box-Muller (four transcendentals at 2 slots and one
    multiply), bilinear cell location and three fields, drift (rcp), EM,
    substep bookkeeping -- 79.5 slots on every path-step -- plus, per axis,
    2 slots for a Dirichlet side distance (complement, minimum) or 4 for a
    periodic wrap (floor, subtract, convert, add), plus 3 for the exit test
    and bridge pre-test when some axis is Dirichlet.  Weights measured with
    the VALU issue-cost probe; the values are the frozen ones: 86.5 for a
    Dirichlet problem, 88.5 with one periodic axis, 87.5 with two."""
    base = 79.5
    axes = sum(4.0 if p else 2.0 for p in (per_xi, per_eta))
    exit_tests = 0.0 if (per_xi and per_eta) else 3.0
    return base + axes + exit_tests


# HBM traffic of one launch of the headline kernel, from two rocprofv3 --pmc
# runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each
# scaled by what the counter reads for a 1 GiB device copy in the same run.
# Valid only for the kernel code it was measured on (kernels_sha1: SHA-1 of
# csrc/kernels.hip without comments) and the workload named; null otherwise.
TRAFFIC_RECORD = {"workload": "front257_8x8_perx", "kernels_sha1": "be45c705c70c2caeb1190e13bbe1a85e5b0331d0",
                  "fetch_kib": 83773.9, "write_kib": 3449590.0, "fetch_scale": 2.0, "write_scale": 1.0}


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


def recorded_traffic(workload: str):
    r = TRAFFIC_RECORD
    if r["workload"] != workload or kernels_code_sha1() != r["kernels_sha1"]:
        return None
    return 1024.0 * (r["fetch_kib"] * r["fetch_scale"] + r["write_kib"] * r["write_scale"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Launch shapes found by the library's autotuner on an MI355X (per grid
# bucket and for multi-instance launches), loaded into every context the
# benchmark creates when the file exists.
TUNE_CACHE = os.path.join(ROOT, "paper_1504_00084_amd", "tune_cache.txt")


def new_ctx(M, budget_bytes=0, stream=None, tune_cache=None):
    """A library context with the tuned shapes of `tune_cache` (default: the
    committed cache, if present)."""
    ctx = M.mesh_sdd_ctx_create(0, budget_bytes, stream)
    path = TUNE_CACHE if tune_cache is None else tune_cache
    if path and os.path.exists(path):
        M.mesh_sdd_tune_load(ctx, path)
    return ctx


def host_threads():
    """Host cores this process may use for the oracle: the CPU affinity, cut
    to the cgroup's CPU quota and to OMP_NUM_THREADS where those are set (a
    container can expose its share of the host that way).  Returns (threads,
    info)."""
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except AttributeError:
        info["affinity"] = os.cpu_count()
    n = info["affinity"] or 1
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, p = f.read().split()[:2]
        if q != "max":
            info["cgroup_quota"] = float(q) / float(p)
            n = min(n, max(1, int(info["cgroup_quota"])))
    except (OSError, ValueError):
        pass
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit() and int(omp) > 0:
        info["omp_num_threads"] = int(omp)
        n = min(n, int(omp))
    info["threads"] = n
    return n, info


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--paths", type=int, default=100_000)
    ap.add_argument("--workload", default="front257", choices=["front257", "rotbump129"],
                    help="step mode: the periodic tanh front 257^2 8x8 (the headline), or the rotating bump "
                         "129^2 4x4")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and its parity check")
    ap.add_argument("--no-mix", action="store_true", help="skip the batched 64-instance mix of the step mode")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run of the step mode")
    ap.add_argument("--tune", action="store_true",
                    help="step mode: autotune the headline's bucket before timing; batch mode: time the mix with "
                         "the default shapes, autotune the batch, time it again")
    ap.add_argument("--tune-cache", default=None,
                    help="tuned shapes to load (default: paper_1504_00084_amd/tune_cache.txt if present; '' for none)")
    ap.add_argument("--tune-save", default="", help="batch mode with --tune: write the tuned shapes here")
    ap.add_argument("--launch", default="", help="fixed launch shape BLOCK,WAVES_PER_SIMD,CHUNK")
    ap.add_argument("--jsonl", default="", help="also write per-node parity and serving records to this JSONL file")
    ap.add_argument("--mode", default="step", choices=["step", "batch", "serve", "mp", "quality", "variants"],
                    help="step: the metric line; batch: the 64-instance mix in one persistent launch; serve: "
                         "Poisson request stream through submit/poll; mp: the rotating-bump moving-mesh loop; "
                         "quality: five-ring mesh quality R against the single-domain mesh; variants: MkP / (MP)l")
    ap.add_argument("--mp-steps", type=int, default=50, help="mesh steps of the mp mode")
    ap.add_argument("--quality-subs", default="2,3,4", help="subdomains per axis of the quality mode")
    ap.add_argument("--quality-K", default="1", help="path substeps per mesh step of the quality mode")
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
    ap.add_argument("--requests", type=int, default=40, help="measured requests of the serve mode")
    ap.add_argument("--serve-warmup", type=int, default=4, help="requests before the measured ones (serve mode)")
    ap.add_argument("--fp64-requests", type=int, default=0,
                    help="serve mode, FP64 leg: measured requests (0: as --requests)")
    ap.add_argument("--fp64-warmup", type=int, default=-1,
                    help="serve mode, FP64 leg: warm-up requests (-1: as --serve-warmup)")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="arrival rate in req/s for serve mode (0: 0.7 x the measured capacity)")
    ap.add_argument("--capacity", type=float, default=0.0,
                    help="serve mode: capacity in nominal path-steps/s behind the 0.7 x rate (0: measure it with "
                         "one batched launch of the mix at 1/20 of its path counts)")
    ap.add_argument("--serve-sizes", default="33,65,129,257,513", help="grid sizes of the serving mix")
    ap.add_argument("--serve-max-paths", type=int, default=1_000_000, help="cap on a request's paths per node")
    ap.add_argument("--serve-precision", default="fp32", choices=["fp32", "fp64", "both"])
    ap.add_argument("--serve-requests", type=int, default=24,
                    help="step mode: measured FP32 requests of its serving run (FP64: a third of them)")
    ap.add_argument("--budget-mb", type=int, default=0, help="HBM budget of the serving context (0: 90%% free)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (--gpus %d requested); "
              "see the design notes for how the work would shard" % args.gpus, file=sys.stderr)
        sys.exit(2)
    runners = {"step": run_step, "batch": run_batch, "serve": run_serve, "mp": run_mp, "quality": run_quality,
               "variants": run_variants}
    return runners[args.mode](args)


def node_diff(a, b, n_paths):
    """Per-node differences of two result dicts (all nodes): max |d mean|
    per component, max |d se|, max exit-count difference, and the largest
    |d mean| in units of the combined standard error."""
    import numpy as np
    dx = np.abs(a["mean_x"] - b["mean_x"])
    dy = np.abs(a["mean_y"] - b["mean_y"])
    dse = np.maximum(np.abs(a["se_x"] - b["se_x"]), np.abs(a["se_y"] - b["se_y"]))
    flips = np.rint(np.abs(a["exit_frac"] - b["exit_frac"]) * n_paths)
    sx = np.hypot(a["se_x"], b["se_x"])
    sy = np.hypot(a["se_y"], b["se_y"])
    z = np.maximum(dx / np.maximum(sx, 1e-300), dy / np.maximum(sy, 1e-300))
    return {"nodes": int(len(dx)), "max_abs_dmean_x": float(dx.max()), "max_abs_dmean_y": float(dy.max()),
            "max_abs_dse": float(dse.max()), "nodes_within_1e-5": int(np.sum(np.maximum(dx, dy) <= 1e-5)),
            "max_exit_count_diff": int(flips.max()), "nodes_with_exit_diff": int(np.sum(flips > 0)),
            "max_z_combined_se": float(z.max())}


def run_step(args):
    import numpy as np
    import torch

    from paper_1504_00084_amd import mesh_sdd as M
    from paper_1504_00084_amd import workloads as W

    M.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    inst = W.config3(n_paths=args.paths) if args.workload == "front257" else W.config2(n_paths=args.paths)
    log("workload %s: grid %dx%d, %dx%d subdomains, periodic (%d, %d), N=%d, K=%d, tau=%g"
        % (inst.name, inst.n_xi, inst.n_eta, inst.sub_xi, inst.sub_eta, inst.periodic_xi, inst.periodic_eta,
           inst.n_paths, inst.K, inst.tau))

    with torch.cuda.stream(stream):
        rho, x, y, b0, b1 = (torch.from_numpy(np.ascontiguousarray(a)).to(dev)
                             for a in (inst.rho, inst.x, inst.y, inst.bnd_t0, inst.bnd_t1))
    stream.synchronize()
    if args.copy_mb:
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("plain copy: %d MiB read, %d MiB written" % (args.copy_mb, args.copy_mb))
        del src, dst
    ctx = new_ctx(M, 0, stream.cuda_stream, args.tune_cache)
    h32 = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
    m = M.mesh_sdd_num_interface_nodes(h32)
    outs = [torch.empty(m, dtype=torch.float64, device=dev) for _ in range(5)]
    res = M.make_result(*outs)
    step = M.make_step(x, y, b0, b1, paths_per_node=inst.n_paths, mesh_step=inst.mesh_step)

    M.mesh_sdd_set_monitor(h32, rho)
    if args.launch:
        bl, wv, ch = (int(v) for v in args.launch.split(","))
        M.mesh_sdd_set_launch(ctx, M.make_launch(bl, wv, ch))
    elif args.tune:
        t = time.time()
        lo = M.mesh_sdd_autotune(h32, step)
        log("autotune: %s (%.1f s)" % (lo.as_dict(), time.time() - t))
    lo = M.mesh_sdd_get_launch(h32)
    log("launch shape: %s" % lo.as_dict())

    def one_step():
        M.mesh_sdd_set_monitor(h32, rho)        # a0: table of the frozen monitor
        M.mesh_sdd_solve_interfaces(h32, step, res)
        return int(res.executed_path_steps), float(res.device_ms)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    executed, kernel_ms = 0, []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e, k = one_step()
        executed += e
        kernel_ms.append(k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rate = executed / wall
    ms_per_step = 1e3 * wall / args.steps
    nominal = m * inst.n_paths * inst.K
    g32 = {k: a.cpu().numpy() for k, a in zip(("mean_x", "mean_y", "se_x", "se_y", "exit_frac"), outs)}
    se_max = float(np.max(np.maximum(g32["se_x"], g32["se_y"])))
    kern_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    log("fp32 batched: %.3e path-steps/s (%.1f ms/step, path kernel %.1f ms avg), executed %.3e of nominal %.3e "
        "per step, max SE %.2e" % (rate, ms_per_step, 1e3 * kern_s, executed / args.steps, nominal, se_max))

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
        g64 = {k: a.cpu().numpy() for k, a in zip(("mean_x", "mean_y", "se_x", "se_y", "exit_frac"), outs64)}
        fp64 = {"value": res64.executed_path_steps / w64, "ms_per_step": 1e3 * w64, "kernel_ms": res64.device_ms,
                "executed_path_steps": int(res64.executed_path_steps),
                "fp32_speedup_at_equal_se": w64 / (ms_per_step / 1e3),
                "fp32_vs_fp64_per_node": node_diff(g32, g64, inst.n_paths)}
        log("fp64 plain: %.3e path-steps/s (%.1f ms); fp32 vs fp64 per node: %s"
            % (fp64["value"], fp64["ms_per_step"], fp64["fp32_vs_fp64_per_node"]))
        M.mesh_sdd_destroy(h64)

    per_launch = executed / args.steps
    W_inst = w_slots(inst.periodic_xi, inst.periodic_eta)
    achieved = W_inst * per_launch / kern_s / 1e12
    kernel = {0: "paths_fp32 (cell records)",
              2: "paths_fp32 (LDS table: rho + dt rho_xi; 1024 threads x 1 workgroup per CU)",
              3: "paths_fp32_win<%d> (LDS windows; 1024 threads x 1 workgroup per CU)"
                 % (inst.periodic_xi + 2 * inst.periodic_eta)}[lo.table_level]
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 3), "unit": "TOP/s",
                "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": recorded_traffic(inst.name),
                "kernel": kernel, "kernel_ms": round(kern_s * 1e3, 3), "path_steps_per_launch": per_launch,
                "slots_per_path_step": W_inst}
    M.mesh_sdd_destroy(h32)
    M.mesh_sdd_ctx_destroy(ctx)

    mix = None if args.no_mix else batch_measure(1.0, 64, "", device_inputs=True, tune_cache=args.tune_cache)
    serving = None
    if not args.no_serve:
        cap32 = mix["nominal_path_steps"] / mix["wall_s"] if mix else rate * nominal / max(per_launch, 1.0)
        serving = {"fp32": serve_measure(args.serve_requests, 2, "fp32", [int(v) for v in args.serve_sizes.split(",")],
                                         args.serve_max_paths, capacity=cap32, quiet=True)}
        if fp64:
            cap64 = fp64["value"] * nominal / max(fp64["executed_path_steps"], 1)
            serving["fp64"] = serve_measure(max(4, args.serve_requests // 3), 1, "fp64",
                                            [int(v) for v in args.serve_sizes.split(",")], args.serve_max_paths,
                                            capacity=cap64, quiet=True)
        for k, s in serving.items():
            log("serving %s: %d requests at %.3f req/s: p50 %.1f ms, p99 %.1f ms, %.3e path-steps/s"
                % (k, s["requests"], s["rate_req_s"], s["p50_ms"], s["p99_ms"], s["throughput_path_steps_s"]))

    cpu, parity = (None, None) if args.no_cpu else cpu_baseline_and_parity(inst.name, args.jsonl)

    line = {
        "metric": "interface-node path-steps/sec at 1 GPU (FP32 batched vs FP64 plain) at sigma<=1e-3; p99 latency",
        "value": rate, "unit": "path-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (paths) / f64 (sums)", "data": "synthetic",
        "config": {"workload": inst.name, "grid": [inst.n_xi, inst.n_eta], "subdomains": [inst.sub_xi, inst.sub_eta],
                   "periodic": [inst.periodic_xi, inst.periodic_eta], "interface_nodes": m,
                   "paths_per_node": inst.n_paths, "K": inst.K, "tau": inst.tau, "nominal_path_steps": nominal,
                   "executed_path_steps_per_step": per_launch, "max_se": se_max,
                   "launch": dict(lo.as_dict(), tune_source=tune_source(args.tune_cache, args.tune))},
        "fp64_plain": fp64,
        "roofline": roofline,
        "batched_mix": mix,
        "serving": serving,
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
    }
    print(json.dumps(line), flush=True)


def tune_source(tune_cache, tuned_now=False):
    if tuned_now:
        return "autotuned in this run"
    path = TUNE_CACHE if tune_cache is None else tune_cache
    return os.path.relpath(path, ROOT) if path and os.path.exists(path) else "library defaults"


def batch_measure(scale: float, count: int, sizes: str, device_inputs: bool = True, launch: str = "",
                  label: str = "batched mix", tune_cache=None, tune: bool = False, tune_save: str = "") -> dict:
    """The batched mix: independent instances (grids 33..513, 2x2..16x16
    subdomains, bump or periodic front, 1e4..1e6 paths) in ONE persistent
    FP32 launch through mesh_sdd_solve_batch; inputs resident on the device.
    Its roofline weighs each instance's executed path-steps by its W."""
    import numpy as np
    import torch

    from paper_1504_00084_amd import mesh_sdd as M
    from paper_1504_00084_amd import workloads as W

    M.load()
    insts = W.config4(count=count)
    if sizes:
        keep = {int(v) for v in sizes.split(",")}
        insts = [it for it in insts if it.n_xi in keep]
    if scale != 1.0:
        for it in insts:
            it.n_paths = max(64, int(it.n_paths * scale) // 64 * 64)
    dev = torch.device("cuda:0")
    ctx = new_ctx(M, 0, None, "" if tune else tune_cache)
    if launch:
        bl, wv, ch = (int(v) for v in launch.split(","))
        M.mesh_sdd_set_launch(ctx, M.make_launch(bl, wv, ch))
    hs, ms, steps, results, arrs, keep_alive = [], [], [], [], [], []
    for it in insts:
        h = M.mesh_sdd_create(ctx, M.desc_for(it, M.FP32))
        M.mesh_sdd_set_monitor(h, it.rho)
        m = M.mesh_sdd_num_interface_nodes(h)
        a, r = M.host_result(m)
        hs.append(h)
        ms.append(m)
        arrs.append(a)
        results.append(r)
        src = [it.x, it.y, it.bnd_t0, it.bnd_t1]
        if device_inputs:
            src = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in src]
            keep_alive.append(src)
        steps.append(M.make_step(*src, paths_per_node=it.n_paths))
    nominal = sum(m * it.n_paths * it.K for m, it in zip(ms, insts))
    log("%s: %d instances, %d interface nodes, nominal %.3e path-steps" % (label, len(insts), sum(ms), nominal))
    untuned = None
    if tune:
        # the library's default shapes first, then the autotuned ones
        torch.cuda.synchronize()
        t = time.perf_counter()
        M.mesh_sdd_solve_batch(hs, steps, results)
        w0 = time.perf_counter() - t
        untuned = {"kernel_ms": results[0].device_ms, "wall_s": w0,
                   "executed_path_steps": sum(int(r.executed_path_steps) for r in results)}
        log("%s, default shapes: kernel %.1f ms" % (label, untuned["kernel_ms"]))
        t = time.perf_counter()
        lo = M.mesh_sdd_autotune_batch(hs, steps, scale_down=50)
        untuned["tuning_s"] = time.perf_counter() - t
        log("autotuned batch (%.1f s): %s" % (untuned["tuning_s"], lo.as_dict()))
        if tune_save:
            M.mesh_sdd_tune_save(ctx, tune_save)
    shapes = {}
    for it, h in zip(insts, hs):
        key = "%d%s" % (it.n_xi, "p" if it.periodic_xi else "")
        if key not in shapes:
            shapes[key] = M.mesh_sdd_get_launch(h).as_dict()
    torch.cuda.synchronize()
    t = time.perf_counter()
    M.mesh_sdd_solve_batch(hs, steps, results)
    wall = time.perf_counter() - t
    executed = sum(int(r.executed_path_steps) for r in results)
    kernel_ms = results[0].device_ms
    slots = sum(w_slots(it.periodic_xi, it.periodic_eta) * int(r.executed_path_steps) for it, r in zip(insts, results))
    se = max(float(np.max(np.maximum(a[2][:m], a[3][:m]))) for a, m in zip(arrs, ms) if m)
    frac = slots / (kernel_ms / 1e3) / 1e12 / VALU_PEAK_TOPS
    by_size = {}
    for it, m, r in zip(insts, ms, results):
        d = by_size.setdefault(str(it.n_xi), {"instances": 0, "executed_path_steps": 0})
        d["instances"] += 1
        d["executed_path_steps"] += int(r.executed_path_steps)
    out = {"value": executed / wall, "unit": "path-steps/s", "kernel": "paths_fp32_win<-1> (one launch)",
           "kernel_ms": kernel_ms, "wall_s": wall, "executed_path_steps": executed, "nominal_path_steps": nominal,
           "instances": len(insts), "interface_nodes": sum(ms), "max_se": se, "path_scale": scale,
           "sizes": sorted({it.n_xi for it in insts}), "by_size": by_size,
           "roofline": {"bound": "alu", "achieved": round(slots / (kernel_ms / 1e3) / 1e12, 3),
                        "peak": round(VALU_PEAK_TOPS, 3), "unit": "TOP/s", "frac": round(frac, 4),
                        "slots_per_path_step": round(slots / max(executed, 1), 3)},
           "launch_shapes": {"tune_source": tune_source(tune_cache, tune), "per_grid": shapes}}
    if untuned:
        untuned["frac"] = round(frac * kernel_ms / untuned["kernel_ms"], 4)
        out["default_shapes"] = untuned
    log("%s: %.3e path-steps/s (kernel %.1f ms, wall %.2f s), frac %.3f, max SE %.2e"
        % (label, executed / wall, kernel_ms, wall, frac, se))
    for h in hs:
        M.mesh_sdd_destroy(h)
    M.mesh_sdd_ctx_destroy(ctx)
    return out


def run_batch(args):
    line = {"metric": "batched mix path-steps/s (one persistent launch)"}
    line.update(batch_measure(args.batch_scale, args.batch_count, args.batch_sizes, launch=args.launch,
                              tune_cache=args.tune_cache, tune=args.tune, tune_save=args.tune_save))
    line["dtype"] = "f32 (paths) / f64 (sums)"
    line["data"] = "synthetic"
    print(json.dumps(line), flush=True)


def serve_measure(requests: int, warmup: int, precision: str, sizes, max_paths: int, rate: float = 0.0,
                  budget_mb: int = 0, capacity: float = 0.0, launch: str = "", quiet: bool = False,
                  jsonl: str = "") -> dict:
    """Poisson stream of interface-solve requests from the batched mix, with
    a per-request standard-error target (log-uniform in [1e-4, 1e-3]) setting
    N (capped at max_paths); requests are created, frozen and submitted at
    their arrival times by client threads and served by the library's
    continuous-batching scheduler.  The first `warmup` requests are left out
    of the percentiles.  rate = 0: 0.7 x capacity (nominal path-steps/s) over
    the mean nominal work of a request.  Latency = submit to completion."""
    import threading

    import numpy as np

    from paper_1504_00084_amd import mesh_sdd as M
    from paper_1504_00084_amd import workloads as W

    M.load()
    prec = M.FP32 if precision == "fp32" else M.FP64
    stream = W.serving_stream(warmup + requests, rate_hz=1.0, sizes=tuple(sizes),   # unit rate, rescaled below
                              max_paths=max_paths)
    work = []
    for _, it, _ in stream:
        m = len(M.mesh_sdd_desc_interface_nodes(M.desc_for(it))[0])
        work.append(m * it.n_paths * it.K)
    if rate <= 0.0:
        if capacity <= 0.0:
            raise ValueError("serve_measure needs a rate or a measured capacity")
        rate = 0.7 * capacity / float(np.mean(work))
    arrivals = [t / rate for t, _, _ in stream]
    ctx = new_ctx(M, budget_mb << 20)
    if launch:
        bl, wv, ch = (int(v) for v in launch.split(","))
        M.mesh_sdd_set_launch(ctx, M.make_launch(bl, wv, ch))
    log("serve: %d + %d requests at %.3f req/s (%s), mean nominal work %.3e path-steps"
        % (warmup, requests, rate, precision, float(np.mean(work))))
    recs = {}
    rejected = []
    lock = threading.Lock()
    t0 = time.perf_counter()

    def client(k):
        ta = arrivals[k]
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        _, it, se_target = stream[k]
        h = M.mesh_sdd_create(ctx, M.desc_for(it, prec))
        try:
            M.mesh_sdd_set_monitor(h, it.rho)
            m = M.mesh_sdd_num_interface_nodes(h)
            a, r = M.host_result(m)
            step = M.make_step(it.x, it.y, it.bnd_t0, it.bnd_t1, paths_per_node=it.n_paths)
            ts = time.perf_counter()
            try:
                tk = M.mesh_sdd_submit(h, step)
            except M.MeshSddError as e:
                if e.code != M.E_BUDGET:
                    raise
                with lock:   # the request alone needs more device memory than the whole budget
                    rejected.append(k)
                return
            M.mesh_sdd_wait(ctx, tk, r, -1)
            lat = time.perf_counter() - ts
        finally:
            M.mesh_sdd_destroy(h)
        se = float(np.max(np.maximum(a[2][:m], a[3][:m]))) if m else 0.0
        with lock:
            recs[k] = {"request": k, "grid": it.n_xi, "nodes": m, "paths_per_node": it.n_paths,
                       "target_se": se_target, "max_se": se, "executed_path_steps": int(r.executed_path_steps),
                       "latency_ms": 1e3 * lat, "warmup": k < warmup}
            if not quiet:
                log("request %d done: grid %d, %d nodes, N %d, %.3e path-steps, %.1f ms"
                    % (k, it.n_xi, m, it.n_paths, float(r.executed_path_steps), 1e3 * lat))

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
    st = M.mesh_sdd_ctx_stats(ctx)
    M.mesh_sdd_ctx_destroy(ctx)
    if errors:
        raise errors[0]
    meas = [r for r in recs.values() if not r["warmup"]]
    lat = np.array([r["latency_ms"] for r in meas]) if meas else np.zeros(0)
    done = sum(r["executed_path_steps"] for r in recs.values())
    if jsonl:
        with open(jsonl, "a") as f:
            for k in sorted(recs):
                f.write(json.dumps(dict(recs[k], kind="serving_request", precision=precision)) + "\n")
    return {"precision": precision, "requests": len(meas), "warmup_requests": warmup, "rate_req_s": rate,
            "completed": int(st.completed), "failed": int(st.failed), "rejected_over_budget": len(rejected),
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_ms": float(lat.mean()) if len(lat) else None,
            "library_p50_ms": st.p50_ms, "library_p99_ms": st.p99_ms,
            "throughput_path_steps_s": done / wall, "busy_ms": st.busy_ms, "wall_s": wall, "ticks": int(st.ticks),
            "sizes": list(sizes), "max_paths": max_paths, "se_target_range": [1e-4, 1e-3],
            "max_se_over_target": max((r["max_se"] / r["target_se"] for r in meas), default=None),
            "budget_mb": budget_mb or None}


def fp64_capacity(count: int = 8, scale: float = 0.02) -> float:
    """Nominal path-steps/s of the FP64 plain path (one launch per instance)
    on the mix's first `count` instances at `scale` of their path counts,
    solved one after the other as the serving scheduler runs FP64 work."""
    from paper_1504_00084_amd import mesh_sdd as M
    from paper_1504_00084_amd import workloads as W

    M.load()
    insts = W.config4(count=64)[:count]
    ctx = new_ctx(M, 0)
    nominal = 0
    t = time.perf_counter()
    for it in insts:
        n = max(64, int(it.n_paths * scale) // 64 * 64)
        r = M.solve_instance(ctx, it, M.FP64, n_paths=n)
        nominal += len(r["mean_x"]) * n * it.K
    wall = time.perf_counter() - t
    M.mesh_sdd_ctx_destroy(ctx)
    log("fp64 capacity probe: %d instances at %.2f of their paths, %.3e nominal path-steps/s"
        % (len(insts), scale, nominal / wall))
    return nominal / wall


def run_serve(args):
    sizes = [int(v) for v in args.serve_sizes.split(",")]
    precs = ["fp32", "fp64"] if args.serve_precision == "both" else [args.serve_precision]
    caps = {}
    for p in precs:   # measured capacities behind the 0.7 x rates (unless given)
        if args.rate > 0.0 or args.capacity > 0.0:
            caps[p] = args.capacity
        elif p == "fp32":
            m = batch_measure(0.05, 64, "", label="capacity probe (mix at 1/20 of its paths)")
            caps[p] = m["nominal_path_steps"] / m["wall_s"]
        else:
            caps[p] = fp64_capacity()
    line = {"metric": "serving p50/p99 latency and throughput (Poisson stream of the batched mix)"}
    for p in precs:
        n_req = args.requests if p == "fp32" or args.fp64_requests <= 0 else args.fp64_requests
        n_warm = args.serve_warmup if p == "fp32" or args.fp64_warmup < 0 else args.fp64_warmup
        line[p] = serve_measure(n_req, n_warm, p, sizes, args.serve_max_paths, args.rate,
                                args.budget_mb, capacity=caps[p], launch=args.launch, jsonl=args.jsonl)
        s = line[p]
        line[p]["capacity_nominal_path_steps_s"] = caps[p]
        log("serving %s: %d requests at %.3f req/s: p50 %.1f ms, p99 %.1f ms, %.3e path-steps/s"
            % (p, s["requests"], s["rate_req_s"], s["p50_ms"], s["p99_ms"], s["throughput_path_steps_s"]))
    line["data"] = "synthetic"
    print(json.dumps(line), flush=True)


def cpu_baseline_and_parity(headline: str, jsonl: str = ""):
    """The FP64 CPU oracle on a bounded sample of every workload -- the
    33^2 bump at its full 1e4 paths, the 129^2 bump and the 257^2 front at
    1e3 paths per node, the mix's first four instances at 128 paths, every
    interface node each -- timed on the host cores this process may use;
    and the GPU kernels on the same samples (same inputs, N and streams),
    compared node by node with it.  cpu_baseline.value is the headline
    workload's oracle rate."""
    import numpy as np

    import oracle
    from paper_1504_00084_amd import mesh_sdd as M
    from paper_1504_00084_amd import workloads as W

    threads, info = host_threads()
    log("cpu oracle on %d threads (%s)" % (threads, info))
    samples = [("bump33_2x1", [W.config1()], 10_000), ("rotbump129_4x4", [W.config2(n_paths=1000)], 1000),
               ("front257_8x8_perx", [W.config3(n_paths=1000)], 1000)]
    mix4 = W.config4(count=64)[:4]
    for it in mix4:
        it.n_paths = 128
    samples.append(("mix_first4", mix4, 128))
    rates, parity = {}, {}
    ctx = M.mesh_sdd_ctx_create(0)
    for name, insts, N in samples:
        t = time.perf_counter()
        ora = []
        steps = 0
        for it in insts:
            P = oracle.Problem(**it.problem_kwargs())
            o = oracle.solve(P, it.rho, it.x, it.y, it.bnd_t0, it.bnd_t1, N, threads=threads)
            steps += int(np.sum(o["steps"]))
            ora.append(o)
        cw = time.perf_counter() - t
        nodes = sum(len(o["mean_x"]) for o in ora)
        rates[name] = {"value": steps / cw, "seconds": cw, "path_steps": steps, "nodes": nodes, "paths_per_node": N}
        log("cpu oracle %s: %.3e path-steps/s (%d nodes x %d paths, %.1f s)" % (name, steps / cw, nodes, N, cw))
        # the GPU kernels on the same sample: FP32 batched (all instances in
        # one launch) and, for the 33^2 bump, FP64 plain
        hs, res, arrs = [], [], []
        for it in insts:
            h = M.mesh_sdd_create(ctx, M.desc_for(it, M.FP32))
            M.mesh_sdd_set_monitor(h, it.rho)
            a, r = M.host_result(M.mesh_sdd_num_interface_nodes(h))
            hs.append(h)
            res.append(r)
            arrs.append(a)
        M.mesh_sdd_solve_batch(hs, [M.make_step(it.x, it.y, it.bnd_t0, it.bnd_t1, paths_per_node=N,
                                                mesh_step=it.mesh_step) for it in insts], res)
        g = {k: np.concatenate([a[q][:len(o["mean_x"])] for a, o in zip(arrs, ora)])
             for q, k in enumerate(("mean_x", "mean_y", "se_x", "se_y", "exit_frac"))}
        o_all = {k: np.concatenate([o[k] for o in ora]) for k in ("mean_x", "mean_y", "se_x", "se_y", "exit_frac")}
        for h in hs:
            M.mesh_sdd_destroy(h)
        parity[name] = {"fp32": node_diff(g, o_all, N)}
        if name == "bump33_2x1":
            g64 = M.solve_instance(ctx, insts[0], M.FP64, n_paths=N)
            parity[name]["fp64"] = node_diff(g64, o_all, N)
        log("gpu vs oracle %s: %s" % (name, parity[name]))
        if jsonl:
            with open(jsonl, "a") as f:
                for k in range(len(g["mean_x"])):
                    f.write(json.dumps({"kind": "node_parity", "workload": name, "paths_per_node": N, "node": k,
                                        "gpu_fp32_mean_x": float(g["mean_x"][k]),
                                        "gpu_fp32_mean_y": float(g["mean_y"][k]),
                                        "oracle_mean_x": float(o_all["mean_x"][k]),
                                        "oracle_mean_y": float(o_all["mean_y"][k]),
                                        "abs_dmean": float(max(abs(g["mean_x"][k] - o_all["mean_x"][k]),
                                                               abs(g["mean_y"][k] - o_all["mean_y"][k]))),
                                        "oracle_se_x": float(o_all["se_x"][k]),
                                        "oracle_se_y": float(o_all["se_y"][k])}) + "\n")
    M.mesh_sdd_ctx_destroy(ctx)
    head = rates.get(headline, rates["front257_8x8_perx"])
    total_s = sum(r["seconds"] for r in rates.values())
    cpu = {"value": head["value"], "unit": "path-steps/s", "cores": threads, "kind": "oracle",
           "sample": "%s: all %d interface nodes x %d paths (%.1f s); all samples: %s (%.1f s of oracle work "
                     "in total)" % (headline, head["nodes"], head["paths_per_node"], head["seconds"],
                                    ", ".join("%s %d nodes x %d" % (k, r["nodes"], r["paths_per_node"])
                                              for k, r in rates.items()), total_s),
           "host": info, "per_workload": rates}
    return cpu, parity


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
    alpha = 0.2, R = 30, on [-1, 1[^2 (the computational square the same
    [-1, 1[^2, so 1.25e-4 per step in unit-square time); the decomposed mesh
    against the single-domain mesh, R_max and R_mean of R = Q_SD / Q_SDD.
    41 nodes per axis (40 distinct) for 2x2 and 4x4; 43 for 3x3 (40 is not a
    multiple of 3)."""
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
