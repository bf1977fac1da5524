"""Thin ctypes binding of libmesh_sdd.so (the C-ABI of include/mesh_sdd.h).

Argument marshalling only: every step of the interface solve runs in the
library's HIP kernels.  Functions keep the C names; a non-OK status raises
:class:`MeshSddError` (PENDING is returned as ``False`` by poll/wait).
Arrays may be numpy arrays (host memory) or torch CUDA tensors (device
memory; passed by ``data_ptr()``).  The library must have been built
(``python -m paper_1504_00084_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmesh_sdd.so")

OK, PENDING = 0, 1
E_INVAL, E_NOMEM, E_BUDGET, E_DEVICE, E_STATE, E_CANCELLED = -1, -2, -3, -4, -5, -6
FP32, FP64 = 0, 1
_NAMES = {OK: "OK", PENDING: "PENDING", E_INVAL: "E_INVAL", E_NOMEM: "E_NOMEM", E_BUDGET: "E_BUDGET",
          E_DEVICE: "E_DEVICE", E_STATE: "E_STATE", E_CANCELLED: "E_CANCELLED"}

# every symbol include/mesh_sdd.h declares
EXPORTS = (
    "mesh_sdd_ctx_create", "mesh_sdd_ctx_destroy", "mesh_sdd_ctx_stats", "mesh_sdd_set_launch",
    "mesh_sdd_get_launch", "mesh_sdd_autotune", "mesh_sdd_create", "mesh_sdd_destroy", "mesh_sdd_set_monitor",
    "mesh_sdd_num_interface_nodes", "mesh_sdd_interface_nodes", "mesh_sdd_solve_interfaces",
    "mesh_sdd_solve_batch", "mesh_sdd_submit", "mesh_sdd_poll", "mesh_sdd_wait", "mesh_sdd_cancel",
    "mesh_sdd_debug_paths", "mesh_sdd_last_error", "mesh_sdd_version", "mesh_sdd_desc_check",
    "mesh_sdd_desc_interface_nodes", "mesh_sdd_edge_generate", "mesh_sdd_subdomain_solve",
    "mesh_sdd_single_domain_solve", "mesh_sdd_mp_step", "mesh_sdd_set_monitor_arclength", "mesh_sdd_get_monitor",
    "mesh_sdd_mesh_quality", "mesh_sdd_transfer_field", "mesh_sdd_desc_work_order",
    "mesh_sdd_solve_interfaces_noalloc", "mesh_sdd_autotune_batch", "mesh_sdd_tune_save", "mesh_sdd_tune_load",
)


class MeshSddError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "?"), code, message))
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n_xi", ctypes.c_int32), ("n_eta", ctypes.c_int32),
                ("sub_xi", ctypes.c_int32), ("sub_eta", ctypes.c_int32), ("periodic_xi", ctypes.c_int32),
                ("periodic_eta", ctypes.c_int32), ("K", ctypes.c_int32), ("Lx", ctypes.c_double),
                ("Ly", ctypes.c_double), ("tau", ctypes.c_double), ("precision", ctypes.c_int32),
                ("bridge", ctypes.c_int32), ("seed", ctypes.c_uint64), ("instance_id", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class Step(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("inputs_on_device", ctypes.c_int32),
                ("x_cur", ctypes.c_void_p), ("y_cur", ctypes.c_void_p), ("bnd_t0", ctypes.c_void_p),
                ("bnd_t1", ctypes.c_void_p), ("paths_per_node", ctypes.c_int64), ("target_se", ctypes.c_double),
                ("max_paths", ctypes.c_int64), ("mesh_step", ctypes.c_uint32),
                ("interface_stride", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("outputs_on_device", ctypes.c_int32),
                ("mean_x", ctypes.c_void_p), ("mean_y", ctypes.c_void_p), ("se_x", ctypes.c_void_p),
                ("se_y", ctypes.c_void_p), ("exit_frac", ctypes.c_void_p),
                ("executed_path_steps", ctypes.c_uint64), ("paths_per_node", ctypes.c_int64),
                ("device_ms", ctypes.c_double)]


class MpOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("fe_substeps", ctypes.c_int32), ("edge_substeps", ctypes.c_int32),
                ("edge_generator", ctypes.c_int32), ("solver", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("fe_cfl", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("submitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64), ("cancelled", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("running", ctypes.c_uint64), ("ticks", ctypes.c_uint64),
                ("hbm_in_use", ctypes.c_uint64), ("hbm_budget", ctypes.c_uint64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double), ("busy_ms", ctypes.c_double),
                ("executed_path_steps", ctypes.c_uint64)]


class Launch(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("block", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("chunk_paths", ctypes.c_int32), ("monitor_table", ctypes.c_int32), ("table_level", ctypes.c_int32),
                ("refill_lanes", ctypes.c_int32), ("max_quarters", ctypes.c_int32), ("window_kind", ctypes.c_int32),
                ("window_margin", ctypes.c_int32), ("job_split", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "struct_size"}


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libmesh_sdd.so not found at %s; build it with "
                           "`python -m paper_1504_00084_amd.build`" % path)
    # torch ships its own HIP runtime; loading it first makes the library bind
    # to that same runtime, so device pointers and streams from torch tensors
    # are valid inside the library (two runtimes in one process see no device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, i64, sz, P = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.POINTER
    sig = {
        "mesh_sdd_ctx_create": [ctypes.c_int, sz, vp, P(vp)],
        "mesh_sdd_ctx_destroy": [vp],
        "mesh_sdd_ctx_stats": [vp, P(Stats)],
        "mesh_sdd_set_launch": [vp, P(Launch)],
        "mesh_sdd_get_launch": [vp, P(Launch)],
        "mesh_sdd_autotune": [vp, P(Step), P(Launch)],
        "mesh_sdd_autotune_batch": [P(vp), P(Step), i32, i32, P(Launch)],
        "mesh_sdd_tune_save": [vp, ctypes.c_char_p],
        "mesh_sdd_tune_load": [vp, ctypes.c_char_p],
        "mesh_sdd_create": [vp, P(Desc), P(vp)],
        "mesh_sdd_destroy": [vp],
        "mesh_sdd_set_monitor": [vp, vp, ctypes.c_int],
        "mesh_sdd_num_interface_nodes": [vp],
        "mesh_sdd_interface_nodes": [vp, vp, vp],
        "mesh_sdd_solve_interfaces": [vp, P(Step), P(Result)],
        "mesh_sdd_solve_interfaces_noalloc": [vp, P(Step), P(Result)],
        "mesh_sdd_solve_batch": [P(vp), P(Step), P(Result), i32, P(i32)],
        "mesh_sdd_submit": [vp, P(Step), P(ctypes.c_uint64)],
        "mesh_sdd_poll": [vp, ctypes.c_uint64, P(Result)],
        "mesh_sdd_wait": [vp, ctypes.c_uint64, P(Result), i64],
        "mesh_sdd_cancel": [vp, ctypes.c_uint64],
        "mesh_sdd_debug_paths": [vp, P(Step), i32, i64, i64, vp, vp, vp, vp, vp, vp],
        "mesh_sdd_desc_check": [P(Desc)],
        "mesh_sdd_desc_interface_nodes": [P(Desc), vp, vp],
        "mesh_sdd_desc_work_order": [P(Desc), ctypes.c_uint32, vp, vp, ctypes.c_int32, P(ctypes.c_int32)],
        "mesh_sdd_last_error": [],
        "mesh_sdd_version": [],
        "mesh_sdd_edge_generate": [vp, vp, vp, P(MpOpts), ctypes.c_int],
        "mesh_sdd_subdomain_solve": [vp, vp, vp, vp, vp, vp, vp, vp, P(MpOpts), ctypes.c_int],
        "mesh_sdd_single_domain_solve": [vp, vp, vp, vp, vp, vp, P(MpOpts), ctypes.c_int],
        "mesh_sdd_mp_step": [vp, P(Step), P(MpOpts), vp, vp, vp, P(Result)],
        "mesh_sdd_set_monitor_arclength": [vp, vp, vp, vp, ctypes.c_double, ctypes.c_int, ctypes.c_int],
        "mesh_sdd_get_monitor": [vp, vp, ctypes.c_int],
        "mesh_sdd_transfer_field": [vp, vp, vp, vp, vp, vp, vp, ctypes.c_int],
        "mesh_sdd_mesh_quality": [vp, vp, vp, vp, vp, vp, P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.mesh_sdd_last_error.restype = ctypes.c_char_p
    lib.mesh_sdd_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        raise MeshSddError(rc, load().mesh_sdd_last_error().decode())
    return rc


# --------------------------------------------------------------------------
# pointer marshalling
# --------------------------------------------------------------------------
def _is_torch_cuda(a) -> bool:
    return hasattr(a, "is_cuda") and bool(a.is_cuda)


def _ptr(a, dtype=np.float64):
    """(address, on_device) of a contiguous array of `dtype`."""
    if a is None:
        return None, False
    if _is_torch_cuda(a):
        if not a.is_contiguous():
            raise ValueError("device tensor must be contiguous")
        return a.data_ptr(), True
    if not isinstance(a, np.ndarray) or a.dtype != dtype or not a.flags["C_CONTIGUOUS"]:
        raise ValueError("host array must be a C-contiguous numpy array of %s" % np.dtype(dtype))
    return a.ctypes.data, False


# --------------------------------------------------------------------------
# C-ABI functions (same names)
# --------------------------------------------------------------------------
def mesh_sdd_version() -> str:
    return load().mesh_sdd_version().decode()


def mesh_sdd_last_error() -> str:
    return load().mesh_sdd_last_error().decode()


def mesh_sdd_ctx_create(device: int = 0, hbm_budget_bytes: int = 0, hip_stream: int | None = None):
    out = ctypes.c_void_p()
    _check(load().mesh_sdd_ctx_create(device, hbm_budget_bytes, hip_stream or None, ctypes.byref(out)))
    return out.value


def mesh_sdd_ctx_destroy(ctx) -> None:
    _check(load().mesh_sdd_ctx_destroy(ctx))


def mesh_sdd_ctx_stats(ctx) -> Stats:
    s = Stats(struct_size=ctypes.sizeof(Stats))
    _check(load().mesh_sdd_ctx_stats(ctx, ctypes.byref(s)))
    return s


def mesh_sdd_set_launch(ctx, launch: Launch | None) -> None:
    _check(load().mesh_sdd_set_launch(ctx, ctypes.byref(launch) if launch is not None else None))


def mesh_sdd_get_launch(inst) -> Launch:
    lo = Launch(struct_size=ctypes.sizeof(Launch))
    _check(load().mesh_sdd_get_launch(inst, ctypes.byref(lo)))
    return lo


def make_launch(block=256, waves_per_simd=3, chunk_paths=128, monitor_table=0, refill_lanes=0, max_quarters=0,
                window_kind=0, window_margin=0, job_split=0) -> Launch:
    """Launch shape; 0 in the last five fields means the library's default."""
    return Launch(ctypes.sizeof(Launch), block, waves_per_simd, chunk_paths, monitor_table, 0, refill_lanes,
                  max_quarters, window_kind, window_margin, job_split)


def mesh_sdd_autotune(inst, step: Step) -> Launch:
    lo = Launch(struct_size=ctypes.sizeof(Launch))
    _check(load().mesh_sdd_autotune(inst, ctypes.byref(step), ctypes.byref(lo)))
    return lo


def mesh_sdd_autotune_batch(insts, steps, scale_down: int = 50) -> Launch:
    n = len(insts)
    arr_i = (ctypes.c_void_p * n)(*insts)
    arr_s = (Step * n)(*steps)
    lo = Launch(struct_size=ctypes.sizeof(Launch))
    _check(load().mesh_sdd_autotune_batch(arr_i, arr_s, n, int(scale_down), ctypes.byref(lo)))
    return lo


def mesh_sdd_tune_save(ctx, path: str) -> None:
    _check(load().mesh_sdd_tune_save(ctx, os.fsencode(path)))


def mesh_sdd_tune_load(ctx, path: str) -> None:
    _check(load().mesh_sdd_tune_load(ctx, os.fsencode(path)))


def make_desc(n_xi, n_eta, sub_xi, sub_eta, periodic_xi=0, periodic_eta=0, K=500, Lx=1.0, Ly=1.0, tau=0.01,
              precision=FP32, bridge=1, seed=0, instance_id=0) -> Desc:
    return Desc(ctypes.sizeof(Desc), n_xi, n_eta, sub_xi, sub_eta, periodic_xi, periodic_eta, K, Lx, Ly, tau,
                precision, bridge, seed, instance_id, 0)


def mesh_sdd_desc_check(desc: Desc) -> None:
    _check(load().mesh_sdd_desc_check(ctypes.byref(desc)))


def mesh_sdd_desc_interface_nodes(desc: Desc):
    m = _check(load().mesh_sdd_desc_interface_nodes(ctypes.byref(desc), None, None))
    i = np.empty(max(m, 1), dtype=np.int32)
    j = np.empty(max(m, 1), dtype=np.int32)
    _check(load().mesh_sdd_desc_interface_nodes(ctypes.byref(desc), i.ctypes.data, j.ctypes.data))
    return i[:m], j[:m]


def mesh_sdd_desc_work_order(desc: Desc, interface_stride: int = 0):
    """(ranks in work order, blocks [n_blocks, 7]: first position, end
    position, window i0, j0, width, height, kind)."""
    nb = ctypes.c_int32(0)
    m = _check(load().mesh_sdd_desc_work_order(ctypes.byref(desc), interface_stride, None, None, 0, ctypes.byref(nb)))
    ranks = np.empty(max(m, 1), dtype=np.int32)
    blocks = np.empty((max(nb.value, 1), 7), dtype=np.int32)
    _check(load().mesh_sdd_desc_work_order(ctypes.byref(desc), interface_stride, ranks.ctypes.data,
                                           blocks.ctypes.data, nb.value, ctypes.byref(nb)))
    return ranks[:m], blocks[:nb.value]


def mesh_sdd_create(ctx, desc: Desc):
    out = ctypes.c_void_p()
    _check(load().mesh_sdd_create(ctx, ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def mesh_sdd_destroy(inst) -> None:
    _check(load().mesh_sdd_destroy(inst))


def mesh_sdd_set_monitor(inst, rho) -> None:
    p, dev = _ptr(rho)
    _check(load().mesh_sdd_set_monitor(inst, p, int(dev)))


def mesh_sdd_num_interface_nodes(inst) -> int:
    return _check(load().mesh_sdd_num_interface_nodes(inst))


def mesh_sdd_interface_nodes(inst):
    m = mesh_sdd_num_interface_nodes(inst)
    i = np.empty(max(m, 1), dtype=np.int32)
    j = np.empty(max(m, 1), dtype=np.int32)
    _check(load().mesh_sdd_interface_nodes(inst, i.ctypes.data, j.ctypes.data))
    return i[:m], j[:m]


def make_step(x_cur, y_cur, bnd_t0, bnd_t1, paths_per_node=0, target_se=0.0, max_paths=0, mesh_step=0,
              interface_stride=0) -> Step:
    """Step descriptor; the arrays must stay alive until the call returns.
    interface_stride > 1 runs paths at every stride-th node of each interface
    line only and interpolates the others."""
    px, dx = _ptr(x_cur)
    py, dy = _ptr(y_cur)
    p0, d0 = _ptr(bnd_t0)
    p1, d1 = _ptr(bnd_t1)
    if len({dx, dy, d0, d1}) != 1:
        raise ValueError("step inputs must be all host arrays or all device tensors")
    st = Step(ctypes.sizeof(Step), int(dx), px, py, p0, p1, int(paths_per_node), float(target_se),
              int(max_paths), int(mesh_step), int(interface_stride))
    st._keep = (x_cur, y_cur, bnd_t0, bnd_t1)
    return st


def make_result(mean_x, mean_y, se_x, se_y, exit_frac) -> Result:
    ptrs = [_ptr(a) for a in (mean_x, mean_y, se_x, se_y, exit_frac)]
    devs = {d for p, d in ptrs if p is not None}
    if len(devs) > 1:
        raise ValueError("result arrays must be all host arrays or all device tensors")
    res = Result(ctypes.sizeof(Result), int(devs.pop() if devs else False), *[p for p, _ in ptrs], 0, 0, 0.0)
    res._keep = (mean_x, mean_y, se_x, se_y, exit_frac)
    return res


def mesh_sdd_solve_interfaces(inst, step: Step, result: Result) -> Result:
    _check(load().mesh_sdd_solve_interfaces(inst, ctypes.byref(step), ctypes.byref(result)))
    return result


def mesh_sdd_solve_interfaces_noalloc(inst, step: Step, result: Result) -> Result:
    """The solve with every per-call buffer in the library's static device
    scratch (device inputs and outputs only)."""
    _check(load().mesh_sdd_solve_interfaces_noalloc(inst, ctypes.byref(step), ctypes.byref(result)))
    return result


def mesh_sdd_solve_batch(insts, steps, results):
    n = len(insts)
    arr_i = (ctypes.c_void_p * n)(*insts)
    arr_s = (Step * n)(*steps)
    arr_r = (Result * n)(*results)
    status = (ctypes.c_int32 * n)()
    rc = load().mesh_sdd_solve_batch(arr_i, arr_s, arr_r, n, status)
    for k in range(n):   # copy the output fields back
        results[k].executed_path_steps = arr_r[k].executed_path_steps
        results[k].paths_per_node = arr_r[k].paths_per_node
        results[k].device_ms = arr_r[k].device_ms
    _check(rc)
    return [int(s) for s in status]


def mesh_sdd_submit(inst, step: Step) -> int:
    t = ctypes.c_uint64()
    _check(load().mesh_sdd_submit(inst, ctypes.byref(step), ctypes.byref(t)))
    return t.value


def mesh_sdd_poll(ctx, ticket: int, result: Result | None) -> bool:
    rc = _check(load().mesh_sdd_poll(ctx, ticket, ctypes.byref(result) if result is not None else None))
    return rc == OK


def mesh_sdd_wait(ctx, ticket: int, result: Result | None, timeout_ms: int = -1) -> bool:
    rc = _check(load().mesh_sdd_wait(ctx, ticket, ctypes.byref(result) if result is not None else None, timeout_ms))
    return rc == OK


def mesh_sdd_cancel(ctx, ticket: int) -> None:
    _check(load().mesh_sdd_cancel(ctx, ticket))


def mesh_sdd_debug_paths(inst, step: Step, node_rank: int, p_begin: int, p_end: int, K: int, trace: bool = False):
    n = p_end - p_begin
    vx, vy = np.empty(max(n, 1)), np.empty(max(n, 1))
    ex, sd, st = (np.empty(max(n, 1), dtype=np.int32) for _ in range(3))
    tr = np.full((max(n, 1), K, 4), np.nan) if trace else None
    _check(load().mesh_sdd_debug_paths(inst, ctypes.byref(step), node_rank, p_begin, p_end, vx.ctypes.data,
                                       vy.ctypes.data, ex.ctypes.data, sd.ctypes.data, st.ctypes.data,
                                       tr.ctypes.data if trace else None))
    out = {"vx": vx[:n], "vy": vy[:n], "exited": ex[:n], "side": sd[:n], "steps": st[:n]}
    if trace:
        out["trace"] = tr[:n]
    return out


# --------------------------------------------------------------------------
# small conveniences over the calls above (still marshalling only)
# --------------------------------------------------------------------------
def desc_for(inst, precision=FP32) -> Desc:
    """Descriptor of a workloads.Instance."""
    return make_desc(inst.n_xi, inst.n_eta, inst.sub_xi, inst.sub_eta, inst.periodic_xi, inst.periodic_eta, inst.K,
                     inst.Lx, inst.Ly, inst.tau, precision, inst.bridge, inst.seed, inst.instance_id)


def host_result(m: int):
    arrs = [np.empty(max(m, 1)) for _ in range(5)]
    return arrs, make_result(*arrs)


def result_dict(arrs, res: Result, m: int) -> dict:
    out = {k: np.asarray(a[:m]) for k, a in zip(("mean_x", "mean_y", "se_x", "se_y", "exit_frac"), arrs)}
    out["executed_path_steps"] = int(res.executed_path_steps)
    out["paths_per_node"] = int(res.paths_per_node)
    out["device_ms"] = float(res.device_ms)
    return out


def solve_instance(ctx, inst, precision=FP32, n_paths=None, mesh_step=None):
    """Create, set the monitor, solve one step from host arrays, destroy."""
    h = mesh_sdd_create(ctx, desc_for(inst, precision))
    try:
        mesh_sdd_set_monitor(h, np.ascontiguousarray(inst.rho))
        m = mesh_sdd_num_interface_nodes(h)
        arrs, res = host_result(m)
        st = make_step(np.ascontiguousarray(inst.x), np.ascontiguousarray(inst.y), inst.bnd_t0, inst.bnd_t1,
                       paths_per_node=n_paths or inst.n_paths,
                       mesh_step=inst.mesh_step if mesh_step is None else mesh_step)
        mesh_sdd_solve_interfaces(h, st, res)
        return result_dict(arrs, res, m)
    finally:
        mesh_sdd_destroy(h)


# --------------------------------------------------------------------------
# the mesh step around the interface estimate
# --------------------------------------------------------------------------
def make_mp_opts(fe_substeps=0, edge_substeps=0, edge_generator=1, solver=0, fe_cfl=0.0) -> MpOpts:
    return MpOpts(ctypes.sizeof(MpOpts), int(fe_substeps), int(edge_substeps), int(edge_generator), int(solver), 0,
                  float(fe_cfl))


def _same_kind(*arrays):
    ptrs = [_ptr(a) for a in arrays]
    devs = {d for p, d in ptrs if p is not None}
    if len(devs) > 1:
        raise ValueError("arrays must be all host arrays or all device tensors")
    return [p for p, _ in ptrs], int(devs.pop() if devs else False)


def _opts(opts):
    return ctypes.byref(opts) if opts is not None else None


def mesh_sdd_edge_generate(inst, bnd_cur, bnd_new, opts: MpOpts | None = None) -> None:
    (pc, pn), dev = _same_kind(bnd_cur, bnd_new)
    _check(load().mesh_sdd_edge_generate(inst, pc, pn, _opts(opts), dev))


def mesh_sdd_subdomain_solve(inst, x_cur, y_cur, bnd_new, iface_x, iface_y, x_new, y_new,
                             opts: MpOpts | None = None) -> None:
    ptrs, dev = _same_kind(x_cur, y_cur, bnd_new, iface_x, iface_y, x_new, y_new)
    _check(load().mesh_sdd_subdomain_solve(inst, *ptrs, _opts(opts), dev))


def mesh_sdd_single_domain_solve(inst, x_cur, y_cur, bnd_new, x_new, y_new, opts: MpOpts | None = None) -> None:
    ptrs, dev = _same_kind(x_cur, y_cur, bnd_new, x_new, y_new)
    _check(load().mesh_sdd_single_domain_solve(inst, *ptrs, _opts(opts), dev))


def mesh_sdd_mp_step(inst, step: Step, x_new, y_new, bnd_new, result: Result, opts: MpOpts | None = None) -> Result:
    (px, py, pb), dev = _same_kind(x_new, y_new, bnd_new)
    if dev != result.outputs_on_device and inst is not None:
        raise ValueError("mesh outputs and result arrays must be of the same memory kind")
    _check(load().mesh_sdd_mp_step(inst, ctypes.byref(step), _opts(opts), px, py, pb, ctypes.byref(result)))
    return result


def mesh_sdd_set_monitor_arclength(inst, u, x, y, alpha: float, normalize: bool = False) -> None:
    (pu, px, py), dev = _same_kind(u, x, y)
    _check(load().mesh_sdd_set_monitor_arclength(inst, pu, px, py, float(alpha), int(bool(normalize)), dev))


def mesh_sdd_get_monitor(inst, rho_out) -> None:
    p, dev = _ptr(rho_out)
    _check(load().mesh_sdd_get_monitor(inst, p, int(dev)))


def mesh_sdd_transfer_field(inst, x_old, y_old, f_old, x_new, y_new, f_new) -> None:
    """f_new at the nodes of (x_new, y_new) from the piecewise-linear
    interpolant of f_old on the mesh (x_old, y_old)."""
    ptrs, dev = _same_kind(x_old, y_old, f_old, x_new, y_new, f_new)
    _check(load().mesh_sdd_transfer_field(inst, *ptrs, dev))


def mesh_sdd_mesh_quality(inst, x_sd, y_sd, x_dd, y_dd, r_cells=None):
    """(R_max, R_mean); fills r_cells ([(n_eta-1), (n_xi-1)]) when given."""
    ptrs, dev = _same_kind(x_sd, y_sd, x_dd, y_dd, r_cells)
    rmax, rmean = ctypes.c_double(), ctypes.c_double()
    _check(load().mesh_sdd_mesh_quality(inst, *ptrs, ctypes.byref(rmax), ctypes.byref(rmean), dev))
    return rmax.value, rmean.value

