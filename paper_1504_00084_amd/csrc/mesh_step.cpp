// Host side of the mesh step around the interface estimate (C-ABI of
// include/mesh_sdd.h, section "the mesh step"): the 1-D edge generator
// (section 2), the subdomain solves and the single-domain reference
// (section 3.5), one whole MP mesh step (sections 3.4-3.6), the arc-length
// monitor on the new mesh (section 3.6) and the mesh-quality ratio
// (section 3.7).  The kernels are in mesh_step.hip; the interface estimate
// itself goes through mesh_sdd_solve_interfaces.

#include <cmath>
#include <cstring>
#include <vector>

#include "msdd_mesh_step.hpp"
#include "runtime_internal.hpp"

using namespace msdd_rt;

namespace {

struct MpOpts {
    int fe_L = 0, edge_L = 0, edge_gen = 1, solver = 0;
    double cfl = 0.9;
};

int read_opts(const mesh_sdd_mp_opts *o, MpOpts &m)
{
    m = MpOpts{};
    if (!o) return MESH_SDD_OK;
    if (o->struct_size != sizeof(mesh_sdd_mp_opts))
        return fail(MESH_SDD_E_INVAL, "opts.struct_size %u != %zu", o->struct_size, sizeof(mesh_sdd_mp_opts));
    if (o->reserved != 0) return fail(MESH_SDD_E_INVAL, "opts.reserved must be 0");
    if (o->fe_substeps < 0 || o->edge_substeps < 0) return fail(MESH_SDD_E_INVAL, "substep counts must be >= 0");
    if (o->edge_generator != 0 && o->edge_generator != 1) return fail(MESH_SDD_E_INVAL, "edge_generator must be 0 or 1");
    if (o->solver < 0 || o->solver > 2) return fail(MESH_SDD_E_INVAL, "solver must be 0, 1 or 2");
    if (!(o->fe_cfl >= 0.0 && o->fe_cfl <= 1.0)) return fail(MESH_SDD_E_INVAL, "fe_cfl must be in [0, 1]");
    m.fe_L = o->fe_substeps;
    m.edge_L = o->edge_substeps;
    m.edge_gen = o->edge_generator;
    m.solver = o->solver;
    m.cfl = o->fe_cfl == 0.0 ? 0.9 : o->fe_cfl;
    return MESH_SDD_OK;
}

constexpr double kMaxSubsteps = 1.0e7;

// Smallest forward-Euler step count within cfl x the stability limit.
int substeps_for(double tau, double dt_max, double cfl, int given, int *out)
{
    if (given > 0) {
        *out = given;
        return MESH_SDD_OK;
    }
    const double L = std::ceil(tau / (cfl * dt_max) - 1e-12);
    if (!(L <= kMaxSubsteps)) return fail(MESH_SDD_E_INVAL, "forward Euler would need %.3g substeps", L);
    *out = L < 1.0 ? 1 : (int)L;
    return MESH_SDD_OK;
}

int fe_substeps(const mesh_sdd_desc &d, const MpOpts &o, int *out)
{
    const double hx = 1.0 / (double)(d.n_xi - 1), hy = 1.0 / (double)(d.n_eta - 1);
    return substeps_for(d.tau, 1.0 / (2.0 / (hx * hx) + 2.0 / (hy * hy)), o.cfl, o.fe_L, out);
}

int edge_substeps(int n, double tau, const MpOpts &o, int *out)
{
    const double h = 1.0 / (double)(n - 1);
    return substeps_for(tau, 0.5 * h * h, o.cfl, o.edge_L, out);
}

size_t grid_size(const mesh_sdd_desc &d) { return (size_t)d.n_xi * d.n_eta; }
size_t bnd_size(const mesh_sdd_desc &d) { return 4u * (size_t)d.n_eta + 4u * (size_t)d.n_xi; }

// A device view of an input array: the caller's device pointer, or a pooled
// copy of a host array.
struct DevIn {
    DevBuf buf;
    const double *p = nullptr;
};

int stage_in(mesh_sdd_ctx *ctx, const double *src, size_t n, int on_device, DevIn &in, hipStream_t st)
{
    if (on_device) {
        in.p = src;
        return MESH_SDD_OK;
    }
    in.buf.pool = &ctx->pool;
    if (in.buf.alloc(n * sizeof(double)) != hipSuccess) return fail(MESH_SDD_E_NOMEM, "device staging failed");
    HIP_TRY(hipMemcpyAsync(in.buf.p, src, n * sizeof(double), hipMemcpyHostToDevice, st));
    in.p = in.buf.as<double>();
    return MESH_SDD_OK;
}

// A device view of an output array: the caller's device pointer, or a pooled
// buffer copied to the caller's host array by finish().
struct DevOut {
    DevBuf buf;
    double *p = nullptr;
    double *host = nullptr;
    size_t n = 0;
};

int stage_out(mesh_sdd_ctx *ctx, double *dst, size_t n, int on_device, DevOut &out)
{
    out.n = n;
    if (on_device) {
        out.p = dst;
        return MESH_SDD_OK;
    }
    out.host = dst;
    out.buf.pool = &ctx->pool;
    if (out.buf.alloc(n * sizeof(double)) != hipSuccess) return fail(MESH_SDD_E_NOMEM, "device staging failed");
    out.p = out.buf.as<double>();
    return MESH_SDD_OK;
}

int finish(DevOut &out, hipStream_t st)
{
    if (out.host && out.n) HIP_TRY(hipMemcpyAsync(out.host, out.p, out.n * sizeof(double), hipMemcpyDeviceToHost, st));
    return MESH_SDD_OK;
}

// Waits for the stream when it goes out of scope.  Declared after the
// pooled buffers of a call, so that on every return (errors included) the
// work that uses them has finished before they go back to the pool.
struct SyncOnExit {
    hipStream_t s;
    ~SyncOnExit() { (void)hipStreamSynchronize(s); }
};

// 1-D generator on every physical side, in place on device boundary arrays.
int edge_dev(mesh_sdd *inst, const MpOpts &o, double *bnd, hipStream_t st)
{
    const mesh_sdd_desc &d = inst->d;
    int L_eta = 1, L_xi = 1;
    int rc = edge_substeps(d.n_eta, d.tau, o, &L_eta);
    if (rc == MESH_SDD_OK) rc = edge_substeps(d.n_xi, d.tau, o, &L_xi);
    if (rc != MESH_SDD_OK) return rc;
    const int n_max = std::max(d.n_xi, d.n_eta);
    if (msdd::edge_gen_lds_bytes(n_max) > msdd::kSubLdsMax)
        return fail(MESH_SDD_E_INVAL, "grid too large for the edge generator (n = %d)", n_max);
    HIP_TRY(msdd::launch_edge_gen(inst->rho.as<double>(), inst->rho_xi.as<double>(), inst->rho_eta.as<double>(),
                                  d.n_xi, d.n_eta, d.periodic_xi, d.periodic_eta, d.Lx, d.Ly, d.tau, L_eta, L_xi, bnd,
                                  st));
    return MESH_SDD_OK;
}

// Subdomain solves (with_interfaces) or the single-domain reference, on
// device arrays.  x_new / y_new must not alias x0 / y0.
int solve_dev(mesh_sdd *inst, const MpOpts &o, const double *x0, const double *y0, const double *bnd1,
              const double *ix, const double *iy, bool with_interfaces, double *x_new, double *y_new, hipStream_t st)
{
    const mesh_sdd_desc &d = inst->d;
    mesh_sdd_ctx *ctx = inst->ctx;
    int L = 1;
    int rc = fe_substeps(d, o, &L);
    if (rc != MESH_SDD_OK) return rc;
    const size_t n = grid_size(d);
    DevBuf tx1, ty1, mask, ax, ay, bx, by;
    tx1.pool = ty1.pool = mask.pool = ax.pool = ay.pool = bx.pool = by.pool = &ctx->pool;
    SyncOnExit sync{st};
    if (tx1.alloc(n * 8) || ty1.alloc(n * 8) || mask.alloc(n))
        return fail(MESH_SDD_E_NOMEM, "device allocation for the mesh step failed");
    msdd::MeshStepArgs a{};
    a.n_xi = d.n_xi;
    a.n_eta = d.n_eta;
    a.sub_xi = with_interfaces ? d.sub_xi : 1;
    a.sub_eta = with_interfaces ? d.sub_eta : 1;
    a.P_xi = (d.n_xi - 1) / a.sub_xi;
    a.P_eta = (d.n_eta - 1) / a.sub_eta;
    a.per_xi = d.periodic_xi;
    a.per_eta = d.periodic_eta;
    a.with_interfaces = with_interfaces ? 1 : 0;
    a.L = L;
    a.Lx = d.Lx;
    a.Ly = d.Ly;
    a.tau = d.tau;
    a.x0 = x0;
    a.y0 = y0;
    a.bnd1 = bnd1;
    a.iface_x = ix;
    a.iface_y = iy;
    a.node_rank = inst->node_rank.as<int32_t>();
    a.rho = inst->rho.as<double>();
    a.rho_xi = inst->rho_xi.as<double>();
    a.rho_eta = inst->rho_eta.as<double>();
    a.tx1 = tx1.as<double>();
    a.ty1 = ty1.as<double>();
    a.mask = mask.as<uint8_t>();
    HIP_TRY(msdd::launch_targets(a, x_new, y_new, st));
    const bool fits = msdd::subdomain_fits_lds(a.P_xi, a.P_eta);
    if (with_interfaces && o.solver == 1 && !fits)
        return fail(MESH_SDD_E_INVAL, "a %dx%d subdomain does not fit in LDS", a.P_xi + 1, a.P_eta + 1);
    if (with_interfaces && o.solver != 2 && fits) {
        HIP_TRY(msdd::launch_subdomain_lds(a, x_new, y_new, st));
        return MESH_SDD_OK;
    }
    // whole-grid sweeps: x0 -> A -> B -> A ..., the last level copied out
    if (ax.alloc(n * 8) || ay.alloc(n * 8) || bx.alloc(n * 8) || by.alloc(n * 8))
        return fail(MESH_SDD_E_NOMEM, "device allocation for the mesh step failed");
    const double *cx = x0, *cy = y0;
    double *nx = ax.as<double>(), *ny = ay.as<double>();
    double *ox = bx.as<double>(), *oy = by.as<double>();
    for (int l = 0; l < L; ++l) {
        const double th1 = (double)(l + 1) / (double)L;
        HIP_TRY(msdd::launch_fe_sweep(a, cx, cy, nx, ny, th1, st));
        cx = nx;
        cy = ny;
        std::swap(nx, ox);
        std::swap(ny, oy);
    }
    HIP_TRY(hipMemcpyAsync(x_new, cx, n * 8, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(y_new, cy, n * 8, hipMemcpyDeviceToDevice, st));
    return MESH_SDD_OK;
}

int check_ready(mesh_sdd *inst)
{
    if (!inst) return fail(MESH_SDD_E_INVAL, "instance is NULL");
    if (!inst->monitor_set) return fail(MESH_SDD_E_STATE, "set_monitor has not been called");
    return MESH_SDD_OK;
}

}  // namespace

extern "C" {

int mesh_sdd_edge_generate(mesh_sdd *inst, const double *bnd_cur, double *bnd_new, const mesh_sdd_mp_opts *opts,
                           int pointers_on_device)
try {
    int rc = check_ready(inst);
    if (rc != MESH_SDD_OK) return rc;
    if (!bnd_cur || !bnd_new) return fail(MESH_SDD_E_INVAL, "NULL boundary array");
    MpOpts o;
    if ((rc = read_opts(opts, o)) != MESH_SDD_OK) return rc;
    mesh_sdd_ctx *ctx = inst->ctx;
    const size_t nb = bnd_size(inst->d);
    std::lock_guard<std::mutex> g(ctx->gpu_mu);
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    DevOut out;
    SyncOnExit sync{st};
    if ((rc = stage_out(ctx, bnd_new, nb, pointers_on_device, out)) != MESH_SDD_OK) return rc;
    if (out.p != bnd_cur)
        HIP_TRY(hipMemcpyAsync(out.p, bnd_cur, nb * 8, pointers_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                               st));
    if ((rc = edge_dev(inst, o, out.p, st)) != MESH_SDD_OK) return rc;
    if ((rc = finish(out, st)) != MESH_SDD_OK) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

static int solve_common(mesh_sdd *inst, const double *x_cur, const double *y_cur, const double *bnd_new,
                        const double *iface_x, const double *iface_y, double *x_new, double *y_new,
                        const mesh_sdd_mp_opts *opts, int on_device, bool with_interfaces)
{
    int rc = check_ready(inst);
    if (rc != MESH_SDD_OK) return rc;
    if (!x_cur || !y_cur || !bnd_new || !x_new || !y_new) return fail(MESH_SDD_E_INVAL, "NULL array");
    if (with_interfaces && inst->M > 0 && (!iface_x || !iface_y)) return fail(MESH_SDD_E_INVAL, "NULL interface values");
    if (x_new == x_cur || x_new == y_cur || y_new == x_cur || y_new == y_cur || x_new == y_new)
        return fail(MESH_SDD_E_INVAL, "output arrays must not alias the input mesh");
    MpOpts o;
    if ((rc = read_opts(opts, o)) != MESH_SDD_OK) return rc;
    mesh_sdd_ctx *ctx = inst->ctx;
    const mesh_sdd_desc &d = inst->d;
    const size_t n = grid_size(d);
    std::lock_guard<std::mutex> g(ctx->gpu_mu);
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    DevIn x0, y0, b1, ix, iy;
    DevOut xo, yo;
    SyncOnExit sync{st};
    if ((rc = stage_in(ctx, x_cur, n, on_device, x0, st)) || (rc = stage_in(ctx, y_cur, n, on_device, y0, st)) ||
        (rc = stage_in(ctx, bnd_new, bnd_size(d), on_device, b1, st)))
        return rc;
    if (with_interfaces && inst->M > 0) {
        if ((rc = stage_in(ctx, iface_x, (size_t)inst->M, on_device, ix, st)) ||
            (rc = stage_in(ctx, iface_y, (size_t)inst->M, on_device, iy, st)))
            return rc;
    }
    if ((rc = stage_out(ctx, x_new, n, on_device, xo)) || (rc = stage_out(ctx, y_new, n, on_device, yo))) return rc;
    rc = solve_dev(inst, o, x0.p, y0.p, b1.p, ix.p, iy.p, with_interfaces, xo.p, yo.p, st);
    if (rc != MESH_SDD_OK) return rc;
    if ((rc = finish(xo, st)) || (rc = finish(yo, st))) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    return MESH_SDD_OK;
}

int mesh_sdd_subdomain_solve(mesh_sdd *inst, const double *x_cur, const double *y_cur, const double *bnd_new,
                             const double *iface_x, const double *iface_y, double *x_new, double *y_new,
                             const mesh_sdd_mp_opts *opts, int pointers_on_device)
try {
    return solve_common(inst, x_cur, y_cur, bnd_new, iface_x, iface_y, x_new, y_new, opts, pointers_on_device, true);
} catch (...) {
    return abi_exception();
}

int mesh_sdd_single_domain_solve(mesh_sdd *inst, const double *x_cur, const double *y_cur, const double *bnd_new,
                                 double *x_new, double *y_new, const mesh_sdd_mp_opts *opts, int pointers_on_device)
try {
    return solve_common(inst, x_cur, y_cur, bnd_new, nullptr, nullptr, x_new, y_new, opts, pointers_on_device, false);
} catch (...) {
    return abi_exception();
}

int mesh_sdd_mp_step(mesh_sdd *inst, const mesh_sdd_step *step, const mesh_sdd_mp_opts *opts, double *x_new,
                     double *y_new, double *bnd_new, mesh_sdd_result *result)
try {
    int rc = check_ready(inst);
    if (rc != MESH_SDD_OK) return rc;
    if (!step || !result || !x_new || !y_new || !bnd_new) return fail(MESH_SDD_E_INVAL, "NULL argument");
    if (step->struct_size != sizeof(mesh_sdd_step) || result->struct_size != sizeof(mesh_sdd_result))
        return fail(MESH_SDD_E_INVAL, "struct_size mismatch");
    MpOpts o;
    if ((rc = read_opts(opts, o)) != MESH_SDD_OK) return rc;
    if (!step->x_cur || !step->y_cur || !step->bnd_t0 || (!o.edge_gen && !step->bnd_t1))
        return fail(MESH_SDD_E_INVAL, "NULL input array");
    mesh_sdd_ctx *ctx = inst->ctx;
    const mesh_sdd_desc &d = inst->d;
    const size_t n = grid_size(d), nb = bnd_size(d), M = (size_t)inst->M;
    const int in_dev = step->inputs_on_device, out_dev = result->outputs_on_device;
    DevIn x0, y0, b0;
    DevOut bo, xo, yo;
    DevOut rs[5];
    SyncOnExit sync{ctx->stream};
    TimerEvents ev;
    {
        std::lock_guard<std::mutex> g(ctx->gpu_mu);
        HIP_TRY(hipSetDevice(ctx->device));
        hipStream_t st = ctx->stream;
        if ((rc = stage_in(ctx, step->x_cur, n, in_dev, x0, st)) || (rc = stage_in(ctx, step->y_cur, n, in_dev, y0, st)) ||
            (rc = stage_in(ctx, step->bnd_t0, nb, in_dev, b0, st)))
            return rc;
        if ((rc = stage_out(ctx, bnd_new, nb, out_dev, bo)) || (rc = stage_out(ctx, x_new, n, out_dev, xo)) ||
            (rc = stage_out(ctx, y_new, n, out_dev, yo)))
            return rc;
        double *dst[5] = {result->mean_x, result->mean_y, result->se_x, result->se_y, result->exit_frac};
        for (int k = 0; k < 5; ++k) {
            if (!dst[k] && M > 0) return fail(MESH_SDD_E_INVAL, "NULL result array");
            if ((rc = stage_out(ctx, dst[k], M, out_dev, rs[k])) != MESH_SDD_OK) return rc;
        }
        HIP_TRY(ev.create());
        HIP_TRY(hipEventRecord(ev.e0, st));
        // boundary arrays at t^{n+1}
        if (o.edge_gen) {
            HIP_TRY(hipMemcpyAsync(bo.p, b0.p, nb * 8, hipMemcpyDeviceToDevice, st));
            if ((rc = edge_dev(inst, o, bo.p, st)) != MESH_SDD_OK) return rc;
        } else {
            HIP_TRY(hipMemcpyAsync(bo.p, step->bnd_t1, nb * 8, in_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                   st));
        }
        HIP_TRY(hipStreamSynchronize(st));
    }
    // interface estimate on device arrays (takes the context lock itself)
    mesh_sdd_step s2 = *step;
    s2.inputs_on_device = 1;
    s2.x_cur = x0.p;
    s2.y_cur = y0.p;
    s2.bnd_t0 = b0.p;
    s2.bnd_t1 = bo.p;
    mesh_sdd_result r2{};
    r2.struct_size = sizeof(mesh_sdd_result);
    r2.outputs_on_device = 1;
    r2.mean_x = rs[0].p;
    r2.mean_y = rs[1].p;
    r2.se_x = rs[2].p;
    r2.se_y = rs[3].p;
    r2.exit_frac = rs[4].p;
    rc = mesh_sdd_solve_interfaces(inst, &s2, &r2);
    if (rc != MESH_SDD_OK) return rc;
    std::lock_guard<std::mutex> g(ctx->gpu_mu);
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    rc = solve_dev(inst, o, x0.p, y0.p, bo.p, rs[0].p, rs[1].p, true, xo.p, yo.p, st);
    if (rc == MESH_SDD_OK) {
        for (DevOut *p : {&bo, &xo, &yo, &rs[0], &rs[1], &rs[2], &rs[3], &rs[4]})
            if ((rc = finish(*p, st)) != MESH_SDD_OK) break;
    }
    if (rc == MESH_SDD_OK) rc = hipEventRecord(ev.e1, st) == hipSuccess ? MESH_SDD_OK : fail(MESH_SDD_E_DEVICE, "event record failed");
    hipError_t se = hipStreamSynchronize(st);
    float ms = 0.0f;
    if (rc == MESH_SDD_OK && se == hipSuccess) (void)hipEventElapsedTime(&ms, ev.e0, ev.e1);
    if (rc != MESH_SDD_OK) return rc;
    if (se != hipSuccess) return fail(MESH_SDD_E_DEVICE, "mesh step failed: %s", hipGetErrorString(se));
    result->executed_path_steps = r2.executed_path_steps;
    result->paths_per_node = r2.paths_per_node;
    result->device_ms = ms;
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_transfer_field(mesh_sdd *inst, const double *x_old, const double *y_old, const double *f_old,
                            const double *x_new, const double *y_new, double *f_new, int pointers_on_device)
try {
    if (!inst) return fail(MESH_SDD_E_INVAL, "instance is NULL");
    if (!x_old || !y_old || !f_old || !x_new || !y_new || !f_new) return fail(MESH_SDD_E_INVAL, "NULL array");
    mesh_sdd_ctx *ctx = inst->ctx;
    const mesh_sdd_desc &d = inst->d;
    const size_t n = grid_size(d);
    if (!pointers_on_device) {
        for (size_t k = 0; k < n; ++k)
            if (!std::isfinite(x_old[k]) || !std::isfinite(y_old[k]) || !std::isfinite(f_old[k]) ||
                !std::isfinite(x_new[k]) || !std::isfinite(y_new[k]))
                return fail(MESH_SDD_E_INVAL, "input value %zu is not finite", k);
    }
    std::lock_guard<std::mutex> g(ctx->gpu_mu);
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    DevIn xo, yo, fo, xn, yn;
    DevOut out;
    SyncOnExit sync{st};
    int rc;
    if ((rc = stage_in(ctx, x_old, n, pointers_on_device, xo, st)) ||
        (rc = stage_in(ctx, y_old, n, pointers_on_device, yo, st)) ||
        (rc = stage_in(ctx, f_old, n, pointers_on_device, fo, st)) ||
        (rc = stage_in(ctx, x_new, n, pointers_on_device, xn, st)) ||
        (rc = stage_in(ctx, y_new, n, pointers_on_device, yn, st)) ||
        (rc = stage_out(ctx, f_new, n, pointers_on_device, out)))
        return rc;
    msdd::TransferArgs a{};
    a.n_xi = d.n_xi;
    a.n_eta = d.n_eta;
    a.per_xi = d.periodic_xi;
    a.per_eta = d.periodic_eta;
    a.Lx = d.Lx;
    a.Ly = d.Ly;
    a.x_old = xo.p;
    a.y_old = yo.p;
    a.f_old = fo.p;
    a.x_new = xn.p;
    a.y_new = yn.p;
    a.f_new = out.p;
    HIP_TRY(msdd::launch_transfer_p1(a, st));
    if ((rc = finish(out, st)) != MESH_SDD_OK) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_set_monitor_arclength(mesh_sdd *inst, const double *u, const double *x, const double *y, double alpha,
                                   int normalize, int pointers_on_device)
try {
    if (!inst || !u || !x || !y) return fail(MESH_SDD_E_INVAL, "NULL argument");
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(MESH_SDD_E_INVAL, "alpha must be finite and >= 0");
    if (inst->inflight.load() > 0) return fail(MESH_SDD_E_STATE, "instance has requests in flight");
    mesh_sdd_ctx *ctx = inst->ctx;
    const mesh_sdd_desc &d = inst->d;
    const size_t n = grid_size(d);
    std::lock_guard<std::mutex> g(ctx->gpu_mu);
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    DevIn du, dx, dy;
    DevBuf gbuf, flags;
    SyncOnExit sync{st};
    int rc;
    if ((rc = stage_in(ctx, u, n, pointers_on_device, du, st)) || (rc = stage_in(ctx, x, n, pointers_on_device, dx, st)) ||
        (rc = stage_in(ctx, y, n, pointers_on_device, dy, st)))
        return rc;
    gbuf.pool = flags.pool = &ctx->pool;
    if (gbuf.alloc(n * 8) || flags.alloc(16)) return fail(MESH_SDD_E_NOMEM, "device allocation failed");
    HIP_TRY(hipMemsetAsync(flags.p, 0, 16, st));
    unsigned long long *gmax = flags.as<unsigned long long>();
    unsigned int *bad = reinterpret_cast<unsigned int *>(gmax + 1);
    HIP_TRY(msdd::launch_arclength(du.p, dx.p, dy.p, d.n_xi, d.n_eta, d.periodic_xi, d.periodic_eta, d.Lx, d.Ly, alpha,
                                   normalize ? 1 : 0, gbuf.as<double>(), gmax, bad, inst->rho_in.as<double>(), st));
    unsigned int hbad = 0;
    HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hbad) {
        inst->monitor_set = false;
        return fail(MESH_SDD_E_INVAL, "|grad u| is not finite somewhere (degenerate mesh or bad input)");
    }
    return install_monitor(inst, st);
} catch (...) {
    return abi_exception();
}

int mesh_sdd_get_monitor(mesh_sdd *inst, double *rho_out, int pointer_on_device)
try {
    int rc = check_ready(inst);
    if (rc != MESH_SDD_OK) return rc;
    if (!rho_out) return fail(MESH_SDD_E_INVAL, "NULL argument");
    mesh_sdd_ctx *ctx = inst->ctx;
    std::lock_guard<std::mutex> g(ctx->gpu_mu);
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipMemcpyAsync(rho_out, inst->rho_in.p, grid_size(inst->d) * 8,
                           pointer_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_mesh_quality(mesh_sdd *inst, const double *x_sd, const double *y_sd, const double *x_dd,
                          const double *y_dd, double *r_cells, double *r_max, double *r_mean, int pointers_on_device)
try {
    if (!inst || !x_sd || !y_sd || !x_dd || !y_dd || !r_max || !r_mean) return fail(MESH_SDD_E_INVAL, "NULL argument");
    mesh_sdd_ctx *ctx = inst->ctx;
    const mesh_sdd_desc &d = inst->d;
    const size_t n = grid_size(d), nc = (size_t)(d.n_xi - 1) * (d.n_eta - 1);
    std::lock_guard<std::mutex> g(ctx->gpu_mu);
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    DevIn a, b, c, e;
    DevOut rc_out;
    DevBuf pm, ps, o2;
    SyncOnExit sync{st};
    int rc;
    if ((rc = stage_in(ctx, x_sd, n, pointers_on_device, a, st)) || (rc = stage_in(ctx, y_sd, n, pointers_on_device, b, st)) ||
        (rc = stage_in(ctx, x_dd, n, pointers_on_device, c, st)) || (rc = stage_in(ctx, y_dd, n, pointers_on_device, e, st)))
        return rc;
    if (r_cells && (rc = stage_out(ctx, r_cells, nc, pointers_on_device, rc_out)) != MESH_SDD_OK) return rc;
    const int parts = msdd::quality_parts(d.n_xi, d.n_eta);
    pm.pool = ps.pool = o2.pool = &ctx->pool;
    if (pm.alloc((size_t)parts * 8) || ps.alloc((size_t)parts * 8) || o2.alloc(16))
        return fail(MESH_SDD_E_NOMEM, "device allocation failed");
    HIP_TRY(msdd::launch_quality(a.p, b.p, c.p, e.p, d.n_xi, d.n_eta, r_cells ? rc_out.p : nullptr, pm.as<double>(),
                                 ps.as<double>(), o2.as<double>(), st));
    double h2[2] = {0.0, 0.0};
    HIP_TRY(hipMemcpyAsync(h2, o2.p, sizeof h2, hipMemcpyDeviceToHost, st));
    if (r_cells && (rc = finish(rc_out, st)) != MESH_SDD_OK) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    if (!std::isfinite(h2[0]) || !std::isfinite(h2[1]))
        return fail(MESH_SDD_E_INVAL, "mesh quality is not finite (degenerate cell)");
    *r_max = h2[0];
    *r_mean = h2[1];
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

}  // extern "C"
