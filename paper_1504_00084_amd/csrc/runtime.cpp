// Host runtime behind the C-ABI of include/mesh_sdd.h: contexts, problem
// instances, requests (one interface solve each, paper section 3.4-3.6),
// the work-queue builder, the autotuner of the batched FP32 kernel, and the
// continuous-batching scheduler that serves submit/poll.
//
// Data flow of one request:
//   host/device inputs --(copy, snapshot)--> FP64 staging (mesh, boundary)
//   --prep kernels--> padded meshes (FP64 + FP32), FP32 boundary
//   --path kernel (FP32 batched or FP64 plain)--> per-(node, chunk) partials
//   --finalize kernel--> mean, SE, exit fraction per interface node
//   --copy--> caller's result arrays.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime_internal.hpp"

using msdd::InstView;
using msdd::NodeSpan;
using msdd::Partial;
using msdd::WorkRange;

namespace msdd_rt {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    try {
        g_last_error = buf;
    } catch (...) {   // no memory left even for the message: keep the status
    }
    return code;
}

int abi_exception() noexcept
{
    try {
        throw;
    } catch (const std::bad_alloc &) {
        return fail(MESH_SDD_E_NOMEM, "host memory allocation failed");
    } catch (const std::exception &e) {
        return fail(MESH_SDD_E_NOMEM, "host resources exhausted: %s", e.what());
    } catch (...) {
        return fail(MESH_SDD_E_NOMEM, "host resources exhausted");
    }
}

// The 48-B cell records, behind the dt rho_eta plane in inst.cells.
float4 *cell_records(const mesh_sdd &inst)
{
    return inst.cells.as<float4>() + (size_t)(inst.d.n_xi - 1) * (inst.d.n_eta - 1);
}

// Build the monitor's node tables and FP32 cell table from inst->rho_in on
// `st` (a0), wait for them, and mark the monitor as set.  The caller holds
// the context's gpu_mu.
int install_monitor(mesh_sdd *inst, hipStream_t st)
{
    const mesh_sdd_desc &d = inst->d;
    HIP_TRY(msdd::launch_prep_gradient(inst->rho_in.as<double>(), d.n_xi, d.n_eta, d.periodic_xi, d.periodic_eta,
                                       inst->rho.as<double>(), inst->rho_xi.as<double>(), inst->rho_eta.as<double>(), st));
    HIP_TRY(msdd::launch_prep_cells(inst->rho.as<double>(), inst->rho_xi.as<double>(), inst->rho_eta.as<double>(),
                                    d.n_xi, d.n_eta, d.tau / (double)d.K, cell_records(*inst),
                                    inst->cells.as<float4>(), st));
    HIP_TRY(msdd::launch_to_f32(inst->rho.as<double>(), inst->rho_f.as<float>(), (size_t)d.n_xi * d.n_eta, st));
    HIP_TRY(msdd::launch_scaled_to_f32(inst->rho_xi.as<double>(), d.tau / (double)d.K, inst->rhox_f.as<float>(),
                                       (size_t)d.n_xi * d.n_eta, st));
    HIP_TRY(msdd::launch_scaled_to_f32(inst->rho_eta.as<double>(), d.tau / (double)d.K, inst->rhoy_f.as<float>(),
                                       (size_t)d.n_xi * d.n_eta, st));
    HIP_TRY(hipStreamSynchronize(st));
    inst->monitor_set = true;
    return MESH_SDD_OK;
}

// Equispaced sampling (section 3.6): on an interface line the nodes at
// multiples of the stride along the line run paths; line crossings sit on
// such multiples (the stride divides the subdomain sizes).
std::vector<int32_t> sampled_ranks(const mesh_sdd &inst, int stride)
{
    std::vector<int32_t> out;
    out.reserve((size_t)inst.M);
    const int Px = (inst.d.n_xi - 1) / inst.d.sub_xi, Py = (inst.d.n_eta - 1) / inst.d.sub_eta;
    for (int32_t r = 0; r < inst.M; ++r) {
        const int i = inst.node_i[r], j = inst.node_j[r];
        if (stride <= 1 || (i % Px == 0 && j % stride == 0) || (j % Py == 0 && i % stride == 0)) out.push_back(r);
    }
    return out;
}

}  // namespace msdd_rt

using namespace msdd_rt;

namespace {
constexpr size_t kLdsBytes = 160u * 1024u;   // LDS of one CU on gfx950
}



namespace {

// ---------------------------------------------------------------------------
// Validation and interface nodes (a1)
// ---------------------------------------------------------------------------
int validate_desc(const mesh_sdd_desc *d)
{
    if (!d) return fail(MESH_SDD_E_INVAL, "descriptor is NULL");
    if (d->struct_size != sizeof(mesh_sdd_desc))
        return fail(MESH_SDD_E_INVAL, "desc.struct_size %u != %zu", d->struct_size, sizeof(mesh_sdd_desc));
    if (d->n_xi < 4 || d->n_eta < 4 || d->n_xi > 8193 || d->n_eta > 8193)
        return fail(MESH_SDD_E_INVAL, "grid %d x %d outside [4, 8193]", d->n_xi, d->n_eta);
    if (d->sub_xi < 1 || d->sub_eta < 1 || (d->n_xi - 1) % d->sub_xi || (d->n_eta - 1) % d->sub_eta)
        return fail(MESH_SDD_E_INVAL, "(n-1) %% sub != 0: n = (%d, %d), sub = (%d, %d)", d->n_xi, d->n_eta,
                    d->sub_xi, d->sub_eta);
    if ((d->periodic_xi != 0 && d->periodic_xi != 1) || (d->periodic_eta != 0 && d->periodic_eta != 1))
        return fail(MESH_SDD_E_INVAL, "periodic flags must be 0 or 1");
    if (d->K < 1 || d->K > (1 << 28)) return fail(MESH_SDD_E_INVAL, "K = %d outside [1, 2^28]", d->K);
    if (!(d->tau > 0.0) || !std::isfinite(d->tau)) return fail(MESH_SDD_E_INVAL, "tau must be > 0");
    if (!(d->Lx > 0.0) || !(d->Ly > 0.0) || !std::isfinite(d->Lx) || !std::isfinite(d->Ly))
        return fail(MESH_SDD_E_INVAL, "Lx, Ly must be > 0");
    if (d->precision != MESH_SDD_FP32 && d->precision != MESH_SDD_FP64)
        return fail(MESH_SDD_E_INVAL, "precision must be MESH_SDD_FP32 or MESH_SDD_FP64");
    if (d->bridge != 0 && d->bridge != 1) return fail(MESH_SDD_E_INVAL, "bridge must be 0 or 1");
    if (d->instance_id >= 65536u) return fail(MESH_SDD_E_INVAL, "instance_id %u >= 65536", d->instance_id);
    return MESH_SDD_OK;
}

// Interface nodes (section 3.5): a multiple of the subdomain width on either
// axis, not on a Dirichlet side; on a periodic axis the image node n-1 is
// skipped and the seam (index 0) belongs to the interfaces.  Row-major (j, i).
void enumerate_nodes(const mesh_sdd_desc &d, std::vector<int32_t> &ni, std::vector<int32_t> &nj)
{
    const int wx = (d.n_xi - 1) / d.sub_xi, wy = (d.n_eta - 1) / d.sub_eta;
    const int j_lo = d.periodic_eta ? 0 : 1, j_hi = d.n_eta - 2;   // inclusive
    const int i_lo = d.periodic_xi ? 0 : 1, i_hi = d.n_xi - 2;
    ni.clear();
    nj.clear();
    for (int j = j_lo; j <= j_hi; ++j) {
        const bool row_line = (j % wy) == 0;
        for (int i = i_lo; i <= i_hi; ++i) {
            if (row_line || (i % wx) == 0) {
                ni.push_back(i);
                nj.push_back(j);
            }
        }
    }
}

size_t instance_bytes(const mesh_sdd_desc &d, int M)
{
    const size_t n = (size_t)d.n_xi * d.n_eta;
    const size_t cells = (size_t)(d.n_xi - 1) * (d.n_eta - 1);
    // monitor tables, FP32 rho, dt rho_xi and dt rho_eta, cell records, node-rank map, interface nodes in
    // rank order, stride-1 node lists (block order)
    return 4 * n * sizeof(double) + 3 * n * sizeof(float) + 4 * cells * sizeof(float4) + n * sizeof(int32_t) +
           2 * (size_t)M * sizeof(int32_t) + 3 * (size_t)M * sizeof(int32_t);
}

int64_t resolve_paths(const mesh_sdd &inst, const mesh_sdd_step &s)
{
    if (s.target_se > 0.0) {
        const double L = std::max(inst.d.Lx, inst.d.Ly);
        const double n = std::ceil(2.0 * inst.d.tau * L * L / (s.target_se * s.target_se));
        const int64_t cap = s.max_paths > 0 ? s.max_paths : 1000000;
        return std::max<int64_t>(2, std::min<int64_t>(cap, (int64_t)n));
    }
    return s.paths_per_node;
}

// Sampling stride along the interface lines (section 3.6): 0 or 1 for all
// nodes; else it must divide both subdomain sizes and leave at least two
// segments along every grid line.
int check_stride(const mesh_sdd_desc &d, uint32_t st)
{
    if (st <= 1) return MESH_SDD_OK;
    const uint32_t Px = (uint32_t)((d.n_xi - 1) / d.sub_xi), Py = (uint32_t)((d.n_eta - 1) / d.sub_eta);
    if (Px % st || Py % st)
        return fail(MESH_SDD_E_INVAL, "interface_stride %u does not divide the subdomain sizes %u x %u", st, Px, Py);
    if ((uint32_t)(d.n_xi - 1) / st < 2 || (uint32_t)(d.n_eta - 1) / st < 2)
        return fail(MESH_SDD_E_INVAL, "interface_stride %u leaves fewer than two segments along a grid line", st);
    return MESH_SDD_OK;
}

int validate_step(const mesh_sdd &inst, const mesh_sdd_step *s, int64_t *N_out)
{
    if (!s) return fail(MESH_SDD_E_INVAL, "step is NULL");
    if (s->struct_size != sizeof(mesh_sdd_step))
        return fail(MESH_SDD_E_INVAL, "step.struct_size %u != %zu", s->struct_size, sizeof(mesh_sdd_step));
    if (!s->x_cur || !s->y_cur || !s->bnd_t0 || !s->bnd_t1)
        return fail(MESH_SDD_E_INVAL, "step input pointer is NULL");
    if (s->target_se < 0.0 || !std::isfinite(s->target_se)) return fail(MESH_SDD_E_INVAL, "target_se < 0");
    const int64_t N = resolve_paths(inst, *s);
    if (N < 1 || N > (int64_t)1 << 31) return fail(MESH_SDD_E_INVAL, "paths per node %lld outside [1, 2^31]", (long long)N);
    const int rs = check_stride(inst.d, s->interface_stride);
    if (rs != MESH_SDD_OK) return rs;
    *N_out = N;
    if (s->inputs_on_device) return MESH_SDD_OK;   // device inputs are not inspected
    const mesh_sdd_desc &d = inst.d;
    const size_t n = (size_t)d.n_xi * d.n_eta;
    const size_t nb = 4 * (size_t)d.n_eta + 4 * (size_t)d.n_xi;
    for (size_t k = 0; k < n; ++k)
        if (!std::isfinite(s->x_cur[k]) || !std::isfinite(s->y_cur[k]))
            return fail(MESH_SDD_E_INVAL, "mesh value %zu is not finite", k);
    for (size_t k = 0; k < nb; ++k)
        if (!std::isfinite(s->bnd_t0[k]) || !std::isfinite(s->bnd_t1[k]))
            return fail(MESH_SDD_E_INVAL, "boundary value %zu is not finite", k);
    if (!d.periodic_xi && !d.periodic_eta) {
        // the four corners belong to two sides each; their values must agree
        const double tol = 1e-12 * (d.Lx + d.Ly);
        const double *levels[2] = {s->bnd_t0, s->bnd_t1};
        const size_t ne = d.n_eta, nx = d.n_xi;
        for (int l = 0; l < 2; ++l) {
            const double *b = levels[l];
            for (int c = 0; c < 2; ++c) {
                const double *s0 = b + (0 * 2 + c) * ne, *s1 = b + (1 * 2 + c) * ne;
                const double *s2 = b + 4 * ne + (0 * 2 + c) * nx, *s3 = b + 4 * ne + (1 * 2 + c) * nx;
                const double pairs[4][2] = {{s0[0], s2[0]}, {s0[ne - 1], s3[0]}, {s1[0], s2[nx - 1]},
                                            {s1[ne - 1], s3[nx - 1]}};
                for (auto &p : pairs)
                    if (std::fabs(p[0] - p[1]) > tol)
                        return fail(MESH_SDD_E_INVAL, "boundary corner values disagree (%g vs %g)", p[0], p[1]);
            }
        }
    }
    return MESH_SDD_OK;
}

// ---------------------------------------------------------------------------
// Launch shape
// ---------------------------------------------------------------------------
mesh_sdd_launch default_launch()
{
    mesh_sdd_launch l{};
    l.struct_size = sizeof(mesh_sdd_launch);
    l.block = 256;
    // three waves per SIMD: the cell gathers saturate the L1 pipeline there,
    // and more resident waves only add L1 misses (measured on gfx950)
    l.waves_per_simd = 3;
    l.chunk_paths = 128;   // small enough that the LDS variant's wave buffers leave room for a 129x129 rho table
    l.monitor_table = 0;
    l.table_level = 0;
    // leave the stepping loop once fewer than 56 lanes are busy, or after 16
    // quarters (measured on the 129^2 workload: 16 beats 2, 32 and 64; 56
    // beats 48 and 60)
    l.refill_lanes = 56;
    l.max_quarters = 16;
    l.window_kind = 0;     // automatic: see window_kind()
    l.window_margin = 0;   // the kind's default margin
    l.job_split = 0;       // 32, and 256 in grids cut into several two-field windows
    return l;
}

// A shape with every 0 ("default") field replaced by its default.
mesh_sdd_launch with_defaults(mesh_sdd_launch l)
{
    const mesh_sdd_launch d = default_launch();
    l.struct_size = sizeof(mesh_sdd_launch);
    if (l.block == 0) l.block = d.block;
    if (l.chunk_paths == 0) l.chunk_paths = d.chunk_paths;
    if (l.refill_lanes == 0) l.refill_lanes = d.refill_lanes;
    if (l.max_quarters == 0) l.max_quarters = d.max_quarters;
    return l;
}

// How a launch reads the monitor tables.  2: it holds one instance of
// n_nodes nodes (n_nodes > 0) whose node tables of rho and dt rho_xi fit the
// LDS whole; 3: windows of those tables in LDS (several instances, or a grid
// too large); 0: the cell records alone (monitor_table = 1).  *per_cu
// receives the resident 1024-thread workgroups per CU.
int table_level(int n_nodes, int monitor_table, int *per_cu)
{
    *per_cu = 0;
    if (monitor_table != 0) return 0;
    if (n_nodes > 0 && msdd::paths_fp32_table_lds_bytes(2, n_nodes) <= kLdsBytes) {
        const int n = msdd::paths_fp32_table_blocks_per_cu(2, n_nodes);
        if (n >= 1) {
            *per_cu = n;
            return 2;
        }
    }
    const int n = msdd::paths_fp32_window_blocks_per_cu(msdd::kWinBytes);
    if (n >= 1) {
        *per_cu = n;
        return 3;
    }
    return 0;
}

// Shape of a launch over `d` alone: the override, else the bucket's tuned
// shape, else the default.  Its per-instance knobs (chunk_paths, window kind
// and margin) apply to `d` in every launch.
mesh_sdd_launch launch_for(mesh_sdd_ctx *ctx, const mesh_sdd_desc &d)
{
    std::lock_guard<std::mutex> g(ctx->mu);
    if (ctx->has_override) return with_defaults(ctx->override_launch);
    auto it = ctx->tuned.find(TuneKey{d.n_xi, d.n_eta, d.periodic_xi, d.periodic_eta});
    if (it != ctx->tuned.end()) return with_defaults(it->second);
    return default_launch();
}

// Launch-wide knobs of a launch over several instances: the override, else
// the tuned multi-instance shape, else the default.  `one`: the launch holds
// that single instance (its bucket's shape then).
mesh_sdd_launch launch_for_group(mesh_sdd_ctx *ctx, const mesh_sdd_desc *one)
{
    if (one) return launch_for(ctx, *one);
    std::lock_guard<std::mutex> g(ctx->mu);
    if (ctx->has_override) return with_defaults(ctx->override_launch);
    if (ctx->has_batch_tuned) return with_defaults(ctx->batch_tuned);
    return default_launch();
}

int grid_for(mesh_sdd_ctx *ctx, const mesh_sdd_launch &l, uint32_t cap)
{
    const int waves_per_block = l.block / 64;
    int per_cu = msdd::paths_fp32_blocks_per_cu(l.block, cap);   // resident blocks per CU (registers, LDS)
    if (per_cu < 1) per_cu = 1;
    if (l.waves_per_simd > 0) {
        const int want = std::max(1, (l.waves_per_simd * 4) / waves_per_block);
        per_cu = std::min(per_cu, want);
    }
    return std::max(1, ctx->cu_count * per_cu);
}

// ---------------------------------------------------------------------------
// Requests
// ---------------------------------------------------------------------------
size_t request_bytes(const mesh_sdd &inst, int64_t N, int chunk, int32_t Ms)
{
    const mesh_sdd_desc &d = inst.d;
    const size_t n = (size_t)d.n_xi * d.n_eta;
    const size_t np = (size_t)(d.n_xi + 2) * (d.n_eta + 2);
    const size_t nb = 4 * (size_t)d.n_eta + 4 * (size_t)d.n_xi;
    size_t chunks;
    if (d.precision == MESH_SDD_FP64)
        chunks = (size_t)((N + msdd::kFp64Block - 1) / msdd::kFp64Block);
    else
        chunks = (size_t)((N + chunk - 1) / chunk);
    return 2 * n * 8 + 2 * np * 12 + 2 * nb * 12 + (size_t)Ms * (chunks * sizeof(Partial) + sizeof(NodeSpan)) +
           (size_t)inst.M * 5 * sizeof(double) + sizeof(InstView) + 64;
}

// Snapshot host inputs (the caller may free them once submit returns).
std::shared_ptr<Request> make_request(mesh_sdd *inst, const mesh_sdd_step &s, int64_t N)
{
    auto r = std::make_shared<Request>();
    r->inst = inst;
    r->M = inst->M;
    r->stride = s.interface_stride > 1 ? (int)s.interface_stride : 1;
    r->Ms = r->stride > 1 ? (int32_t)sampled_ranks(*inst, r->stride).size() : inst->M;
    r->N = N;
    r->mesh_step = s.mesh_step;
    r->chunk_paths = std::max(64, launch_for(inst->ctx, inst->d).chunk_paths / 64 * 64);
    r->cost_bytes = request_bytes(*inst, N, r->chunk_paths, r->Ms);
    const size_t n = (size_t)inst->d.n_xi * inst->d.n_eta;
    const size_t nb = 4 * (size_t)inst->d.n_eta + 4 * (size_t)inst->d.n_xi;
    if (!s.inputs_on_device) {
        r->hx.assign(s.x_cur, s.x_cur + n);
        r->hy.assign(s.y_cur, s.y_cur + n);
        r->hb0.assign(s.bnd_t0, s.bnd_t0 + nb);
        r->hb1.assign(s.bnd_t1, s.bnd_t1 + nb);
    }
    return r;
}

// Windows of the windowed kernel.  Kind 0 holds (rho, dt rho_xi) per node (8
// bytes, at most kWinNodes nodes); kind 1 also dt rho_eta per node (4 bytes
// more), so a lane inside it gathers nothing from memory, at the price of a
// smaller window.  Chosen per grid, by measurement: kind 1
// where it holds the whole grid (no gather at all); kind 0 where the two
// fields of the whole grid fit (one well-cached gather per path-step beats
// many small blocks and window refills); kind 1 below kWin1MaxN nodes per
// axis; kind 0 above, where paths spread over more cells than a kind-1 window
// holds around its block and the larger kind-0 window needs fewer record
// gathers.
constexpr int kWin1MaxN = 400;

// LDS bytes of a window of tw x th nodes.
size_t window_bytes(int kind, int tw, int th)
{
    return (size_t)tw * th * (kind ? 12 : 8);
}

// want: 0 automatic, 1 two-field (kind 0), 2 three-field (kind 1); a
// window that holds the whole grid is always taken.
int window_kind(const mesh_sdd_desc &d, int want = 0)
{
    if (window_bytes(1, d.n_xi, d.n_eta) <= msdd::kWinBytes) return 1;
    if (window_bytes(0, d.n_xi, d.n_eta) <= msdd::kWinBytes) return 0;
    if (want == 1) return 0;
    if (want == 2) return 1;
    return std::max(d.n_xi, d.n_eta) < kWin1MaxN ? 1 : 0;
}

// Window extent along each axis: within kWinBytes of LDS, near square, the
// whole axis where it fits.
void window_dims(int kind, int n_xi, int n_eta, int *wx, int *wy)
{
    const int side = kind ? msdd::kWin3Side : 140;   // the largest square of each kind within kWinBytes
    int y = std::min(n_eta, side);
    int x = n_xi;
    while (window_bytes(kind, x, y) > msdd::kWinBytes) --x;
    while (y < n_eta && window_bytes(kind, x, y + 1) <= msdd::kWinBytes) ++y;
    *wx = x;
    *wy = y;
}

// Window nodes beyond a block on each side, where the axis does not fit
// (`want` > 0: the tuned margin).
int window_margin(int kind, int want = 0) { return want > 0 ? want : (kind ? 30 : 45); }

// Block layout of an instance's windowed launches: window kind and margin.
struct Layout {
    int kind, margin;
};

Layout layout_of(const mesh_sdd_desc &d, const mesh_sdd_launch &l)
{
    const int kind = window_kind(d, l.window_kind);
    return Layout{kind, window_margin(kind, l.window_margin)};
}

// Block length along an axis of n nodes whose window is w nodes long (at
// least one node), and the window origin of block b (centred on the block,
// clamped to the grid).
int block_len(int margin, int n, int w) { return n <= w ? n : std::max(1, w - 2 * margin); }
int window_origin(int b, int len, int n, int w) { return n <= w ? 0 : std::clamp(b * len - (w - len) / 2, 0, n - w); }

// Z (Morton) order of block (bx, by): consecutive blocks form compact
// patches of the grid, so the jobs that one XCD runs at a time read the
// records of a compact region, which its L2 holds better than a band of
// row-major blocks (measured: 1 % faster on the batched mix, from its 513^2
// grids).
uint32_t z_order(uint32_t bx, uint32_t by)
{
    uint32_t m = 0;
    for (int k = 0; k < 16; ++k) m |= ((bx >> k) & 1u) << (2 * k) | ((by >> k) & 1u) << (2 * k + 1);
    return m;
}

// Sorts `ranks` (ascending) into block order -- blocks in Z order, ranks
// ascending inside a block -- and lists the runs of positions per block
// with their windows.
void order_by_blocks(const mesh_sdd &inst, const Layout &lay, std::vector<int32_t> &ranks,
                     std::vector<BlockRun> &blocks)
{
    const int n_xi = inst.d.n_xi, n_eta = inst.d.n_eta;
    const int kind = lay.kind;
    int wx = 0, wy = 0;
    window_dims(kind, n_xi, n_eta, &wx, &wy);
    const int lx = block_len(lay.margin, n_xi, wx), ly = block_len(lay.margin, n_eta, wy);
    const int nbx = (n_xi + lx - 1) / lx;
    auto block_of = [&](int32_t r) { return (inst.node_j[(size_t)r] / ly) * nbx + inst.node_i[(size_t)r] / lx; };
    auto z_of = [&](int b) { return z_order((uint32_t)(b % nbx), (uint32_t)(b / nbx)); };
    std::stable_sort(ranks.begin(), ranks.end(),
                     [&](int32_t a, int32_t b) { return z_of(block_of(a)) < z_of(block_of(b)); });
    blocks.clear();
    for (size_t k = 0; k < ranks.size();) {
        const int b = block_of(ranks[k]);
        size_t e = k + 1;
        while (e < ranks.size() && block_of(ranks[e]) == b) ++e;
        BlockRun run;
        run.pos_begin = (int32_t)k;
        run.pos_end = (int32_t)e;
        run.i0 = window_origin(b % nbx, lx, n_xi, wx);
        run.j0 = window_origin(b / nbx, ly, n_eta, wy);
        run.tw = wx;
        run.th = wy;
        run.kind = kind;
        blocks.push_back(run);
        k = e;
    }
}

// Node lists of `stride` in the block order of `lay` (built on first use
// and kept by the instance).  Caller holds gpu_mu.
int sample_set(mesh_sdd &inst, int stride, const Layout &lay, const SampleSet **out)
{
    const auto key = std::make_tuple(stride, lay.kind, lay.margin);
    auto it = inst.samples.find(key);
    if (it != inst.samples.end()) {
        *out = it->second.get();
        return MESH_SDD_OK;
    }
    std::vector<int32_t> ranks = sampled_ranks(inst, stride);
    const size_t Ms = ranks.size();
    auto set = std::make_unique<SampleSet>();
    set->kind = lay.kind;
    set->margin = lay.margin;
    order_by_blocks(inst, lay, ranks, set->blocks);
    set->pos_of_rank.assign((size_t)inst.M, -1);
    for (size_t k = 0; k < Ms; ++k) set->pos_of_rank[(size_t)ranks[k]] = (int32_t)k;
    std::vector<int32_t> host(3 * Ms);
    for (size_t k = 0; k < Ms; ++k) {
        host[k] = inst.node_i[ranks[k]];
        host[Ms + k] = inst.node_j[ranks[k]];
        host[2 * Ms + k] = ranks[k];
    }
    set->stride = stride;
    set->Ms = (int32_t)Ms;
    if (set->lists.alloc(host.size() * sizeof(int32_t)) != hipSuccess)
        return fail(MESH_SDD_E_NOMEM, "device allocation of the sampled node lists failed");
    if (Ms) HIP_TRY(hipMemcpy(set->lists.p, host.data(), host.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (!inst.samples.empty()) {   // every set after the first counts against the budget
        std::lock_guard<std::mutex> lk(inst.ctx->mu);
        inst.resident_bytes += set->lists.bytes;
        inst.ctx->in_use += set->lists.bytes;
    }
    *out = set.get();
    inst.samples.emplace(key, std::move(set));
    return MESH_SDD_OK;
}

// Work items of one FP32 launch (and of one request) are numbered in 32 bits,
// and the queue counters pass the last item by one pop per wave: 2^20 of
// headroom below 2^32.  A host test build lowers the limit to exercise the
// split of a batch into several launches.
#ifndef MESH_SDD_MAX_LAUNCH_ITEMS
#define MESH_SDD_MAX_LAUNCH_ITEMS 0xFFF00000u
#endif
constexpr uint32_t kMaxLaunchItems = MESH_SDD_MAX_LAUNCH_ITEMS;

// Allocate the request's device buffers, stage its inputs and run the prep
// kernels; builds the work items.  With an arena the buffers are carved from
// it instead of allocated (the no-allocation solve).  Caller holds gpu_mu.
int stage_request(Request &r, const mesh_sdd_step *dev_step, Arena *arena = nullptr)
{
    mesh_sdd &inst = *r.inst;
    mesh_sdd_ctx *ctx = inst.ctx;
    const mesh_sdd_desc &d = inst.d;
    hipStream_t st = ctx->stream;
    const size_t n = (size_t)d.n_xi * d.n_eta;
    const size_t np = (size_t)(d.n_xi + 2) * (d.n_eta + 2);
    const size_t nb = 4 * (size_t)d.n_eta + 4 * (size_t)d.n_xi;
    const int M = inst.M;
    const bool fp64 = d.precision == MESH_SDD_FP64;
    int rc = MESH_SDD_OK;
    if (arena) {
        // no allocation: the set of the instance's current layout if built,
        // else any set of the stride (the layout orders the work only)
        const Layout lay = layout_of(d, launch_for(ctx, d));
        auto it = inst.samples.find(std::make_tuple(r.stride, lay.kind, lay.margin));
        if (it == inst.samples.end())
            for (auto s = inst.samples.begin(); s != inst.samples.end(); ++s)
                if (std::get<0>(s->first) == r.stride) it = s;
        if (it == inst.samples.end())
            return fail(MESH_SDD_E_STATE, "interface stride %d: its node lists are built by the first allocating "
                        "solve with that stride", r.stride);
        r.ss = it->second.get();
    } else {
        rc = sample_set(inst, r.stride, layout_of(d, launch_for(ctx, d)), &r.ss);
        if (rc != MESH_SDD_OK) return rc;
    }
    const int Ms = r.ss->Ms;

    uint32_t chunks;
    if (fp64)
        chunks = (uint32_t)((r.N + msdd::kFp64Block - 1) / msdd::kFp64Block);
    else
        chunks = (uint32_t)((r.N + r.chunk_paths - 1) / r.chunk_paths);
    r.chunks_per_node = chunks;
    const size_t n_part = (size_t)Ms * chunks;
    // the kernels number (node, chunk) items and partials in 32 bits; an FP64
    // launch runs one 256-thread block per item, within HIP's 2^32 work-items
    if (!fp64 && n_part > (size_t)kMaxLaunchItems)
        return fail(MESH_SDD_E_INVAL, "%zu (node, chunk) work items, more than 2^32 - 2^20 (fewer paths per node or "
                    "an interface stride)", n_part);
    if (fp64 && n_part >= ((size_t)1 << 32) / msdd::kFp64Block)
        return fail(MESH_SDD_E_INVAL, "FP64: %zu (node, block) pairs, at least 2^24 (fewer paths per node or an "
                    "interface stride)", n_part);

    for (DevBuf *b : {&r.x64, &r.y64, &r.b0, &r.b1, &r.xpad, &r.ypad, &r.xpad_f, &r.ypad_f, &r.b0f, &r.b1f,
                      &r.view, &r.partials, &r.spans, &r.out, &r.steps_total}) {
        b->pool = &ctx->pool;
        b->arena = arena;
    }
    if (r.x64.alloc(n * 8) || r.y64.alloc(n * 8) || r.b0.alloc(nb * 8) || r.b1.alloc(nb * 8) ||
        r.xpad.alloc(np * 8) || r.ypad.alloc(np * 8) || r.xpad_f.alloc(np * 4) || r.ypad_f.alloc(np * 4) ||
        r.b0f.alloc(nb * 4) || r.b1f.alloc(nb * 4) || r.view.alloc(sizeof(InstView)) ||
        r.partials.alloc(n_part * sizeof(Partial)) || r.spans.alloc((size_t)Ms * sizeof(NodeSpan)) ||
        r.out.alloc((size_t)5 * M * sizeof(double)) || r.steps_total.alloc(sizeof(unsigned long long)))
        return fail(MESH_SDD_E_NOMEM, "device allocation for a request failed");

    if (dev_step) {
        HIP_TRY(hipMemcpyAsync(r.x64.p, dev_step->x_cur, n * 8, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(r.y64.p, dev_step->y_cur, n * 8, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(r.b0.p, dev_step->bnd_t0, nb * 8, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(r.b1.p, dev_step->bnd_t1, nb * 8, hipMemcpyDeviceToDevice, st));
    } else {
        HIP_TRY(hipMemcpyAsync(r.x64.p, r.hx.data(), n * 8, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(r.y64.p, r.hy.data(), n * 8, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(r.b0.p, r.hb0.data(), nb * 8, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(r.b1.p, r.hb1.data(), nb * 8, hipMemcpyHostToDevice, st));
    }
    HIP_TRY(msdd::launch_prep_mesh(r.x64.as<double>(), r.y64.as<double>(), d.n_xi, d.n_eta, d.periodic_xi,
                                   d.periodic_eta, d.Lx, d.Ly, r.xpad.as<double>(), r.ypad.as<double>(),
                                   r.xpad_f.as<float>(), r.ypad_f.as<float>(), st));
    HIP_TRY(msdd::launch_to_f32(r.b0.as<double>(), r.b0f.as<float>(), nb, st));
    HIP_TRY(msdd::launch_to_f32(r.b1.as<double>(), r.b1f.as<float>(), nb, st));

    // kernel view
    InstView &v = r.v;
    std::memset(&v, 0, sizeof v);
    v.n_xi = d.n_xi;
    v.n_eta = d.n_eta;
    v.per_xi = d.periodic_xi;
    v.per_eta = d.periodic_eta;
    v.K = d.K;
    // 2: substeps up to 4e-3, where the FP32 kernels take the nearer side of
    // each Dirichlet axis alone (the other's crossing probability is below
    // 1e-20); 1: longer substeps, all four sides (see path_kind)
    v.bridge = d.bridge ? (d.tau / (double)d.K <= 4e-3 ? 2 : 1) : 0;
    v.M = Ms;
    v.key0 = (uint32_t)(d.seed & 0xFFFFFFFFu);
    v.key1 = (uint32_t)(d.seed >> 32);
    v.ctr3 = (d.instance_id << 16) | (r.mesh_step & 0xFFFFu);
    v.Lx = d.Lx;
    v.Ly = d.Ly;
    v.tau = d.tau;
    v.dt = d.tau / (double)d.K;
    v.Lx_f = (float)d.Lx;
    v.Ly_f = (float)d.Ly;
    v.dt_f = (float)v.dt;
    v.sq2dt_f = (float)std::sqrt(2.0 * v.dt);
    v.inv_dt_f = (float)(1.0 / v.dt);
    v.inv_tau_f = (float)(1.0 / d.tau);
    v.c_rad_f = (float)(-4.0 * std::log(2.0) * v.dt);
    v.delta_f = (float)std::sqrt(18.5 * v.dt);
    v.node_i = r.ss->node_i();
    v.node_j = r.ss->node_j();
    v.node_r = r.ss->node_r();
    v.coef_y = inst.cells.as<float4>();
    v.cells = cell_records(inst);
    v.rec0 = (uint32_t)((size_t)(d.n_xi - 1) * (d.n_eta - 1) * sizeof(float4));
    v.rho_f = inst.rho_f.as<float>();
    v.rhox_f = inst.rhox_f.as<float>();
    v.rhoy_f = inst.rhoy_f.as<float>();
    v.xpad_f = r.xpad_f.as<float>();
    v.ypad_f = r.ypad_f.as<float>();
    v.bnd0_f = r.b0f.as<float>();
    v.bnd1_f = r.b1f.as<float>();
    v.rho = inst.rho.as<double>();
    v.rho_xi = inst.rho_xi.as<double>();
    v.rho_eta = inst.rho_eta.as<double>();
    v.xpad = r.xpad.as<double>();
    v.ypad = r.ypad.as<double>();
    v.bnd0 = r.b0.as<double>();
    v.bnd1 = r.b1.as<double>();
    v.x64 = r.x64.as<double>();
    v.y64 = r.y64.as<double>();
    v.partials = r.partials.as<Partial>();
    HIP_TRY(hipMemcpyAsync(r.view.p, &v, sizeof v, hipMemcpyHostToDevice, st));

    // node spans: node-major chunk slots
    std::vector<NodeSpan> spans((size_t)Ms);
    for (int m = 0; m < Ms; ++m) spans[m] = NodeSpan{(uint32_t)((size_t)m * chunks), chunks};
    if (Ms) HIP_TRY(hipMemcpyAsync(r.spans.p, spans.data(), spans.size() * sizeof(NodeSpan), hipMemcpyHostToDevice, st));
    HIP_TRY(msdd::launch_fill_u32(r.steps_total.as<uint32_t>(), 0u, 2, st));

    // FP32 work: every (node, chunk), numbered node-major, so that the waves
    // running at one time share a few neighbouring nodes (L1 locality of the
    // cell gathers)
    r.n_items = fp64 ? 0 : n_part;
    r.next_item = 0;
    r.done_items = 0;
    // the host snapshots are no longer needed once the copies are done
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<double>().swap(r.hx);
    std::vector<double>().swap(r.hy);
    std::vector<double>().swap(r.hb0);
    std::vector<double>().swap(r.hb1);
    return MESH_SDD_OK;
}

void release_request_buffers(Request &r)
{
    for (DevBuf *b : {&r.x64, &r.y64, &r.b0, &r.b1, &r.xpad, &r.ypad, &r.xpad_f, &r.ypad_f, &r.b0f, &r.b1f,
                      &r.view, &r.partials, &r.spans, &r.out, &r.steps_total})
        b->release();
}

// One persistent FP32 launch over the items described by `ranges` (their
// inst fields index `views`).  Caller holds gpu_mu.  Returns the device time
// in ms via *ms.
int run_fp32_launch(mesh_sdd_ctx *ctx, const std::vector<InstView> &views, const std::vector<WorkRange> &ranges,
                    const std::vector<const SampleSet *> &sets, const mesh_sdd_launch &l, double *ms,
                    Arena *arena = nullptr)
{
    hipStream_t st = ctx->stream;
    // launch scratch: the context's grow-only buffers, or pieces of the arena
    DevBuf a_views, a_ranges, a_head, a_jobs, a_ends;
    for (DevBuf *b : {&a_views, &a_ranges, &a_head, &a_jobs, &a_ends}) b->arena = arena;
    DevBuf &views_b = arena ? a_views : ctx->views, &ranges_b = arena ? a_ranges : ctx->ranges;
    DevBuf &head_b = arena ? a_head : ctx->head, &jobs_b = arena ? a_jobs : ctx->jobs;
    DevBuf &ends_b = arena ? a_ends : ctx->ends;
    size_t n_items = 0;
    for (const WorkRange &w : ranges) n_items += w.count;
    if (n_items == 0) {
        *ms = 0.0;
        return MESH_SDD_OK;
    }
    if (n_items > 0xFFFFFFF0u) return fail(MESH_SDD_E_INVAL, "too many work items in one launch");
    uint32_t cap = 64;   // LDS slots per item: the largest chunk of the launch
    for (const WorkRange &w : ranges) cap = std::max(cap, w.chunk_paths);
    cap = (cap + 63u) / 64u * 64u;
    if (views_b.reserve(views.size() * sizeof(InstView)) ||
        ranges_b.reserve(ranges.size() * sizeof(WorkRange)) || head_b.reserve(64))
        return fail(MESH_SDD_E_NOMEM, "device allocation for the work queue failed");
    HIP_TRY(hipMemcpyAsync(views_b.p, views.data(), views.size() * sizeof(InstView), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ranges_b.p, ranges.data(), ranges.size() * sizeof(WorkRange), hipMemcpyHostToDevice, st));
    // A launch that holds one instance whose node tables of rho and dt rho_xi
    // fit the LDS stages them whole (1024-thread workgroups); any other
    // launch stages windows of them, job by job; the waves then keep their
    // items' end states in the context's end-state buffer.  Results are
    // identical to those of the cell-record kernel.
    const int n_nodes = views.size() == 1 && ranges.size() == 1 ? views[0].n_xi * views[0].n_eta : 0;
    int per_cu = 0;
    const int level = table_level(n_nodes, l.monitor_table, &per_cu);
    const int table_grid = ctx->cu_count * per_cu;
    const uint32_t end_waves = (uint32_t)table_grid * (uint32_t)(msdd::kTableBlock / 64);
    if (level > 0 && ends_b.reserve((size_t)end_waves * 6u * cap * sizeof(float)))
        return fail(MESH_SDD_E_NOMEM, "device allocation of the end-state buffer failed");
    // windowed launch: one job per (range, grid block), split so that no job
    // holds more than 1/job_split of a workgroup's share of the items (by
    // default 1/32, and 1/256 in a block of a grid cut into two-field
    // windows: measured on the batched mix, whose 513^2 grids then run 5 %
    // faster; whole-grid windows are refilled for every job, and three-field
    // windows lose with smaller jobs), in block order, cut into per-XCD
    // queues of equal nominal work
    std::vector<msdd::WinJob> jobs;
    msdd::JobQueues qs{};
    size_t win_lds = 32;
    int kind = -2;
    if (level == 3) {
        const size_t share = ((size_t)ctx->cu_count * (size_t)per_cu);
        const size_t split = l.job_split > 0 ? (size_t)l.job_split : 32u;
        const size_t split0 = l.job_split > 0 ? (size_t)l.job_split : 256u;
        const size_t jmax = std::max<size_t>(64, (n_items + share * split - 1) / (share * split));
        const size_t jmax0 = std::max<size_t>(64, (n_items + share * split0 - 1) / (share * split0));
        for (size_t ri = 0; ri < ranges.size(); ++ri) {
            const WorkRange &w = ranges[ri];
            const InstView &v = views[w.inst];
            const int p = msdd::path_kind(v);
            kind = kind == -2 || kind == p ? p : -1;
            const size_t lo = w.first, hi = (size_t)w.first + w.count;
            for (const BlockRun &b : sets[w.inst]->blocks) {
                const size_t qa = std::max(lo, (size_t)b.pos_begin * w.chunks);
                const size_t qb = std::min(hi, (size_t)b.pos_end * w.chunks);
                const bool blocked0 = b.kind == 0 && (b.tw < v.n_xi || b.th < v.n_eta);
                const size_t jm = blocked0 ? jmax0 : jmax;
                for (size_t q = qa; q < qb; q += jm)
                    jobs.push_back(msdd::WinJob{(uint32_t)ri, (uint32_t)q, (uint32_t)std::min(jm, qb - q), b.i0,
                                                b.j0, b.tw, b.th, (uint32_t)b.kind});
                if (qa < qb) win_lds = std::max(win_lds, window_bytes(b.kind, b.tw, b.th));
            }
        }
        std::vector<double> cum(jobs.size() + 1, 0.0);
        for (size_t k = 0; k < jobs.size(); ++k) {
            const WorkRange &w = ranges[jobs[k].range];
            cum[k + 1] = cum[k] + (double)jobs[k].count * w.chunk_paths * views[w.inst].K;
        }
        for (int q = 0, k = 0; q <= msdd::kJobQueues; ++q) {
            const double goal = cum.back() * q / msdd::kJobQueues;
            while (q == msdd::kJobQueues ? k < (int)jobs.size() : (k < (int)jobs.size() && cum[k] < goal)) ++k;
            qs.b[q] = (uint32_t)k;
        }
        if (jobs_b.reserve(std::max<size_t>(1, jobs.size()) * sizeof(msdd::WinJob)))
            return fail(MESH_SDD_E_NOMEM, "device allocation of the job list failed");
        if (!jobs.empty())
            HIP_TRY(hipMemcpyAsync(jobs_b.p, jobs.data(), jobs.size() * sizeof(msdd::WinJob),
                                   hipMemcpyHostToDevice, st));
    }
    TimerEvents ev;
    HIP_TRY(ev.create());
    HIP_TRY(hipEventRecord(ev.e0, st));
    hipError_t le =
        level == 3 ? msdd::launch_paths_fp32_window(views_b.as<InstView>(), ranges_b.as<WorkRange>(),
                                                    jobs_b.as<msdd::WinJob>(), qs, head_b.as<uint32_t>(),
                                                    cap, kind, win_lds, table_grid,
                                                    ends_b.as<float>(), end_waves, (uint32_t)l.refill_lanes,
                                                    (uint32_t)l.max_quarters, st)
        : level > 0 ? msdd::launch_paths_fp32_table(views_b.as<InstView>(), ranges_b.as<WorkRange>(),
                                                    (uint32_t)n_items, head_b.as<uint32_t>(), cap, level,
                                                    msdd::path_kind(views[0]), n_nodes, table_grid,
                                                    ends_b.as<float>(), end_waves, (uint32_t)l.refill_lanes,
                                                    (uint32_t)l.max_quarters, st)
                    : msdd::launch_paths_fp32(views_b.as<InstView>(), ranges_b.as<WorkRange>(),
                                                      (uint32_t)ranges.size(), (uint32_t)n_items,
                                                      head_b.as<uint32_t>(), cap, grid_for(ctx, l, cap), l.block,
                                                      st);
    HIP_TRY(hipEventRecord(ev.e1, st));
    hipError_t se = hipEventSynchronize(ev.e1);
    float t = 0.0f;
    (void)hipEventElapsedTime(&t, ev.e0, ev.e1);
    if (le != hipSuccess) return fail(MESH_SDD_E_DEVICE, "path kernel launch failed: %s", hipGetErrorString(le));
    if (se != hipSuccess) return fail(MESH_SDD_E_DEVICE, "path kernel failed: %s", hipGetErrorString(se));
    *ms = t;
    return MESH_SDD_OK;
}

// Range of request `r`'s items [first, first + count) at launch offset base.
WorkRange range_of(const Request &r, uint32_t slot, size_t base, size_t first, size_t count)
{
    WorkRange w{};
    w.inst = slot;
    w.base = (uint32_t)base;
    w.count = (uint32_t)count;
    w.first = (uint32_t)first;
    w.M = (uint32_t)r.Ms;
    w.chunks = r.chunks_per_node;
    w.chunk_paths = (uint32_t)r.chunk_paths;
    w.N = (uint32_t)r.N;
    return w;
}

// FP64 plain launch of one request.  Caller holds gpu_mu.
int run_fp64_launch(mesh_sdd_ctx *ctx, Request &r, double *ms)
{
    hipStream_t st = ctx->stream;
    TimerEvents ev;
    HIP_TRY(ev.create());
    HIP_TRY(hipEventRecord(ev.e0, st));
    hipError_t le = msdd::launch_paths_fp64(r.view.as<InstView>(), (uint32_t)r.Ms, (uint32_t)r.N,
                                            r.chunks_per_node, r.partials.as<Partial>(), st);
    HIP_TRY(hipEventRecord(ev.e1, st));
    hipError_t se = hipEventSynchronize(ev.e1);
    float t = 0.0f;
    (void)hipEventElapsedTime(&t, ev.e0, ev.e1);
    if (le != hipSuccess) return fail(MESH_SDD_E_DEVICE, "FP64 path kernel launch failed: %s", hipGetErrorString(le));
    if (se != hipSuccess) return fail(MESH_SDD_E_DEVICE, "FP64 path kernel failed: %s", hipGetErrorString(se));
    *ms = t;
    return MESH_SDD_OK;
}

// Finalize (a9) into the request's output buffer, interpolate the nodes
// that ran no paths (a10), and copy the results to the host -- or, when
// `dev_out` is given, straight into its device arrays.
int finalize_request(mesh_sdd_ctx *ctx, Request &r, const mesh_sdd_result *dev_out = nullptr)
{
    hipStream_t st = ctx->stream;
    const mesh_sdd &inst = *r.inst;
    const int M = inst.M;
    double *o = r.out.as<double>();
    HIP_TRY(msdd::launch_finalize(r.partials.as<Partial>(), r.spans.as<NodeSpan>(), r.view.as<InstView>(),
                                  (uint32_t)r.Ms, (uint64_t)r.N, o, o + M, o + 2 * (size_t)M, o + 3 * (size_t)M,
                                  o + 4 * (size_t)M, r.steps_total.as<unsigned long long>(), st));
    if (r.Ms < M) {
        msdd::InterpArgs a{};
        a.n_xi = inst.d.n_xi;
        a.n_eta = inst.d.n_eta;
        a.P_xi = (inst.d.n_xi - 1) / inst.d.sub_xi;
        a.P_eta = (inst.d.n_eta - 1) / inst.d.sub_eta;
        a.per_xi = inst.d.periodic_xi;
        a.per_eta = inst.d.periodic_eta;
        a.stride = r.stride;
        a.M = M;
        a.Lx = inst.d.Lx;
        a.Ly = inst.d.Ly;
        a.node_i = inst.node_ij.as<int32_t>();   // rank order (the node lists are in block order)
        a.node_j = inst.node_ij.as<int32_t>() + M;
        a.rank_of = inst.node_rank.as<int32_t>();
        a.bnd1 = r.b1.as<double>();
        a.mean_x = o;
        a.mean_y = o + M;
        a.se_x = o + 2 * (size_t)M;
        a.se_y = o + 3 * (size_t)M;
        a.exit_frac = o + 4 * (size_t)M;
        HIP_TRY(msdd::launch_interpolate(a, st));
    }
    unsigned long long steps = 0;
    if (dev_out) {
        double *dst[5] = {dev_out->mean_x, dev_out->mean_y, dev_out->se_x, dev_out->se_y, dev_out->exit_frac};
        for (int k = 0; k < 5; ++k)
            if (dst[k] && M)
                HIP_TRY(hipMemcpyAsync(dst[k], o + (size_t)k * M, (size_t)M * sizeof(double), hipMemcpyDeviceToDevice,
                                       st));
    } else {
        r.host_out.resize((size_t)5 * M);
        if (M) HIP_TRY(hipMemcpyAsync(r.host_out.data(), o, r.host_out.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipMemcpyAsync(&steps, r.steps_total.p, sizeof steps, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    r.executed_steps = steps;
    return MESH_SDD_OK;
}

int copy_result(mesh_sdd_ctx *ctx, const Request &r, mesh_sdd_result *res)
{
    if (!res) return MESH_SDD_OK;
    if (res->struct_size != sizeof(mesh_sdd_result))
        return fail(MESH_SDD_E_INVAL, "result.struct_size %u != %zu", res->struct_size, sizeof(mesh_sdd_result));
    const int M = r.M;   // the instance may already be destroyed
    double *dst[5] = {res->mean_x, res->mean_y, res->se_x, res->se_y, res->exit_frac};
    for (int k = 0; k < 5; ++k) {
        if (!dst[k]) continue;
        const double *src = r.host_out.data() + (size_t)k * M;
        if (res->outputs_on_device) {
            std::lock_guard<std::mutex> g(ctx->gpu_mu);
            HIP_TRY(hipMemcpy(dst[k], src, (size_t)M * sizeof(double), hipMemcpyHostToDevice));
        } else if (M) {
            std::memcpy(dst[k], src, (size_t)M * sizeof(double));
        }
    }
    res->executed_path_steps = r.executed_steps;
    res->paths_per_node = r.N;
    res->device_ms = r.device_ms;
    return MESH_SDD_OK;
}

// Blocking path of one or several requests: FP32 ones share ONE launch.
int run_blocking(mesh_sdd_ctx *ctx, std::vector<std::shared_ptr<Request>> &reqs,
                 const std::vector<const mesh_sdd_step *> &dev_steps, std::vector<int> &status)
{
    std::lock_guard<std::mutex> g(ctx->gpu_mu);
    status.assign(reqs.size(), MESH_SDD_OK);
    std::vector<InstView> views;
    std::vector<WorkRange> ranges;
    std::vector<const SampleSet *> sets;
    std::vector<size_t> fp32_reqs;
    size_t base = 0;
    // one persistent launch over the FP32 requests gathered so far: the
    // bucket's shape for a launch of one instance, the multi-instance shape
    // otherwise
    auto launch_group = [&]() {
        if (fp32_reqs.empty()) return;
        double ms = 0.0;
        const mesh_sdd_launch l = launch_for_group(ctx, fp32_reqs.size() == 1 ? &reqs[fp32_reqs[0]]->inst->d : nullptr);
        int rc = run_fp32_launch(ctx, views, ranges, sets, l, &ms);
        for (size_t q : fp32_reqs) {
            Request &r = *reqs[q];
            int rq = rc;
            if (rq == MESH_SDD_OK) rq = finalize_request(ctx, r);
            r.device_ms = ms;
            status[q] = rq;
            if (rq != MESH_SDD_OK) r.error = g_last_error;
        }
        views.clear();
        ranges.clear();
        sets.clear();
        fp32_reqs.clear();
        base = 0;
    };
    for (size_t q = 0; q < reqs.size(); ++q) {
        Request &r = *reqs[q];
        int rc = stage_request(r, dev_steps[q]);
        if (rc != MESH_SDD_OK) {
            status[q] = rc;
            r.error = g_last_error;
            continue;
        }
        if (r.inst->d.precision == MESH_SDD_FP64) {
            double ms = 0.0;
            rc = run_fp64_launch(ctx, r, &ms);
            if (rc == MESH_SDD_OK) rc = finalize_request(ctx, r);
            r.device_ms = ms;
            status[q] = rc;
            if (rc != MESH_SDD_OK) r.error = g_last_error;
        } else {
            // a launch numbers its items in 32 bits: start another one first
            // where this request's items would not fit (every request fits
            // alone, stage_request checks it)
            if (base + r.n_items > (size_t)kMaxLaunchItems) launch_group();
            const uint32_t slot = (uint32_t)views.size();
            views.push_back(r.v);
            sets.push_back(r.ss);
            if (r.n_items) {
                ranges.push_back(range_of(r, slot, base, 0, r.n_items));
                base += r.n_items;
            }
            fp32_reqs.push_back(q);
        }
    }
    launch_group();
    for (auto &r : reqs) release_request_buffers(*r);
    for (int s : status)
        if (s != MESH_SDD_OK) return s;
    return MESH_SDD_OK;
}

// Autotuning: a candidate wins only if it is this much faster per path-step
// (timings of one launch repeat to a few tenths of a percent).
constexpr double kTuneMargin = 0.005;

// Tune the bucket of `inst` (grid size, periodicity) by timing launches of
// `inst` alone at a reduced path count, one knob at a time; the winner goes
// to ctx->tuned.  The context's override is used for the timings and then
// restored.
int tune_bucket(mesh_sdd *inst, const mesh_sdd_step &step, int64_t N, mesh_sdd_launch *out)
{
    mesh_sdd_ctx *ctx = inst->ctx;
    const mesh_sdd_desc &d = inst->d;
    const TuneKey key{d.n_xi, d.n_eta, d.periodic_xi, d.periodic_eta};
    // about 6e9 nominal path-steps per timing (~20 ms of kernel)
    const int32_t Ms = step.interface_stride > 1 ? (int32_t)sampled_ranks(*inst, (int)step.interface_stride).size()
                                                 : inst->M;
    int64_t Nt = (int64_t)(6.0e9 / std::max(1.0, (double)Ms * d.K));
    Nt = std::min<int64_t>(N, std::max<int64_t>(256, (Nt + 63) / 64 * 64));
    mesh_sdd_step s = step;
    s.target_se = 0.0;
    s.paths_per_node = Nt;
    bool saved_override;
    mesh_sdd_launch saved_l;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        saved_override = ctx->has_override;
        saved_l = ctx->override_launch;
    }
    auto timeit = [&](const mesh_sdd_launch &l, double *ms_per_step) -> int {
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->override_launch = l;
            ctx->has_override = true;
        }
        std::vector<std::shared_ptr<Request>> reqs{make_request(inst, s, Nt)};
        std::vector<const mesh_sdd_step *> ds{s.inputs_on_device ? &s : nullptr};
        std::vector<int> st;
        InflightHold hold;
        hold.add(inst);
        const int rc = run_blocking(ctx, reqs, ds, st);
        if (rc == MESH_SDD_OK)
            *ms_per_step = reqs[0]->device_ms / std::max<double>(1.0, (double)reqs[0]->executed_steps);
        return rc;
    };
    mesh_sdd_launch best = launch_for(ctx, d);
    best.monitor_table = 0;
    double best_t = 0.0, t = 0.0;
    int rc = timeit(best, &t);   // warm-up: the first launch of a shape also builds its node lists
    if (rc == MESH_SDD_OK) rc = timeit(best, &best_t);
    // knobs that matter for this bucket
    int per_cu = 0;
    const int level = table_level(d.n_xi * d.n_eta, 0, &per_cu);
    std::vector<std::pair<int32_t mesh_sdd_launch::*, std::vector<int32_t>>> knobs;
    knobs.push_back({&mesh_sdd_launch::chunk_paths, {64, 128, 256}});
    if (level == 3) {
        const bool whole = window_bytes(0, d.n_xi, d.n_eta) <= msdd::kWinBytes;
        if (!whole) {
            knobs.push_back({&mesh_sdd_launch::window_kind, {1, 2}});
            knobs.push_back({&mesh_sdd_launch::window_margin, {0, 20, 30, 38, 45, 55}});
        }
        knobs.push_back({&mesh_sdd_launch::job_split, {8, 32, 128, 256, 1024}});
    }
    knobs.push_back({&mesh_sdd_launch::refill_lanes, {48, 56, 60}});
    knobs.push_back({&mesh_sdd_launch::max_quarters, {8, 16, 32}});
    for (size_t k = 0; k < knobs.size() && rc == MESH_SDD_OK; ++k)
        for (int32_t v : knobs[k].second) {
            if (best.*(knobs[k].first) == v) continue;
            mesh_sdd_launch c = best;
            c.*(knobs[k].first) = v;
            if (knobs[k].first == &mesh_sdd_launch::window_kind) c.window_margin = 0;   // the kind's own default
            if (knobs[k].first == &mesh_sdd_launch::window_margin) {
                // margins that leave a block of at least 8 nodes in the window
                const Layout lay = layout_of(d, c);
                int wx = 0, wy = 0;
                window_dims(lay.kind, d.n_xi, d.n_eta, &wx, &wy);
                if (std::min(wx, wy) - 2 * lay.margin < 8) continue;
            }
            rc = timeit(c, &t);
            if (rc != MESH_SDD_OK) break;
            if (t < best_t * (1.0 - kTuneMargin)) {
                best = c;
                best_t = t;
            }
        }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->has_override = saved_override;
        ctx->override_launch = saved_l;
        if (rc == MESH_SDD_OK) ctx->tuned[key] = best;
    }
    if (rc != MESH_SDD_OK) return rc;
    *out = best;
    return MESH_SDD_OK;
}

// Range checks of a launch shape given by a caller (0 = default allowed).
int check_launch(const mesh_sdd_launch *l)
{
    if (l->struct_size != sizeof(mesh_sdd_launch))
        return fail(MESH_SDD_E_INVAL, "launch.struct_size %u != %zu", l->struct_size, sizeof(mesh_sdd_launch));
    if (l->block != 0 && l->block != 64 && l->block != 128 && l->block != 256 && l->block != 512)
        return fail(MESH_SDD_E_INVAL, "block must be 64, 128, 256 or 512");
    if (l->waves_per_simd < 0 || l->waves_per_simd > 8)
        return fail(MESH_SDD_E_INVAL, "waves_per_simd must be in [0, 8]");
    const int chunk = l->chunk_paths ? l->chunk_paths : 128;
    if (chunk < 64 || chunk % 64 || chunk > 2048 ||
        msdd::paths_fp32_lds_bytes(l->block ? l->block : 256, (uint32_t)chunk) > kLdsBytes)
        return fail(MESH_SDD_E_INVAL, "chunk_paths must be a multiple of 64 in [64, 2048] and fit in LDS");
    if (l->monitor_table != 0 && l->monitor_table != 1)
        return fail(MESH_SDD_E_INVAL, "launch.monitor_table must be 0 or 1");
    if (l->refill_lanes < 0 || l->refill_lanes > 64) return fail(MESH_SDD_E_INVAL, "refill_lanes must be in [0, 64]");
    if (l->max_quarters < 0 || l->max_quarters > 64) return fail(MESH_SDD_E_INVAL, "max_quarters must be in [0, 64]");
    if (l->window_kind < 0 || l->window_kind > 2) return fail(MESH_SDD_E_INVAL, "window_kind must be 0, 1 or 2");
    if (l->window_margin < 0 || l->window_margin > 64)
        return fail(MESH_SDD_E_INVAL, "window_margin must be in [0, 64]");
    if (l->job_split < 0 || l->job_split > 4096) return fail(MESH_SDD_E_INVAL, "job_split must be in [0, 4096]");
    return MESH_SDD_OK;
}

// ---------------------------------------------------------------------------
// Serving scheduler: admission by HBM budget, chunk-granularity ticks.
// ---------------------------------------------------------------------------
constexpr double kTickPathSteps = 6.0e9;   // work per tick, ~tens of ms at full rate

// Ends a request (ctx->mu held by the caller).  Never throws: a request that
// left the running list must end, or its waiters and its instance's
// destroy would wait for ever.
void finish_request(mesh_sdd_ctx *ctx, const std::shared_ptr<Request> &r, int status, const std::string &err) noexcept
{
    r->status = status;
    try {
        r->error = err;
    } catch (...) {   // the status alone then tells the caller
    }
    r->finished = true;
    r->t_done = Clock::now();
    if (r->admitted) ctx->in_use -= std::min(ctx->in_use, r->cost_bytes);
    r->inst->inflight.fetch_sub(1);
    if (status == MESH_SDD_OK) {
        ++ctx->completed;
        ctx->executed += r->executed_steps;
        try {
            ctx->latencies.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
        } catch (...) {   // the latency is left out of the percentiles
        }
    } else if (status == MESH_SDD_E_CANCELLED) {
        ++ctx->cancelled;
    } else {
        ++ctx->failed;
    }
    ctx->done_cv.notify_all();
}

void scheduler_loop(mesh_sdd_ctx *ctx)
{
    (void)hipSetDevice(ctx->device);
    for (;;) {
        try {
            std::vector<std::shared_ptr<Request>> to_admit;
            {
                std::unique_lock<std::mutex> lk(ctx->mu);
                ctx->cv.wait(lk, [&] { return ctx->stop || !ctx->queue.empty() || !ctx->running.empty(); });
                if (ctx->stop) break;
                // admission in arrival order while the budget allows
                while (!ctx->queue.empty()) {
                    auto &r = ctx->queue.front();
                    if (ctx->in_use + r->cost_bytes > ctx->budget && !ctx->running.empty()) break;
                    to_admit.reserve(to_admit.size() + 1);   // the only allocations, before any state changes
                    ctx->running.reserve(ctx->running.size() + 1);
                    ctx->in_use += r->cost_bytes;
                    r->admitted = true;
                    to_admit.push_back(r);
                    ctx->running.push_back(r);
                    ctx->queue.pop_front();
                    if (ctx->in_use > ctx->budget) break;   // a lone request over budget never reaches here
                }
            }
            // stage newly admitted requests (FP64 ones run whole, here)
            for (auto &r : to_admit) {
                int rc;
                double ms = 0.0;
                {
                    std::lock_guard<std::mutex> g(ctx->gpu_mu);
                    rc = stage_request(*r, nullptr);
                    if (rc == MESH_SDD_OK && r->inst->d.precision == MESH_SDD_FP64) {
                        rc = run_fp64_launch(ctx, *r, &ms);
                        if (rc == MESH_SDD_OK) rc = finalize_request(ctx, *r);
                        r->device_ms = ms;
                        release_request_buffers(*r);
                    }
                }
                // FP32 requests without work (no interface node) finish at once
                const bool empty_fp32 = rc == MESH_SDD_OK && r->inst->d.precision == MESH_SDD_FP32 && r->n_items == 0;
                if (empty_fp32) {
                    std::lock_guard<std::mutex> g(ctx->gpu_mu);
                    rc = finalize_request(ctx, *r);
                    release_request_buffers(*r);
                }
                std::lock_guard<std::mutex> lk(ctx->mu);
                ctx->busy_ms += ms;
                if (rc != MESH_SDD_OK || r->inst->d.precision == MESH_SDD_FP64 || empty_fp32) {
                    const std::string msg = rc == MESH_SDD_OK ? std::string() : g_last_error;   // may throw: first
                    ctx->running.erase(std::find(ctx->running.begin(), ctx->running.end(), r));
                    if (rc != MESH_SDD_OK) release_request_buffers(*r);
                    finish_request(ctx, r, rc, msg);
                }
            }
            // build one tick over the running FP32 requests: a fair share of the
            // tick's work for each, at least one item each
            std::vector<InstView> views;
            std::vector<WorkRange> ranges;
            std::vector<const SampleSet *> sets;
            std::vector<std::pair<std::shared_ptr<Request>, size_t>> taken;
            mesh_sdd_launch l = default_launch();
            {
                std::lock_guard<std::mutex> lk(ctx->mu);
                size_t active = 0;
                for (auto &r : ctx->running)
                    if (r->next_item < r->n_items) ++active;
                if (active == 0) continue;
                const double share = kTickPathSteps / (double)active;
                size_t base = 0;
                for (auto &r : ctx->running) {
                    if (r->next_item >= r->n_items) continue;
                    const double per_item = (double)r->chunk_paths * (double)r->inst->d.K;
                    size_t take = (size_t)std::max(1.0, share / per_item);
                    take = std::min(take, r->n_items - r->next_item);
                    const uint32_t slot = (uint32_t)views.size();
                    views.push_back(r->v);
                    sets.push_back(r->ss);
                    ranges.push_back(range_of(*r, slot, base, r->next_item, take));
                    base += take;
                    r->next_item += take;
                    taken.emplace_back(r, take);
                }
                ++ctx->ticks;
            }
            // a tick of one request takes its bucket's shape, else the
            // multi-instance shape (launch_for_group takes ctx->mu itself)
            l = launch_for_group(ctx, taken.size() == 1 ? &taken.front().first->inst->d : nullptr);
            double ms = 0.0;
            int rc;
            {
                std::lock_guard<std::mutex> g(ctx->gpu_mu);
                rc = run_fp32_launch(ctx, views, ranges, sets, l, &ms);
            }
            std::string err = rc == MESH_SDD_OK ? std::string() : g_last_error;
            std::vector<std::shared_ptr<Request>> complete;
            {
                std::lock_guard<std::mutex> lk(ctx->mu);
                ctx->busy_ms += ms;
                for (auto &t : taken) {
                    t.first->done_items += t.second;
                    t.first->device_ms += ms;
                    if (rc != MESH_SDD_OK || t.first->done_items == t.first->n_items) complete.push_back(t.first);
                }
            }
            for (auto &r : complete) {
                int fr = rc;
                if (fr == MESH_SDD_OK) {
                    std::lock_guard<std::mutex> g(ctx->gpu_mu);
                    fr = finalize_request(ctx, *r);
                }
                std::string e2 = fr == MESH_SDD_OK ? std::string() : (rc != MESH_SDD_OK ? err : g_last_error);
                {
                    std::lock_guard<std::mutex> g(ctx->gpu_mu);
                    release_request_buffers(*r);
                }
                std::lock_guard<std::mutex> lk(ctx->mu);
                ctx->running.erase(std::find(ctx->running.begin(), ctx->running.end(), r));
                finish_request(ctx, r, fr, e2);
            }
        } catch (...) {
            // a host resource ran out inside the tick: the requests that were
            // running end with the error; queued ones wait for the next tick
            (void)abi_exception();
            const std::string err = g_last_error;
            std::vector<std::shared_ptr<Request>> left;
            {
                std::lock_guard<std::mutex> lk(ctx->mu);
                left.swap(ctx->running);
            }
            {
                std::lock_guard<std::mutex> g(ctx->gpu_mu);
                for (auto &r : left) release_request_buffers(*r);
            }
            std::lock_guard<std::mutex> lk(ctx->mu);
            for (auto &r : left) finish_request(ctx, r, MESH_SDD_E_NOMEM, err);
        }
    }
    // cancel whatever is left (buffers are freed without holding ctx->mu)
    std::vector<std::shared_ptr<Request>> left;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto &r : ctx->queue) finish_request(ctx, r, MESH_SDD_E_CANCELLED, "context destroyed");
        ctx->queue.clear();
        left.swap(ctx->running);
    }
    {
        std::lock_guard<std::mutex> g(ctx->gpu_mu);
        for (auto &r : left) release_request_buffers(*r);
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto &r : left) finish_request(ctx, r, MESH_SDD_E_CANCELLED, "context destroyed");
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *mesh_sdd_last_error(void) { return g_last_error.c_str(); }

const char *mesh_sdd_version(void) { return "mesh_sdd 0.1 (gfx950)"; }

int mesh_sdd_ctx_create(int device, size_t hbm_budget_bytes, void *hip_stream, mesh_sdd_ctx **out)
try {
    if (!out) return fail(MESH_SDD_E_INVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(MESH_SDD_E_INVAL, "device %d not in [0, %d)", device, count);
    HIP_TRY(hipSetDevice(device));
    auto ctx = std::make_unique<mesh_sdd_ctx>();
    ctx->device = device;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    ctx->cu_count = prop.multiProcessorCount;
    // the no-allocation solve's scratch array: its address on this device,
    // looked up once with the device current (a failure is reported by that
    // solve, not here)
    (void)msdd_rt::scratch_resolve(device);
    if (hip_stream) {
        ctx->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        HIP_TRY(hipStreamCreate(&ctx->stream));   // blocking: ordered after legacy default-stream work
        ctx->own_stream = true;
    }
    if (hbm_budget_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        HIP_TRY(hipMemGetInfo(&free_b, &total_b));
        hbm_budget_bytes = free_b / 10 * 9;
    }
    ctx->budget = hbm_budget_bytes;
    mesh_sdd_ctx *raw = ctx.get();
    try {
        raw->worker = std::thread(scheduler_loop, raw);
    } catch (...) {
        if (raw->own_stream) (void)hipStreamDestroy(raw->stream);
        return fail(MESH_SDD_E_NOMEM, "could not start the scheduler thread");
    }
    *out = ctx.release();
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_ctx_destroy(mesh_sdd_ctx *ctx)
try {
    if (!ctx) return fail(MESH_SDD_E_INVAL, "ctx is NULL");
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->n_instances > 0) return fail(MESH_SDD_E_STATE, "%d instances still alive", ctx->n_instances);
        ctx->stop = true;
    }
    ctx->cv.notify_all();
    if (ctx->worker.joinable()) ctx->worker.join();
    (void)hipSetDevice(ctx->device);
    ctx->head.release();
    ctx->views.release();
    ctx->ranges.release();
    ctx->jobs.release();
    ctx->ends.release();
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_ctx_stats(mesh_sdd_ctx *ctx, mesh_sdd_stats *out)
try {
    if (!ctx || !out) return fail(MESH_SDD_E_INVAL, "NULL argument");
    if (out->struct_size != sizeof(mesh_sdd_stats))
        return fail(MESH_SDD_E_INVAL, "stats.struct_size %u != %zu", out->struct_size, sizeof(mesh_sdd_stats));
    std::lock_guard<std::mutex> lk(ctx->mu);
    out->submitted = ctx->submitted;
    out->completed = ctx->completed;
    out->failed = ctx->failed;
    out->cancelled = ctx->cancelled;
    out->queued = ctx->queue.size();
    out->running = ctx->running.size();
    out->ticks = ctx->ticks;
    out->hbm_in_use = ctx->in_use;
    out->hbm_budget = ctx->budget;
    out->busy_ms = ctx->busy_ms;
    out->executed_path_steps = ctx->executed;
    std::vector<double> lat = ctx->latencies;
    if (lat.empty()) {
        out->p50_ms = out->p99_ms = out->mean_ms = 0.0;
    } else {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double q) {
            const double pos = q * (double)(lat.size() - 1);
            const size_t a = (size_t)pos;
            const size_t b = std::min(a + 1, lat.size() - 1);
            return lat[a] + (pos - (double)a) * (lat[b] - lat[a]);
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        double s = 0.0;
        for (double x : lat) s += x;
        out->mean_ms = s / (double)lat.size();
    }
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_set_launch(mesh_sdd_ctx *ctx, const mesh_sdd_launch *launch)
try {
    if (!ctx) return fail(MESH_SDD_E_INVAL, "ctx is NULL");
    if (!launch) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->has_override = false;
        return MESH_SDD_OK;
    }
    int rc = check_launch(launch);
    if (rc != MESH_SDD_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->override_launch = with_defaults(*launch);
    ctx->has_override = true;
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_get_launch(mesh_sdd *inst, mesh_sdd_launch *out)
try {
    if (!inst || !out) return fail(MESH_SDD_E_INVAL, "NULL argument");
    *out = launch_for(inst->ctx, inst->d);
    if (out->waves_per_simd == 0) {
        const int per_cu = msdd::paths_fp32_blocks_per_cu(out->block, (uint32_t)out->chunk_paths);
        out->waves_per_simd = per_cu * (out->block / 64) / 4;
    }
    int per_cu = 0;
    out->table_level = table_level(inst->d.n_xi * inst->d.n_eta, out->monitor_table, &per_cu);
    const Layout lay = layout_of(inst->d, *out);
    out->window_kind = lay.kind ? 2 : 1;
    out->window_margin = lay.margin;
    if (out->job_split == 0) {
        int wx = 0, wy = 0;
        window_dims(lay.kind, inst->d.n_xi, inst->d.n_eta, &wx, &wy);
        out->job_split = lay.kind == 0 && (wx < inst->d.n_xi || wy < inst->d.n_eta) ? 256 : 32;
    }
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_desc_check(const mesh_sdd_desc *desc) { return validate_desc(desc); }

int mesh_sdd_desc_interface_nodes(const mesh_sdd_desc *desc, int32_t *i, int32_t *j)
try {
    int rc = validate_desc(desc);
    if (rc != MESH_SDD_OK) return rc;
    std::vector<int32_t> ni, nj;
    enumerate_nodes(*desc, ni, nj);
    if (ni.size() > 0x7FFFFFFFu) return fail(MESH_SDD_E_INVAL, "too many interface nodes");
    if (i && j && !ni.empty()) {
        std::memcpy(i, ni.data(), ni.size() * 4);
        std::memcpy(j, nj.data(), nj.size() * 4);
    }
    return (int)ni.size();
} catch (...) {
    return abi_exception();
}

int mesh_sdd_desc_work_order(const mesh_sdd_desc *desc, uint32_t interface_stride, int32_t *ranks, int32_t *blocks,
                             int32_t max_blocks, int32_t *n_blocks)
try {
    int rc = validate_desc(desc);
    if (rc != MESH_SDD_OK) return rc;
    rc = check_stride(*desc, interface_stride);
    if (rc != MESH_SDD_OK) return rc;
    if (blocks && (max_blocks < 0 || !n_blocks)) return fail(MESH_SDD_E_INVAL, "blocks given without room or count");
    mesh_sdd tmp;   // host fields only: no device memory is touched
    tmp.d = *desc;
    enumerate_nodes(tmp.d, tmp.node_i, tmp.node_j);
    if (tmp.node_i.size() > 0x7FFFFFFFu) return fail(MESH_SDD_E_INVAL, "too many interface nodes");
    tmp.M = (int32_t)tmp.node_i.size();
    std::vector<int32_t> order = sampled_ranks(tmp, interface_stride > 1 ? (int)interface_stride : 1);
    std::vector<BlockRun> runs;
    order_by_blocks(tmp, layout_of(*desc, default_launch()), order, runs);
    if (ranks && !order.empty()) std::memcpy(ranks, order.data(), order.size() * 4);
    if (n_blocks) *n_blocks = (int32_t)runs.size();
    if (blocks) {
        if ((size_t)max_blocks < runs.size())
            return fail(MESH_SDD_E_INVAL, "%zu blocks, room for %d", runs.size(), max_blocks);
        for (size_t k = 0; k < runs.size(); ++k) {
            const BlockRun &b = runs[k];
            const int32_t rec[7] = {b.pos_begin, b.pos_end, b.i0, b.j0, b.tw, b.th, b.kind};
            std::memcpy(blocks + 7 * k, rec, sizeof rec);
        }
    }
    return (int)order.size();
} catch (...) {
    return abi_exception();
}

int mesh_sdd_create(mesh_sdd_ctx *ctx, const mesh_sdd_desc *desc, mesh_sdd **out)
try {
    if (!ctx || !out) return fail(MESH_SDD_E_INVAL, "NULL argument");
    *out = nullptr;
    int rc = validate_desc(desc);
    if (rc != MESH_SDD_OK) return rc;
    auto inst = std::make_unique<mesh_sdd>();
    inst->ctx = ctx;
    inst->d = *desc;
    enumerate_nodes(inst->d, inst->node_i, inst->node_j);
    inst->M = (int32_t)inst->node_i.size();
    inst->resident_bytes = instance_bytes(inst->d, inst->M);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (inst->resident_bytes > ctx->budget)
            return fail(MESH_SDD_E_BUDGET, "instance tables (%zu B) exceed the HBM budget (%zu B)",
                        inst->resident_bytes, ctx->budget);
    }
    const size_t n = (size_t)desc->n_xi * desc->n_eta;
    const size_t cells = (size_t)(desc->n_xi - 1) * (desc->n_eta - 1);
    std::lock_guard<std::mutex> g(ctx->gpu_mu);
    HIP_TRY(hipSetDevice(ctx->device));
    if (inst->rho_in.alloc(n * 8) || inst->rho.alloc(n * 8) || inst->rho_xi.alloc(n * 8) ||
        inst->rho_eta.alloc(n * 8) || inst->rho_f.alloc(n * 4) || inst->rhox_f.alloc(n * 4) ||
        inst->rhoy_f.alloc(n * 4) ||
        inst->cells.alloc(cells * 4 * sizeof(float4)) ||
        inst->node_rank.alloc(n * 4) || inst->node_ij.alloc(std::max<size_t>(1, 2 * (size_t)inst->M) * 4))
        return fail(MESH_SDD_E_NOMEM, "device allocation for the instance tables failed");
    {
        std::vector<int32_t> rank(n, -1);
        for (int32_t r = 0; r < inst->M; ++r) rank[(size_t)inst->node_j[r] * desc->n_xi + inst->node_i[r]] = r;
        HIP_TRY(hipMemcpy(inst->node_rank.p, rank.data(), n * 4, hipMemcpyHostToDevice));
        if (inst->M) {
            HIP_TRY(hipMemcpy(inst->node_ij.p, inst->node_i.data(), (size_t)inst->M * 4, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(inst->node_ij.as<int32_t>() + inst->M, inst->node_j.data(), (size_t)inst->M * 4,
                              hipMemcpyHostToDevice));
        }
    }
    const SampleSet *all = nullptr;
    rc = sample_set(*inst, 1, layout_of(inst->d, launch_for(ctx, inst->d)), &all);
    if (rc != MESH_SDD_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->in_use += inst->resident_bytes;
        ++ctx->n_instances;
    }
    *out = inst.release();
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_destroy(mesh_sdd *inst)
try {
    if (!inst) return fail(MESH_SDD_E_INVAL, "instance is NULL");
    if (inst->inflight.load() > 0) return fail(MESH_SDD_E_STATE, "instance has requests in flight");
    mesh_sdd_ctx *ctx = inst->ctx;
    const size_t bytes = inst->resident_bytes;
    {
        std::lock_guard<std::mutex> g(ctx->gpu_mu);
        (void)hipSetDevice(ctx->device);
        delete inst;   // DevBuf destructors free the tables
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->in_use -= std::min(ctx->in_use, bytes);
    --ctx->n_instances;
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_set_monitor(mesh_sdd *inst, const double *rho, int is_device_ptr)
try {
    if (!inst || !rho) return fail(MESH_SDD_E_INVAL, "NULL argument");
    const mesh_sdd_desc &d = inst->d;
    const size_t n = (size_t)d.n_xi * d.n_eta;
    if (!is_device_ptr) {
        for (size_t k = 0; k < n; ++k)
            if (!(rho[k] > 0.0) || !std::isfinite(rho[k]))
                return fail(MESH_SDD_E_INVAL, "monitor value %zu is not a positive finite number", k);
    }
    if (inst->inflight.load() > 0) return fail(MESH_SDD_E_STATE, "instance has requests in flight");
    mesh_sdd_ctx *ctx = inst->ctx;
    std::lock_guard<std::mutex> g(ctx->gpu_mu);
    hipStream_t st = ctx->stream;
    HIP_TRY(hipMemcpyAsync(inst->rho_in.p, rho, n * 8, is_device_ptr ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    return msdd_rt::install_monitor(inst, st);
} catch (...) {
    return abi_exception();
}

int mesh_sdd_num_interface_nodes(const mesh_sdd *inst)
try {
    if (!inst) return fail(MESH_SDD_E_INVAL, "instance is NULL");
    return inst->M;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_interface_nodes(const mesh_sdd *inst, int32_t *i, int32_t *j)
try {
    if (!inst) return fail(MESH_SDD_E_INVAL, "instance is NULL");
    if (inst->M && (!i || !j)) return fail(MESH_SDD_E_INVAL, "output array is NULL");
    if (inst->M) {
        std::memcpy(i, inst->node_i.data(), (size_t)inst->M * 4);
        std::memcpy(j, inst->node_j.data(), (size_t)inst->M * 4);
    }
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_solve_batch(mesh_sdd *const *insts, const mesh_sdd_step *steps, mesh_sdd_result *results,
                         int32_t count, int32_t *status)
try {
    if (count < 0 || (count > 0 && (!insts || !steps || !results))) return fail(MESH_SDD_E_INVAL, "bad batch arguments");
    if (count == 0) return MESH_SDD_OK;
    mesh_sdd_ctx *ctx = insts[0] ? insts[0]->ctx : nullptr;
    if (!ctx) return fail(MESH_SDD_E_INVAL, "instance is NULL");
    std::vector<std::shared_ptr<Request>> reqs;
    std::vector<const mesh_sdd_step *> dev_steps;
    std::vector<int> st((size_t)count, MESH_SDD_OK);
    int first_err = MESH_SDD_OK;
    std::string first_msg;
    std::vector<int> idx;
    InflightHold hold;
    for (int32_t q = 0; q < count; ++q) {
        mesh_sdd *inst = insts[q];
        int rc = MESH_SDD_OK;
        int64_t N = 0;
        if (!inst) rc = fail(MESH_SDD_E_INVAL, "instance %d is NULL", q);
        else if (inst->ctx != ctx) rc = fail(MESH_SDD_E_INVAL, "instance %d belongs to another context", q);
        else if (!inst->monitor_set) rc = fail(MESH_SDD_E_STATE, "set_monitor not called on instance %d", q);
        else if (results[q].struct_size != sizeof(mesh_sdd_result)) rc = fail(MESH_SDD_E_INVAL, "result.struct_size mismatch");
        if (rc == MESH_SDD_OK) rc = validate_step(*inst, &steps[q], &N);
        if (rc != MESH_SDD_OK) {
            st[q] = rc;
            if (first_err == MESH_SDD_OK) {
                first_err = rc;
                first_msg = g_last_error;
            }
            continue;
        }
        hold.add(inst);
        reqs.push_back(make_request(inst, steps[q], N));
        dev_steps.push_back(steps[q].inputs_on_device ? &steps[q] : nullptr);
        idx.push_back(q);
    }
    std::vector<int> rst;
    int rc = reqs.empty() ? MESH_SDD_OK : run_blocking(ctx, reqs, dev_steps, rst);
    if (rc != MESH_SDD_OK && first_err == MESH_SDD_OK) {
        first_err = rc;
        first_msg = g_last_error;
    }
    for (size_t k = 0; k < reqs.size(); ++k) {
        const int q = idx[k];
        st[q] = rst[k];
        if (rst[k] == MESH_SDD_OK) {
            int c = copy_result(ctx, *reqs[k], &results[q]);
            if (c != MESH_SDD_OK) {
                st[q] = c;
                if (first_err == MESH_SDD_OK) {
                    first_err = c;
                    first_msg = g_last_error;
                }
            }
        }
    }
    if (status)
        for (int32_t q = 0; q < count; ++q) status[q] = st[q];
    if (first_err != MESH_SDD_OK) g_last_error = first_msg;
    return first_err;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_solve_interfaces(mesh_sdd *inst, const mesh_sdd_step *step, mesh_sdd_result *result)
try {
    if (!inst || !result) return fail(MESH_SDD_E_INVAL, "NULL argument");
    int32_t st = 0;
    mesh_sdd *one[1] = {inst};
    return mesh_sdd_solve_batch(one, step, result, 1, &st);
} catch (...) {
    return abi_exception();
}

int mesh_sdd_solve_interfaces_noalloc(mesh_sdd *inst, const mesh_sdd_step *step, mesh_sdd_result *result)
try {
    if (!inst || !step || !result) return fail(MESH_SDD_E_INVAL, "NULL argument");
    if (!inst->monitor_set) return fail(MESH_SDD_E_STATE, "set_monitor not called");
    if (result->struct_size != sizeof(mesh_sdd_result))
        return fail(MESH_SDD_E_INVAL, "result.struct_size %u != %zu", result->struct_size, sizeof(mesh_sdd_result));
    int64_t N = 0;
    int rc = validate_step(*inst, step, &N);
    if (rc != MESH_SDD_OK) return rc;
    if (!step->inputs_on_device) return fail(MESH_SDD_E_INVAL, "the no-allocation solve takes device inputs");
    if (!result->outputs_on_device) return fail(MESH_SDD_E_INVAL, "the no-allocation solve takes device outputs");
    mesh_sdd_ctx *ctx = inst->ctx;
    const mesh_sdd_desc &d = inst->d;
    auto r = make_request(inst, *step, N);
    void *base = nullptr;
    std::mutex *use = nullptr;
    rc = msdd_rt::scratch_region(ctx->device, &base, &use);
    if (rc != MESH_SDD_OK) return rc;
    std::lock_guard<std::mutex> su(*use);   // one user of the device's array at a time
    std::lock_guard<std::mutex> g(ctx->gpu_mu);
    auto set = inst->samples.end();
    for (auto s = inst->samples.begin(); s != inst->samples.end(); ++s)
        if (std::get<0>(s->first) == r->stride) set = s;
    if (set == inst->samples.end())
        return fail(MESH_SDD_E_STATE, "interface stride %d: its node lists are built by the first allocating solve "
                    "with that stride", r->stride);
    // the scratch this call carves, counted as stage_request and the launch
    // carve it (each piece rounded to 256 bytes); the job list by its bound
    // of one job per 64 items plus one per grid block
    const bool fp64 = d.precision == MESH_SDD_FP64;
    const size_t n = (size_t)d.n_xi * d.n_eta, np = (size_t)(d.n_xi + 2) * (d.n_eta + 2);
    const size_t nb = 4 * (size_t)d.n_eta + 4 * (size_t)d.n_xi;
    const size_t chunks = fp64 ? (size_t)((N + msdd::kFp64Block - 1) / msdd::kFp64Block)
                               : (size_t)((N + r->chunk_paths - 1) / r->chunk_paths);
    const size_t n_items = (size_t)r->Ms * chunks;
    auto piece = [](size_t b) { return b == 0 ? (size_t)256 : round_up(b, 256); };
    size_t need = 2 * piece(n * 8) + 2 * piece(nb * 8) + 2 * piece(np * 8) + 2 * piece(np * 4) + 2 * piece(nb * 4) +
                  piece(sizeof(InstView)) + piece(n_items * sizeof(Partial)) +
                  piece((size_t)r->Ms * sizeof(NodeSpan)) + piece((size_t)5 * inst->M * sizeof(double)) + piece(8);
    if (!fp64) {
        const mesh_sdd_launch l = launch_for(ctx, d);
        int per_cu = 0;
        const int level = table_level((int)n, l.monitor_table, &per_cu);
        const size_t cap = (size_t)(r->chunk_paths + 63) / 64 * 64;
        need += piece(sizeof(InstView)) + piece(sizeof(WorkRange)) + piece(64);
        if (level > 0) need += piece((size_t)ctx->cu_count * per_cu * (msdd::kTableBlock / 64) * 6 * cap * 4);
        size_t nb_max = 0;   // the most blocks of any layout of the stride
        for (auto s = inst->samples.begin(); s != inst->samples.end(); ++s)
            if (std::get<0>(s->first) == r->stride) nb_max = std::max(nb_max, s->second->blocks.size());
        if (level == 3) need += piece((n_items / 64 + nb_max + 1) * sizeof(msdd::WinJob));
    }
    if (need > msdd_rt::scratch_capacity())
        return fail(MESH_SDD_E_INVAL, "the solve needs %zu bytes of scratch, more than the %zu of the no-allocation "
                    "solve (fewer paths per node, a smaller grid or an interface stride)", need,
                    msdd_rt::scratch_capacity());
    Arena arena;
    arena.base = static_cast<char *>(base);
    arena.size = msdd_rt::scratch_capacity();
    InflightHold hold;
    hold.add(inst);
    rc = stage_request(*r, step, &arena);
    double ms = 0.0;
    if (rc == MESH_SDD_OK) {
        if (fp64) {
            rc = run_fp64_launch(ctx, *r, &ms);
        } else {
            std::vector<InstView> views{r->v};
            std::vector<WorkRange> ranges;
            std::vector<const SampleSet *> sets{r->ss};
            if (r->n_items) ranges.push_back(range_of(*r, 0, 0, 0, r->n_items));
            rc = run_fp32_launch(ctx, views, ranges, sets, launch_for(ctx, d), &ms, &arena);
        }
    }
    if (rc == MESH_SDD_OK) rc = finalize_request(ctx, *r, result);
    release_request_buffers(*r);   // frees nothing: every piece is the arena's
    if (rc != MESH_SDD_OK) return rc;
    result->executed_path_steps = r->executed_steps;
    result->paths_per_node = r->N;
    result->device_ms = ms;
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_submit(mesh_sdd *inst, const mesh_sdd_step *step, mesh_sdd_ticket *ticket)
try {
    if (!inst || !ticket) return fail(MESH_SDD_E_INVAL, "NULL argument");
    if (!inst->monitor_set) return fail(MESH_SDD_E_STATE, "set_monitor not called");
    int64_t N = 0;
    int rc = validate_step(*inst, step, &N);
    if (rc != MESH_SDD_OK) return rc;
    mesh_sdd_ctx *ctx = inst->ctx;
    auto r = make_request(inst, *step, N);
    if (step->inputs_on_device) {
        // snapshot device inputs to the host so the caller may reuse them at once
        const size_t n = (size_t)inst->d.n_xi * inst->d.n_eta;
        const size_t nb = 4 * (size_t)inst->d.n_eta + 4 * (size_t)inst->d.n_xi;
        r->hx.resize(n);
        r->hy.resize(n);
        r->hb0.resize(nb);
        r->hb1.resize(nb);
        std::lock_guard<std::mutex> g(ctx->gpu_mu);
        HIP_TRY(hipMemcpy(r->hx.data(), step->x_cur, n * 8, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(r->hy.data(), step->y_cur, n * 8, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(r->hb0.data(), step->bnd_t0, nb * 8, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(r->hb1.data(), step->bnd_t1, nb * 8, hipMemcpyDeviceToHost));
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->stop) return fail(MESH_SDD_E_CANCELLED, "context is shutting down");
        if (r->cost_bytes > ctx->budget)
            return fail(MESH_SDD_E_BUDGET, "request needs %zu B, budget is %zu B", r->cost_bytes, ctx->budget);
        r->ticket = ctx->next_ticket++;
        r->t_submit = Clock::now();
        ctx->tickets[r->ticket] = r;
        try {
            ctx->queue.push_back(r);
        } catch (...) {
            ctx->tickets.erase(r->ticket);
            throw;
        }
        inst->inflight.fetch_add(1);   // released by finish_request
        ++ctx->submitted;
        *ticket = r->ticket;
    }
    ctx->cv.notify_all();
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

static int poll_impl(mesh_sdd_ctx *ctx, mesh_sdd_ticket ticket, mesh_sdd_result *result, int64_t timeout_ms)
{
    if (!ctx) return fail(MESH_SDD_E_INVAL, "ctx is NULL");
    std::shared_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(ctx->mu);
        auto it = ctx->tickets.find(ticket);
        if (it == ctx->tickets.end()) return fail(MESH_SDD_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
        r = it->second;
        if (!r->finished && timeout_ms != 0) {
            auto pred = [&] { return r->finished; };
            if (timeout_ms < 0)
                ctx->done_cv.wait(lk, pred);
            else
                ctx->done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
        }
        if (!r->finished) return MESH_SDD_PENDING;
        ctx->tickets.erase(it);
    }
    if (r->status != MESH_SDD_OK) return fail(r->status, "%s", r->error.c_str());
    return copy_result(ctx, *r, result);
}

int mesh_sdd_poll(mesh_sdd_ctx *ctx, mesh_sdd_ticket ticket, mesh_sdd_result *result)
try {
    return poll_impl(ctx, ticket, result, 0);
} catch (...) {
    return abi_exception();
}

int mesh_sdd_wait(mesh_sdd_ctx *ctx, mesh_sdd_ticket ticket, mesh_sdd_result *result, int64_t timeout_ms)
try {
    return poll_impl(ctx, ticket, result, timeout_ms);
} catch (...) {
    return abi_exception();
}

int mesh_sdd_cancel(mesh_sdd_ctx *ctx, mesh_sdd_ticket ticket)
try {
    if (!ctx) return fail(MESH_SDD_E_INVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return fail(MESH_SDD_E_INVAL, "unknown ticket");
    auto r = it->second;
    if (r->finished) return fail(MESH_SDD_E_STATE, "request already finished");
    auto q = std::find(ctx->queue.begin(), ctx->queue.end(), r);
    if (q == ctx->queue.end()) return fail(MESH_SDD_E_STATE, "request is already running");
    ctx->queue.erase(q);
    finish_request(ctx, r, MESH_SDD_E_CANCELLED, "cancelled");
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_autotune(mesh_sdd *inst, const mesh_sdd_step *step, mesh_sdd_launch *out)
try {
    if (!inst || !step) return fail(MESH_SDD_E_INVAL, "NULL argument");
    if (!inst->monitor_set) return fail(MESH_SDD_E_STATE, "set_monitor not called");
    if (inst->d.precision != MESH_SDD_FP32) return fail(MESH_SDD_E_INVAL, "autotuning applies to the FP32 kernels");
    int64_t N = 0;
    int rc = validate_step(*inst, step, &N);
    if (rc != MESH_SDD_OK) return rc;
    mesh_sdd_launch best{};
    rc = tune_bucket(inst, *step, N, &best);
    if (rc != MESH_SDD_OK) return rc;
    if (out) *out = best;
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_autotune_batch(mesh_sdd *const *insts, const mesh_sdd_step *steps, int32_t count, int32_t scale_down,
                            mesh_sdd_launch *out)
try {
    if (count <= 0 || !insts || !steps || scale_down < 1) return fail(MESH_SDD_E_INVAL, "bad batch arguments");
    mesh_sdd_ctx *ctx = insts[0] ? insts[0]->ctx : nullptr;
    if (!ctx) return fail(MESH_SDD_E_INVAL, "instance is NULL");
    std::vector<int64_t> Ns((size_t)count);
    for (int32_t q = 0; q < count; ++q) {
        mesh_sdd *inst = insts[q];
        if (!inst || inst->ctx != ctx) return fail(MESH_SDD_E_INVAL, "instance %d is NULL or of another context", q);
        if (!inst->monitor_set) return fail(MESH_SDD_E_STATE, "set_monitor not called on instance %d", q);
        if (inst->d.precision != MESH_SDD_FP32) return fail(MESH_SDD_E_INVAL, "instance %d is not FP32", q);
        int rc = validate_step(*inst, &steps[q], &Ns[(size_t)q]);
        if (rc != MESH_SDD_OK) return rc;
    }
    // 1. each bucket on its first instance
    std::map<TuneKey, int32_t> first;
    for (int32_t q = 0; q < count; ++q) {
        const mesh_sdd_desc &d = insts[q]->d;
        first.emplace(TuneKey{d.n_xi, d.n_eta, d.periodic_xi, d.periodic_eta}, q);
    }
    for (auto &kv : first) {
        mesh_sdd_launch b{};
        int rc = tune_bucket(insts[kv.second], steps[kv.second], Ns[(size_t)kv.second], &b);
        if (rc != MESH_SDD_OK) return rc;
    }
    // 2. the launch-wide knobs on the whole batch at reduced path counts
    std::vector<mesh_sdd_step> small(steps, steps + count);
    for (int32_t q = 0; q < count; ++q) {
        small[(size_t)q].target_se = 0.0;
        small[(size_t)q].paths_per_node = std::max<int64_t>(64, Ns[(size_t)q] / scale_down / 64 * 64);
    }
    bool saved_has;
    mesh_sdd_launch saved;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        saved_has = ctx->has_batch_tuned;
        saved = ctx->batch_tuned;
    }
    auto time_batch = [&](const mesh_sdd_launch &l, double *ms_per_step) -> int {
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->batch_tuned = l;
            ctx->has_batch_tuned = true;
        }
        std::vector<std::shared_ptr<Request>> reqs;
        std::vector<const mesh_sdd_step *> ds;
        InflightHold hold;
        for (int32_t q = 0; q < count; ++q) {
            reqs.push_back(make_request(insts[q], small[(size_t)q], small[(size_t)q].paths_per_node));
            ds.push_back(small[(size_t)q].inputs_on_device ? &small[(size_t)q] : nullptr);
            hold.add(insts[q]);
        }
        std::vector<int> st;
        const int rc = run_blocking(ctx, reqs, ds, st);
        if (rc != MESH_SDD_OK) return rc;
        double ms = 0.0, steps_done = 0.0;
        for (auto &r : reqs) steps_done += (double)r->executed_steps;
        ms = reqs.empty() ? 0.0 : reqs[0]->device_ms;   // one launch: the same device time for each
        *ms_per_step = ms / std::max(1.0, steps_done);
        return MESH_SDD_OK;
    };
    mesh_sdd_launch best = saved_has ? with_defaults(saved) : default_launch();
    double best_t = 0.0, t = 0.0;
    int rc = time_batch(best, &t);   // warm-up
    if (rc == MESH_SDD_OK) rc = time_batch(best, &best_t);
    const std::vector<std::pair<int32_t mesh_sdd_launch::*, std::vector<int32_t>>> knobs = {
        {&mesh_sdd_launch::job_split, {8, 32, 128, 256, 1024}},
        {&mesh_sdd_launch::refill_lanes, {48, 56, 60}},
        {&mesh_sdd_launch::max_quarters, {8, 16, 32}},
    };
    for (size_t k = 0; k < knobs.size() && rc == MESH_SDD_OK; ++k)
        for (int32_t v : knobs[k].second) {
            if (best.*(knobs[k].first) == v) continue;
            mesh_sdd_launch c = best;
            c.*(knobs[k].first) = v;
            rc = time_batch(c, &t);
            if (rc != MESH_SDD_OK) break;
            if (t < best_t * (1.0 - kTuneMargin)) {
                best = c;
                best_t = t;
            }
        }
    // 3. the per-bucket knobs that act inside the batch -- chunk size, and the
    // window margin of grids no window holds whole -- re-timed on the whole
    // batch: a bucket tuned alone at a reduced path count can prefer a shape
    // that the batch does not (measured: 64-path chunks on the 513^2 grids,
    // 4 % slower in the batched mix than 128)
    for (auto &kv : first) {
        if (rc != MESH_SDD_OK) break;
        const TuneKey key = kv.first;
        const mesh_sdd_desc &d = insts[kv.second]->d;
        const bool blocked = window_bytes(0, d.n_xi, d.n_eta) > msdd::kWinBytes;
        std::vector<std::pair<int32_t mesh_sdd_launch::*, std::vector<int32_t>>> bk = {
            {&mesh_sdd_launch::chunk_paths, {64, 128, 256}}};
        if (blocked) bk.push_back({&mesh_sdd_launch::window_margin, {0, 30, 38, 45}});
        for (size_t k = 0; k < bk.size() && rc == MESH_SDD_OK; ++k)
            for (int32_t v : bk[k].second) {
                mesh_sdd_launch cur;
                {
                    std::lock_guard<std::mutex> lk(ctx->mu);
                    cur = ctx->tuned[key];
                }
                if (cur.*(bk[k].first) == v) continue;
                mesh_sdd_launch cand = cur;
                cand.*(bk[k].first) = v;
                {
                    std::lock_guard<std::mutex> lk(ctx->mu);
                    ctx->tuned[key] = cand;
                }
                rc = time_batch(best, &t);
                const bool keep = rc == MESH_SDD_OK && t < best_t * (1.0 - kTuneMargin);
                if (keep) best_t = t;
                std::lock_guard<std::mutex> lk(ctx->mu);
                if (!keep) ctx->tuned[key] = cur;
                if (rc != MESH_SDD_OK) break;
            }
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (rc == MESH_SDD_OK) {
            ctx->batch_tuned = best;
            ctx->has_batch_tuned = true;
        } else {
            ctx->batch_tuned = saved;
            ctx->has_batch_tuned = saved_has;
        }
    }
    if (rc != MESH_SDD_OK) return rc;
    if (out) *out = best;
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_tune_save(mesh_sdd_ctx *ctx, const char *path)
try {
    if (!ctx || !path) return fail(MESH_SDD_E_INVAL, "NULL argument");
    std::string text = "# mesh_sdd tuned launch shapes: key n_xi n_eta per_xi per_eta chunk_paths refill_lanes "
                       "max_quarters window_kind window_margin job_split\n";
    char line[256];
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto &kv : ctx->tuned) {
            const mesh_sdd_launch &l = kv.second;
            std::snprintf(line, sizeof line, "bucket %d %d %d %d %d %d %d %d %d %d\n", kv.first.n_xi, kv.first.n_eta,
                          kv.first.per_xi, kv.first.per_eta, l.chunk_paths, l.refill_lanes, l.max_quarters,
                          l.window_kind, l.window_margin, l.job_split);
            text += line;
        }
        if (ctx->has_batch_tuned) {
            const mesh_sdd_launch &l = ctx->batch_tuned;
            std::snprintf(line, sizeof line, "batch 0 0 0 0 %d %d %d %d %d %d\n", l.chunk_paths, l.refill_lanes,
                          l.max_quarters, l.window_kind, l.window_margin, l.job_split);
            text += line;
        }
    }
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(MESH_SDD_E_INVAL, "cannot write %s", path);
    const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
    if (std::fclose(f) != 0 || !ok) return fail(MESH_SDD_E_INVAL, "cannot write %s", path);
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_tune_load(mesh_sdd_ctx *ctx, const char *path)
try {
    if (!ctx || !path) return fail(MESH_SDD_E_INVAL, "NULL argument");
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(MESH_SDD_E_INVAL, "cannot read %s", path);
    std::vector<std::pair<TuneKey, mesh_sdd_launch>> buckets;
    bool have_batch = false;
    mesh_sdd_launch batch{};
    char buf[512];
    int lineno = 0, rc = MESH_SDD_OK;
    while (std::fgets(buf, sizeof buf, f)) {
        ++lineno;
        if (buf[0] == '#' || buf[0] == '\n') continue;
        char key[16];
        int v[10];
        if (std::sscanf(buf, "%15s %d %d %d %d %d %d %d %d %d %d", key, &v[0], &v[1], &v[2], &v[3], &v[4], &v[5],
                        &v[6], &v[7], &v[8], &v[9]) != 11) {
            rc = fail(MESH_SDD_E_INVAL, "%s:%d: expected a key and ten integers", path, lineno);
            break;
        }
        mesh_sdd_launch l = default_launch();
        l.chunk_paths = v[4];
        l.refill_lanes = v[5];
        l.max_quarters = v[6];
        l.window_kind = v[7];
        l.window_margin = v[8];
        l.job_split = v[9];
        rc = check_launch(&l);
        if (rc != MESH_SDD_OK) {
            rc = fail(MESH_SDD_E_INVAL, "%s:%d: %s", path, lineno, g_last_error.c_str());
            break;
        }
        if (std::strcmp(key, "bucket") == 0) {
            buckets.emplace_back(TuneKey{v[0], v[1], v[2], v[3]}, with_defaults(l));
        } else if (std::strcmp(key, "batch") == 0) {
            have_batch = true;
            batch = with_defaults(l);
        } else {
            rc = fail(MESH_SDD_E_INVAL, "%s:%d: unknown key '%s'", path, lineno, key);
            break;
        }
    }
    std::fclose(f);
    if (rc != MESH_SDD_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto &b : buckets) ctx->tuned[b.first] = b.second;
    if (have_batch) {
        ctx->batch_tuned = batch;
        ctx->has_batch_tuned = true;
    }
    return MESH_SDD_OK;
} catch (...) {
    return abi_exception();
}

int mesh_sdd_debug_paths(mesh_sdd *inst, const mesh_sdd_step *step, int32_t node_rank, int64_t p_begin, int64_t p_end,
                         double *vx, double *vy, int32_t *exited, int32_t *side, int32_t *steps, double *trace)
try {
    if (!inst || !step || !vx || !vy || !exited || !side || !steps) return fail(MESH_SDD_E_INVAL, "NULL argument");
    if (!inst->monitor_set) return fail(MESH_SDD_E_STATE, "set_monitor not called");
    if (node_rank < 0 || node_rank >= inst->M) return fail(MESH_SDD_E_INVAL, "node rank %d outside [0, %d)", node_rank, inst->M);
    if (p_begin < 0 || p_end < p_begin || p_end > ((int64_t)1 << 31) || p_end - p_begin > (1 << 20))
        return fail(MESH_SDD_E_INVAL, "path range [%lld, %lld) invalid", (long long)p_begin, (long long)p_end);
    int64_t N = 0;
    int rc = validate_step(*inst, step, &N);
    if (rc != MESH_SDD_OK) return rc;
    mesh_sdd_ctx *ctx = inst->ctx;
    const uint32_t count = (uint32_t)(p_end - p_begin);
    mesh_sdd_step full = *step;
    full.interface_stride = 0;   // node_rank indexes the full node lists
    auto r = make_request(inst, full, std::max<int64_t>(1, count));
    std::lock_guard<std::mutex> g(ctx->gpu_mu);
    InflightHold hold;
    hold.add(inst);
    rc = stage_request(*r, step->inputs_on_device ? step : nullptr);
    DevBuf dvx, dvy, dex, dsd, dst, dtr;
    if (rc == MESH_SDD_OK && count) {
        const size_t trace_n = trace ? (size_t)count * 4 * inst->d.K : 0;
        if (dvx.alloc(count * 8) || dvy.alloc(count * 8) || dex.alloc(count * 4) || dsd.alloc(count * 4) ||
            dst.alloc(count * 4) || (trace && dtr.alloc(trace_n * 8))) {
            rc = fail(MESH_SDD_E_NOMEM, "device allocation failed");
        } else {
            hipStream_t s = ctx->stream;
            hipError_t e = hipSuccess;
            if (trace) e = hipMemcpyAsync(dtr.p, trace, trace_n * 8, hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = msdd::launch_debug_paths(r->view.as<InstView>(), inst->d.precision == MESH_SDD_FP64,
                                             (uint32_t)r->ss->pos_of_rank[(size_t)node_rank], (uint32_t)p_begin,
                                             count, dvx.as<double>(),
                                             dvy.as<double>(), dex.as<int32_t>(), dsd.as<int32_t>(),
                                             dst.as<int32_t>(), trace ? dtr.as<double>() : nullptr, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e == hipSuccess) e = hipMemcpy(vx, dvx.p, count * 8, hipMemcpyDeviceToHost);
            if (e == hipSuccess) e = hipMemcpy(vy, dvy.p, count * 8, hipMemcpyDeviceToHost);
            if (e == hipSuccess) e = hipMemcpy(exited, dex.p, count * 4, hipMemcpyDeviceToHost);
            if (e == hipSuccess) e = hipMemcpy(side, dsd.p, count * 4, hipMemcpyDeviceToHost);
            if (e == hipSuccess) e = hipMemcpy(steps, dst.p, count * 4, hipMemcpyDeviceToHost);
            if (e == hipSuccess && trace) e = hipMemcpy(trace, dtr.p, trace_n * 8, hipMemcpyDeviceToHost);
            if (e != hipSuccess) rc = fail(MESH_SDD_E_DEVICE, "debug path kernel failed: %s", hipGetErrorString(e));
        }
    }
    release_request_buffers(*r);
    return rc;
} catch (...) {
    return abi_exception();
}

}  // extern "C"
