// Device-visible records shared by the host runtime and the HIP kernels of
// the interface-node Monte-Carlo solver (paper section 3.4-3.6).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msdd {

// The work of one request inside one launch of the batched kernel.  A
// request's work items are numbered node-major (item = node * chunks + c):
// item q covers paths [c * chunk_paths, min(N, (c + 1) * chunk_paths)) of
// node q div chunks, with c = q mod chunks, and its sums go to partial slot
// q itself.  Concurrent waves then work on a few neighbouring nodes, whose
// paths visit the same cells, so the cell gathers hit in the L1 cache.  The range holds the request's items
// [first, first + count), which are items [base, base + count) of the launch.
struct WorkRange {
    uint32_t inst;         // InstView slot in the launch
    uint32_t base;         // first launch-wide item of the range
    uint32_t count;        // items in the range
    uint32_t first;        // first request-wide item
    uint32_t M;            // interface nodes of the request
    uint32_t chunks;       // chunks per node
    uint32_t chunk_paths;  // paths per full chunk
    uint32_t N;            // paths per node
};

// One job of the windowed kernel: the request-wide items [q0, q0 + count)
// of range `range`, whose nodes all lie in one block of the grid, and the
// window of the node tables that the workgroup stages in LDS for them:
// nodes [i0, i0 + tw) x [j0, j0 + th), inside the grid.  kind 0: the window
// holds (rho, dt rho_xi) per node (8 B); kind 1: also dt rho_eta per node
// (4 B each, after the pairs).
struct WinJob {
    uint32_t range;
    uint32_t q0;
    uint32_t count;
    int32_t i0, j0, tw, th;
    uint32_t kind;
};

// The job list of a windowed launch cut into kJobQueues contiguous queues:
// queue x holds jobs [b[x], b[x + 1]).  Workgroup w serves queue w mod
// kJobQueues first -- workgroups are dealt round-robin to the 8 XCDs, so each
// XCD's L2 caches the tables of one region of the job list -- and takes jobs
// from the following queues once its own is empty.
constexpr int kJobQueues = 8;
struct JobQueues {
    uint32_t b[kJobQueues + 1];
};

// Shifted sums of one (node, chunk): S1 = sum(v - v_ref), S2 = sum((v - v_ref)^2).
struct Partial {
    double s1x, s2x, s1y, s2y;
    unsigned long long exits;
    unsigned long long steps;
};

// One problem instance as the kernels see it.  All pointers are device
// addresses owned by the instance.  Grids are row-major [n_eta][n_xi].
struct InstView {
    int32_t n_xi, n_eta;          // nodes per axis
    int32_t per_xi, per_eta;      // periodic flags
    int32_t K;                    // substeps
    int32_t bridge;               // Brownian-bridge test: 0 off, 1 on, 2 on with substeps up to 4e-3
    int32_t M;                    // nodes that run paths (entries of node_i / node_j / node_r)
    int32_t pad0;
    uint32_t key0, key1;          // Philox key (seed low / high word)
    uint32_t ctr3;                // instance_id << 16 | mesh_step & 0xffff
    uint32_t rec0;                // byte offset of `cells` from `coef_y` (one allocation)
    double Lx, Ly, tau, dt;       // extents, mesh step, substep
    float Lx_f, Ly_f, dt_f, sq2dt_f, inv_dt_f, inv_tau_f;
    float c_rad_f;                // -4 ln2 dt
    float delta_f;                // sqrt(18.5 dt)

    // The nodes that run paths, in order: grid indices and interface rank.
    // The rank is the node's random-stream identity and its result slot, so
    // a node's estimate does not depend on which other nodes run.  All
    // interface nodes (node_r[k] = k) unless the step subsamples them.
    const int32_t *node_i, *node_j;
    const uint32_t *node_r;

    // FP32 path: per-cell records of three float4, (n_xi-1)(n_eta-1) cells:
    // (rho, dt rho_xi) at the corners 00, 10, then 01, 11, then dt rho_eta
    // at 00, 10, 01, 11; dt rho_eta again as a compact plane in difference
    // form, e00, e10 - e00, e01, e11 - e01 (coef_y, read by the kernels that
    // take rho and dt rho_xi alone from LDS), in the same
    // allocation ahead of the records (cells = coef_y + rec0 bytes); the FP32
    // node tables of rho, dt rho_xi and dt rho_eta [n_eta][n_xi] (the same
    // corner values, staged in LDS whole by launches that hold this instance
    // alone when they fit, else in windows); padded
    // mesh [n_eta+2][n_xi+2] with ghost /
    // wrapped values, origin at node (-1, -1); boundary arrays in the C-ABI
    // layout.
    const float4 *cells, *coef_y;
    const float *rho_f, *rhox_f, *rhoy_f;
    const float *xpad_f, *ypad_f;
    const float *bnd0_f, *bnd1_f;

    // FP64 path: node tables rho, rho_xi, rho_eta; padded mesh; boundary.
    const double *rho, *rho_xi, *rho_eta;
    const double *xpad, *ypad;
    const double *bnd0, *bnd1;

    // FP64 mesh at t^n (for the reference values of the shifted sums).
    const double *x64, *y64;

    // Partial sums of this request's work items.
    Partial *partials;
};

// The FP32 path kernels' compile-time kind of an instance: its periodicity
// (per_xi + 2 per_eta) plus 4 where the bridge test must take all four sides
// (bridge on with substeps above 4e-3 and some axis Dirichlet); the kernels
// take the nearer side of each Dirichlet axis alone otherwise.
__host__ __device__ inline int path_kind(int per_xi, int per_eta, int bridge)
{
    return per_xi + 2 * per_eta + (bridge == 1 && !(per_xi && per_eta) ? 4 : 0);
}
__host__ __device__ inline int path_kind(const InstView &v) { return path_kind(v.per_xi, v.per_eta, v.bridge); }

// Per-node finalize descriptor: the partials of one node are
// partials[first .. first + count) in chunk order.
struct NodeSpan {
    uint32_t first;
    uint32_t count;
};

// Interpolation of the interface nodes that ran no paths (section 3.6,
// equispaced sampling with stride `stride` along every interface line).
// Result arrays have one entry per interface rank; the estimated entries
// are read, the others written.
struct InterpArgs {
    int32_t n_xi, n_eta;          // nodes per axis
    int32_t P_xi, P_eta;          // subdomain cells per axis
    int32_t per_xi, per_eta;      // periodic flags
    int32_t stride;               // > 1
    int32_t M;                    // interface nodes
    double Lx, Ly;                // quasi-periodic offsets
    const int32_t *node_i, *node_j;   // all interface nodes in rank order
    const int32_t *rank_of;           // [n_eta][n_xi]: interface rank or -1
    const double *bnd1;               // boundary arrays at t^{n+1} (C-ABI layout)
    double *mean_x, *mean_y, *se_x, *se_y, *exit_frac;
};

}  // namespace msdd
