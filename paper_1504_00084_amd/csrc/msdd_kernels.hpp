// Host-callable launchers of the HIP kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "msdd_device.hpp"

namespace msdd {

// a0: finite-difference gradient of the frozen monitor (section 3.4) into
// FP64 node tables; on a periodic axis node n-1 receives node 0's values.
hipError_t launch_prep_gradient(const double *rho_in, int n_xi, int n_eta, int per_xi, int per_eta,
                                double *rho, double *rho_xi, double *rho_eta, hipStream_t s);

// a0 (FP32 path): per-cell records of three float4: (rho, s rho_xi) at the
// corners 00, 10, then 01, 11, then s rho_eta at 00, 10, 01, 11, with s =
// grad_scale (the substep dt); coef_y gets s rho_eta of every cell again, as
// a compact plane, in difference form: e00, e10 - e00, e01, e11 - e01.
hipError_t launch_prep_cells(const double *rho, const double *rho_xi, const double *rho_eta, int n_xi,
                             int n_eta, double grad_scale, float4 *cells, float4 *coef_y, hipStream_t s);

// a7 set-up: padded mesh [n_eta+2][n_xi+2] (ghost rows / columns by Keys'
// rule on Dirichlet axes, wrapped with quasi-periodic offsets on periodic
// axes) in FP64 and FP32, for x (offset Lx along xi) and y (Ly along eta).
hipError_t launch_prep_mesh(const double *x, const double *y, int n_xi, int n_eta, int per_xi, int per_eta,
                            double Lx, double Ly, double *xpad, double *ypad, float *xpad_f, float *ypad_f,
                            hipStream_t s);

hipError_t launch_to_f32(const double *in, float *out, size_t n, hipStream_t s);
// out = (float)(scale * in), elementwise (the FP32 node table of dt rho_xi).
hipError_t launch_scaled_to_f32(const double *in, double scale, float *out, size_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t s);

// a2-a8, FP32: persistent batched kernel over a work queue of n_items items
// described by n_ranges ranges (sorted by base, contiguous from 0).  `head`
// is the queue counter (zeroed by this launcher).
// `cap` >= every range's chunk_paths: each wave holds two items' per-path
// end states in LDS (6 * cap words per wave).
hipError_t launch_paths_fp32(const InstView *insts, const WorkRange *ranges, uint32_t n_ranges, uint32_t n_items,
                             uint32_t *head, uint32_t cap, int grid, int block, hipStream_t s);
size_t paths_fp32_lds_bytes(int block, uint32_t cap);

// The same kernel for a launch that holds ONE instance (n_ranges = 1): each
// 1024-thread workgroup (16 waves, 4 per SIMD) copies that instance's FP32
// node tables of rho and dt rho_xi into LDS, interleaved (level 2, the only
// level; n_nodes * 8 bytes), and reads those corner values there instead of
// from the cell records; `ends` holds the waves' item end
// states (6 * cap floats per wave, room for `end_waves` >= grid * 16 waves).
// Results are identical to launch_paths_fp32's.
constexpr int kTableBlock = 1024;
size_t paths_fp32_table_lds_bytes(int level, int n_nodes);
// `kind` = path_kind of the instance, 0..6 (compiled in).
// refill_lanes, max_quarters (1..64): a wave leaves its stepping loop for the
// refill once fewer than refill_lanes of its lanes have a path in flight, or
// after max_quarters groups of four substeps (no result depends on them).
hipError_t launch_paths_fp32_table(const InstView *insts, const WorkRange *ranges, uint32_t n_items, uint32_t *head,
                                   uint32_t cap, int level, int kind, int n_nodes, int grid, float *ends,
                                   uint32_t end_waves, uint32_t refill_lanes, uint32_t max_quarters, hipStream_t s);
int paths_fp32_table_blocks_per_cu(int level, int n_nodes);

// The windowed form for launches whose tables do not fit the LDS whole (many
// instances, or one large grid): `jobs` lists qs.b[kJobQueues] jobs (items of
// one range whose nodes lie in one grid block, and the node-table window
// around that block), cut into kJobQueues queues; each 1024-thread workgroup
// pops jobs from its queue and then the others (`head`: kJobQueues counters,
// zeroed here), stages the job's window in LDS -- (rho, dt rho_xi) per node,
// 8 bytes, and for kind-1 jobs dt rho_eta per node too, 4 bytes -- and runs
// its items; lanes outside the window
// read the cell records.  `lds` = the largest window of the launch in bytes
// (at most kWinBytes).  `kind` = path_kind shared by every instance of the
// launch (compiled in), or -1 (each job runs the loop of its instance's).  `ends`,
// refill_lanes and max_quarters as for the table kernel.  Results are
// identical to launch_paths_fp32's.
constexpr size_t kWinBytes = 156800;   // LDS of one window (of the 160 KB of a CU)
constexpr int kWinNodes = 19600;       // two-field windows: at most 140 x 140 nodes
constexpr int kWin3Side = 114;         // three-field windows: at most 114 x 114 nodes when square
hipError_t launch_paths_fp32_window(const InstView *insts, const WorkRange *ranges, const WinJob *jobs,
                                    const JobQueues &qs, uint32_t *head, uint32_t cap, int kind, size_t lds,
                                    int grid, float *ends, uint32_t end_waves, uint32_t refill_lanes,
                                    uint32_t max_quarters, hipStream_t s);
int paths_fp32_window_blocks_per_cu(size_t lds);

// a2-a8, FP64 plain: one thread per path, one launch per instance; the
// partial of (node, chunk) goes to partials[node * chunks + chunk].
hipError_t launch_paths_fp64(const InstView *inst, uint32_t M, uint32_t n_paths, uint32_t chunks_per_node,
                             Partial *partials, hipStream_t s);
constexpr int kFp64Block = 256;

// a9: fixed-order combine of each node's partials; mean, SE, exit fraction,
// written at the node's interface rank (inst->node_r).
hipError_t launch_finalize(const Partial *partials, const NodeSpan *spans, const InstView *inst, uint32_t M,
                           uint64_t n_paths, double *mean_x, double *mean_y, double *se_x, double *se_y,
                           double *exit_frac, unsigned long long *steps_total, hipStream_t s);

// a10 (subsampled steps): every interface node that ran no paths takes
// the Keys cubic interpolant along its interface line of the estimates at
// the multiples of the stride, the boundary values at t^{n+1} where the
// line meets a Dirichlet side (with Keys' end rule beyond it) and the
// periodic images across a seam; its standard error is that of the same
// combination of independent estimates, its exit fraction NaN.
hipError_t launch_interpolate(const InterpArgs &a, hipStream_t s);

// Diagnostics: one path per thread with the FP32 or FP64 path arithmetic.
hipError_t launch_debug_paths(const InstView *inst, int fp64, uint32_t node, uint32_t p_begin, uint32_t count,
                              double *vx, double *vy, int32_t *exited, int32_t *side, int32_t *steps,
                              double *trace, hipStream_t s);

// Occupancy of the FP32 kernel: resident workgroups per CU for `block` and
// LDS capacity `cap`.
int paths_fp32_blocks_per_cu(int block, uint32_t cap);
// Register / LDS usage of the FP32 kernel for `block` (for reports).
int paths_fp32_attributes(int block, int *vgprs, int *sgprs, int *lds_bytes);

}  // namespace msdd
