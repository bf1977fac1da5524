// Stand-ins for the HIP kernel launchers (kernels.hip, mesh_step.hip) and the
// static scratch of the no-allocation solve (noalloc.hip), for the host-only
// sanitizer builds of the library's runtime.  TEST INFRASTRUCTURE ONLY: they
// compute nothing of the method; they write the outputs the host code reads
// back (zeros, a monitor of ones, a quality ratio of one) so that every host
// code path runs to its end.
#include <atomic>
#include <cstdlib>
#include <mutex>

#include "msdd_kernels.hpp"
#include "msdd_mesh_step.hpp"
#include "runtime_internal.hpp"

namespace msdd {

hipError_t launch_prep_gradient(const double *rho_in, int n_xi, int n_eta, int, int, double *rho, double *rho_xi,
                                double *rho_eta, hipStream_t)
{
    const size_t n = (size_t)n_xi * n_eta;
    for (size_t k = 0; k < n; ++k) {
        rho[k] = rho_in[k];
        rho_xi[k] = rho_eta[k] = 0.0;
    }
    return hipSuccess;
}
hipError_t launch_prep_cells(const double *, const double *, const double *, int n_xi, int n_eta, double,
                             float4 *cells, float4 *coef_y, hipStream_t)
{
    const size_t c = (size_t)(n_xi - 1) * (n_eta - 1);
    std::memset(coef_y, 0, c * sizeof(float4));
    std::memset(cells, 0, 3 * c * sizeof(float4));
    return hipSuccess;
}
hipError_t launch_prep_mesh(const double *, const double *, int n_xi, int n_eta, int, int, double, double,
                            double *xpad, double *ypad, float *xpad_f, float *ypad_f, hipStream_t)
{
    const size_t n = (size_t)(n_xi + 2) * (n_eta + 2);
    std::memset(xpad, 0, n * 8);
    std::memset(ypad, 0, n * 8);
    std::memset(xpad_f, 0, n * 4);
    std::memset(ypad_f, 0, n * 4);
    return hipSuccess;
}
hipError_t launch_to_f32(const double *in, float *out, size_t n, hipStream_t)
{
    for (size_t k = 0; k < n; ++k) out[k] = (float)in[k];
    return hipSuccess;
}
hipError_t launch_scaled_to_f32(const double *in, double scale, float *out, size_t n, hipStream_t)
{
    for (size_t k = 0; k < n; ++k) out[k] = (float)(scale * in[k]);
    return hipSuccess;
}
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t)
{
    for (size_t k = 0; k < n; ++k) p[k] = v;
    return hipSuccess;
}
// FP32 path launches made so far (any form), read by the harness
std::atomic<int> g_fp32_launches{0};

hipError_t launch_paths_fp32(const InstView *, const WorkRange *, uint32_t, uint32_t, uint32_t *head, uint32_t, int,
                             int, hipStream_t)
{
    *head = 0;
    ++g_fp32_launches;
    return hipSuccess;
}
size_t paths_fp32_lds_bytes(int block, uint32_t cap) { return (size_t)(block / 64) * 6u * cap * sizeof(float); }
size_t paths_fp32_table_lds_bytes(int level, int n_nodes) { return (size_t)n_nodes * level * sizeof(float); }
hipError_t launch_paths_fp32_table(const InstView *, const WorkRange *, uint32_t, uint32_t *head, uint32_t, int, int,
                                   int, int, float *, uint32_t, uint32_t lanes, uint32_t quarters, hipStream_t)
{
    if (lanes < 1 || lanes > 64 || quarters < 1 || quarters > 64) return hipErrorInvalidValue;
    *head = 0;
    ++g_fp32_launches;
    return hipSuccess;
}
int paths_fp32_table_blocks_per_cu(int level, int n_nodes)
{
    return level == 2 && paths_fp32_table_lds_bytes(level, n_nodes) <= 160u * 1024u ? 1 : 0;
}
hipError_t launch_paths_fp32_window(const InstView *, const WorkRange *, const WinJob *, const JobQueues &qs,
                                    uint32_t *head, uint32_t, int periodic, size_t lds, int, float *, uint32_t,
                                    uint32_t lanes, uint32_t quarters, hipStream_t)
{
    for (int q = 0; q < kJobQueues; ++q)
        if (qs.b[q] > qs.b[q + 1]) return hipErrorInvalidValue;
    if (periodic < -1 || periodic > 3 || lds > kWinBytes || lanes < 1 || lanes > 64 || quarters < 1 || quarters > 64)
        return hipErrorInvalidValue;
    for (int q = 0; q < kJobQueues; ++q) head[q] = 0;
    ++g_fp32_launches;
    return hipSuccess;
}
int paths_fp32_window_blocks_per_cu(size_t) { return 1; }
hipError_t launch_paths_fp64(const InstView *, uint32_t, uint32_t, uint32_t, Partial *, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_finalize(const Partial *, const NodeSpan *, const InstView *, uint32_t M, uint64_t, double *mx,
                           double *my, double *sx, double *sy, double *ef, unsigned long long *, hipStream_t)
{
    for (uint32_t k = 0; k < M; ++k) mx[k] = my[k] = sx[k] = sy[k] = ef[k] = 0.0;
    return hipSuccess;
}
hipError_t launch_interpolate(const InterpArgs &, hipStream_t) { return hipSuccess; }
hipError_t launch_debug_paths(const InstView *, int, uint32_t, uint32_t, uint32_t count, double *vx, double *vy,
                              int32_t *ex, int32_t *side, int32_t *steps, double *, hipStream_t)
{
    for (uint32_t k = 0; k < count; ++k) {
        vx[k] = vy[k] = 0.0;
        ex[k] = steps[k] = 0;
        side[k] = -1;
    }
    return hipSuccess;
}
int paths_fp32_blocks_per_cu(int, uint32_t) { return 1; }
int paths_fp32_attributes(int, int *vgprs, int *sgprs, int *lds)
{
    if (vgprs) *vgprs = 128;
    if (sgprs) *sgprs = 0;
    if (lds) *lds = 0;
    return 0;
}

size_t edge_gen_lds_bytes(int n_max) { return (size_t)n_max * 8 * 6; }
hipError_t launch_edge_gen(const double *, const double *, const double *, int, int, int, int, double, double, double,
                           int, int, double *, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_targets(const MeshStepArgs &, double *, double *, hipStream_t) { return hipSuccess; }
size_t subdomain_lds_bytes(int P_xi, int P_eta) { return (size_t)(P_xi + 1) * (P_eta + 1) * 8 * 4; }
bool subdomain_fits_lds(int P_xi, int P_eta) { return subdomain_lds_bytes(P_xi, P_eta) <= kSubLdsMax; }
hipError_t launch_subdomain_lds(const MeshStepArgs &, double *, double *, hipStream_t) { return hipSuccess; }
hipError_t launch_fe_sweep(const MeshStepArgs &, const double *, const double *, double *, double *, double,
                           hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_arclength(const double *, const double *, const double *, int n_xi, int n_eta, int, int, double,
                            double, double, int, double *, unsigned long long *gmax_bits, unsigned int *bad,
                            double *rho, hipStream_t)
{
    for (size_t k = 0; k < (size_t)n_xi * n_eta; ++k) rho[k] = 1.0;
    *gmax_bits = 0;
    *bad = 0;
    return hipSuccess;
}
hipError_t launch_transfer_p1(const TransferArgs &a, hipStream_t)
{
    for (size_t k = 0; k < (size_t)a.n_xi * a.n_eta; ++k) a.f_new[k] = a.f_old[k];
    return hipSuccess;
}
int quality_parts(int, int) { return 1; }
hipError_t launch_quality(const double *, const double *, const double *, const double *, int, int, double *,
                          double *part_max, double *part_sum, double *out2, hipStream_t)
{
    part_max[0] = part_sum[0] = 1.0;
    out2[0] = out2[1] = 1.0;
    return hipSuccess;
}

}  // namespace msdd

namespace msdd_rt {
namespace {
constexpr size_t kHarnessScratch = (size_t)64 << 20;
std::mutex g_mu, g_use;
unsigned char *g_scratch = nullptr;
}  // namespace
size_t scratch_capacity() { return kHarnessScratch; }
hipError_t scratch_resolve(int device)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (device != 0) return hipErrorInvalidDevice;
    if (!g_scratch) g_scratch = static_cast<unsigned char *>(std::calloc(kHarnessScratch, 1));
    return g_scratch ? hipSuccess : hipErrorOutOfMemory;
}
int scratch_region(int device, void **base, std::mutex **use)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (device != 0 || !g_scratch) return fail(MESH_SDD_E_DEVICE, "no scratch on device %d", device);
    *base = g_scratch;
    *use = &g_use;
    return MESH_SDD_OK;
}
}  // namespace msdd_rt
