// Issue-cost probe of the VALU instruction classes used by the path kernel on
// gfx950, for the roofline of the FP32 path.  Each kernel runs eight
// independent dependency chains per lane of one instruction class plus one
// full-rate filler operation (add / xor), over a grid that fills every CU
// with several waves per SIMD; the time per chain step, relative to a plain
// FP32 FMA chain, gives the cost of the class in full-rate issue slots.
// Two more kernels test whether a transcendental overlaps ordinary VALU work:
// eight chains of a bare exp2 (the negation is a source modifier), and the
// same eight chains interleaved with eight independent FMA chains.  If the
// mixed kernel costs the sum of the two, nothing overlaps; if it costs their
// maximum, the transcendental runs beside the FMAs.
// Prints one JSON object on stdout.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                         \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                 \
            std::exit(1);                                                                \
        }                                                                                \
    } while (0)

enum Op { FMA, MAD64, MULHI, XOR, LOG2, SQRT, SIN, EXP2, RCP, PHILOX, EXPN, MIX };

__device__ __forceinline__ float stepf(int op, float x)
{
    switch (op) {
    case FMA: return fmaf(x, 0.999f, 0.001f);
    case LOG2: return __builtin_amdgcn_logf(x) + 3.0f;
    case SQRT: return __builtin_amdgcn_sqrtf(x) + 1.0f;
    case SIN: return __builtin_amdgcn_sinf(x) + 0.5f;
    case EXP2: return __builtin_amdgcn_exp2f(-x) + 0.5f;
    case RCP: return __builtin_amdgcn_rcpf(x) + 1.0f;
    case EXPN: return __builtin_amdgcn_exp2f(-x);
    default: return x;
    }
}

__device__ __forceinline__ uint32_t stepu(int op, uint32_t u)
{
    switch (op) {
    case MAD64: {
        const uint64_t p = (uint64_t)0xD2511F53u * (uint64_t)u;
        return (uint32_t)(p >> 32) ^ (uint32_t)p;
    }
    case MULHI: return __umulhi(u, 0xCD9E8D57u) + 0x9E3779B9u;
    case XOR: return (u ^ 0x9E3779B9u) + 1u;
    default: return u;
    }
}

__device__ __forceinline__ void philox(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3, uint32_t k0,
                                       uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        const uint32_t y0 = (uint32_t)(m1 >> 32) ^ x1 ^ k0;
        const uint32_t y2 = (uint32_t)(m0 >> 32) ^ x3 ^ k1;
        x1 = (uint32_t)m1;
        x3 = (uint32_t)m0;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

template <int OP>
__global__ __launch_bounds__(256) void probe(float *outf, uint32_t *outu, int iters, uint32_t k0, uint32_t k1)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (OP == PHILOX) {   // two independent blocks per iteration
        uint32_t a = t, b = 1, c = 2, d = 3, e = t ^ 0x55555555u, f = 5, g = 6, h = 7, acc = 0;
        for (int i = 0; i < iters; ++i) {
            philox(a, b, c, d, k0, k1);
            philox(e, f, g, h, k0, k1);
            acc ^= a ^ e;
            a += 1u;
            e += 1u;
        }
        outu[t] = acc ^ b ^ c ^ d ^ f ^ g ^ h;
        return;
    }
    if (OP == MAD64 || OP == MULHI || OP == XOR) {
        uint32_t u[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) u[k] = t * 8u + (uint32_t)k + 1u;
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int k = 0; k < 8; ++k) u[k] = stepu(OP, u[k]);
        }
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) s ^= u[k];
        outu[t] = s;
        return;
    }
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = 1.0f + 0.001f * (float)((t + k) & 255);
    if (OP == MIX) {   // eight exp2 chains beside eight FMA chains
        float y[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) y[k] = 0.5f + 0.001f * (float)((t + 3 * k) & 255);
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                x[k] = stepf(EXPN, x[k]);
                y[k] = stepf(FMA, y[k]);
            }
        }
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < 8; ++k) s += x[k] + y[k];
        outf[t] = s;
        return;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = stepf(OP, x[k]);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k];
    outf[t] = s;
}

template <int OP>
double time_op(int grid, int iters, float *df, uint32_t *du)
{
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    hipLaunchKernelGGL(probe<OP>, dim3(grid), dim3(256), 0, 0, df, du, iters / 8, 1u, 2u);   // warm-up
    CHECK(hipEventRecord(a, 0));
    hipLaunchKernelGGL(probe<OP>, dim3(grid), dim3(256), 0, 0, df, du, iters, 1u, 2u);
    CHECK(hipEventRecord(b, 0));
    CHECK(hipEventSynchronize(b));
    float ms = 0.0f;
    CHECK(hipEventElapsedTime(&ms, a, b));
    CHECK(hipEventDestroy(a));
    CHECK(hipEventDestroy(b));
    return ms;
}

int main()
{
    hipDeviceProp_t p;
    CHECK(hipGetDeviceProperties(&p, 0));
    const int cus = p.multiProcessorCount;
    const int grid = cus * 16;   // 16 blocks of 4 waves per CU: 16 waves per SIMD requested
    const size_t n = (size_t)grid * 256;
    float *df;
    uint32_t *du;
    CHECK(hipMalloc(&df, n * sizeof(float)));
    CHECK(hipMalloc(&du, n * sizeof(uint32_t)));
    const int iters = 4096;
    const double chains = (double)n * iters * 8.0;
    const double t_fma = time_op<FMA>(grid, iters, df, du);
    const double lane_slots_per_s = chains / (t_fma * 1e-3);   // FMA chain: 1 slot per step
    struct R { const char *name; double ms; double per; };
    R r[] = {
        {"fma_f32", t_fma, 1.0},
        {"mad_u64_u32+xor", time_op<MAD64>(grid, iters, df, du), 1.0},
        {"mul_hi_u32+add", time_op<MULHI>(grid, iters, df, du), 1.0},
        {"xor+add", time_op<XOR>(grid, iters, df, du), 1.0},
        {"log_f32+add", time_op<LOG2>(grid, iters, df, du), 1.0},
        {"sqrt_f32+add", time_op<SQRT>(grid, iters, df, du), 1.0},
        {"sin_f32+add", time_op<SIN>(grid, iters, df, du), 1.0},
        {"exp_f32+add", time_op<EXP2>(grid, iters, df, du), 1.0},
        {"rcp_f32+add", time_op<RCP>(grid, iters, df, du), 1.0},
        {"philox4x32_10_block", time_op<PHILOX>(grid, iters, df, du), 2.0 / 8.0},
        {"exp_f32_bare", time_op<EXPN>(grid, iters, df, du), 1.0},
        {"exp_f32_bare+independent_fma", time_op<MIX>(grid, iters, df, du), 1.0},
    };
    std::printf("{\"device\": \"%s\", \"cus\": %d, \"clock_mhz\": %d, \"fma_lane_slots_per_s\": %.6e, "
                "\"effective_clock_ghz\": %.4f, \"slots\": {",
                p.gcnArchName, cus, p.clockRate / 1000, lane_slots_per_s, lane_slots_per_s / (cus * 64.0) / 1e9);
    for (size_t k = 0; k < sizeof r / sizeof r[0]; ++k) {
        // slots per chain step (the Philox kernel runs one chain per lane)
        const double steps = chains * r[k].per;
        const double slots = r[k].ms * 1e-3 * lane_slots_per_s / steps;
        std::printf("%s\"%s\": %.3f", k ? ", " : "", r[k].name, slots);
    }
    std::printf("}}\n");
    CHECK(hipFree(df));
    CHECK(hipFree(du));
    return 0;
}
