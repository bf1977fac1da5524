// HIP kernels (gfx950) of the interface-node Monte-Carlo solver for the
// linearised parabolic mesh generator (Bihlo, Haynes & Walsh,
// arXiv:1504.00084, section 3.4):
//
//   Phi^{k+1} = Phi^k + (grad rho / rho)(Phi^k) dt + sqrt(2 dt) N(0, 1)   (EM)
//
// with rho and grad rho bilinearly interpolated from a finite-difference
// table, a Brownian-bridge exit test per substep on Dirichlet sides, wrap
// with winding on periodic axes, bicubic (Keys) evaluation of the mesh at
// t^n for survivors, boundary data (linear in time) for exits, and FP64
// shifted sums per (node, path chunk).
//
// Two path kernels:
//   * paths_fp32: the production kernel.  FP32 path arithmetic with the
//     hardware transcendentals, per-cell records of the bilinear data read
//     through the caches (or, for a launch of one instance, node tables of
//     rho and dt rho_xi staged in LDS), a persistent grid of waves pulling
//     (instance, node, chunk) items from a queue, lanes refilled with the
//     chunk's next path when a path ends, path values evaluated when an
//     item drains, FP64 per-lane sums reduced by wave shuffles.
//   * paths_fp64: the plain baseline.  One thread per path, FP64 throughout
//     (software transcendentals), one launch per instance, block reduction.
//
// The random stream of path p of interface node r: word q is word (q mod 4)
// of Philox4x32-10 (Salmon et al., SC'11) at counter
// (q div 4, p, r, instance << 16 | mesh_step); substep k uses words 3k and
// 3k+1 (Box-Muller) and 3k+2 (bridge uniform).  A lane advances its path
// four substeps at a time, which is exactly three Philox blocks.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "msdd_device.hpp"
#include "msdd_kernels.hpp"

// Multiply-add contraction only inside one expression (a * b + c written
// as such becomes one FMA).  The compiler's default also fuses across
// statements, where the choice depends on the surrounding code: the same
// source line then rounds differently in different kernels (e.g. the cell
// coordinate x * (n - 1) - cell, fused or not depending on whether the
// rounded product is still in a register), and the kernel variants that
// must give identical results would not.
#pragma clang fp contract(on)

namespace msdd {

// Pointers into device global memory: loads through them compile to global
// (not flat) instructions with a scalar base and 32-bit lane offsets.
#define GLOBAL __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ const GLOBAL T *gptr(const T *p) { return (const GLOBAL T *)p; }
template <class T> __device__ __forceinline__ GLOBAL T *gptr_rw(T *p) { return (GLOBAL T *)p; }
typedef float f32x4 __attribute__((ext_vector_type(4)));   // plain 16-byte vector load

// ---------------------------------------------------------------------------
// Philox4x32-10 and uniforms
// ---------------------------------------------------------------------------
struct Words4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, uint32_t k0,
                                                uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        // three-input XOR in one instruction (truth table 0x96)
        const uint32_t y0 = __builtin_amdgcn_bitop3_b32((uint32_t)(m1 >> 32), x1, k0, 0x96);
        const uint32_t y2 = __builtin_amdgcn_bitop3_b32((uint32_t)(m0 >> 32), x3, k1, 0x96);
        x1 = (uint32_t)m1;
        x3 = (uint32_t)m0;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words4{x0, x1, x2, x3};
}

// (2 floor(r / 2^9) + 1) 2^-24, exactly: v_alignbit puts r[31:9] under the
// exponent of 1.0, giving 1 + floor(r / 2^9) 2^-23 in [1, 2), and the
// subtraction of 1 - 2^-24 is exact (the difference needs at most 24
// significant bits).
__device__ __forceinline__ float uniform_f32(uint32_t r)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, r, 9u)) - 0x1.fffffep-1f;
}

__device__ __forceinline__ double uniform_f64(uint32_t r)
{
    return fma((double)(r >> 9), 0x1.0p-23, 0x1.0p-24);
}

// ---------------------------------------------------------------------------
// FP32 path: per-instance constants (wave-uniform)
// ---------------------------------------------------------------------------
struct ConstF {
    int n_xi, n_eta, nx1, ny1;
    int per_xi, per_eta, bridge, K;
    int four;      // 1: the bridge test takes all four sides, 0: the nearer side per Dirichlet axis
    float fnx1, fny1, dt, inv_dt, inv_tau, Lx, Ly;
    float c_rad;   // -4 ln2 dt, so that sqrt(c_rad log2 u) = sqrt(2 dt) sqrt(-2 ln u)
    float sq2dt;   // sqrt(2 dt) (diagnostics only)
    float delta;   // sqrt(18.5 dt): farther from every side, no bridge crossing can matter
    // The instance's cell data, one allocation: first the compact plane of
    // the dt rho_eta corner values (16 B per cell), then from byte `rec0` the
    // 48-B cell records ((rho, dt rho_xi) at corners 00, 10, 01, 11; the dt
    // rho_eta corners again).  Every gather is this scalar base plus a
    // 32-bit lane offset (the two parts together stay below 2^32 bytes).
    const GLOBAL char *cdata;
    uint32_t rec0;
};

// PER >= 0: the instance's path kind (path_kind) as a compile-time constant:
// the periodic flags PER & 1 (xi) and (PER >> 1) & 1 (eta), and PER >> 2 for
// the four-side bridge test -- the launch (or the job) holds instances of
// that kind -- so the tests and selects they guard vanish from the code;
// PER < 0: from I.
template <int PER>
__device__ __forceinline__ ConstF load_const_f(const InstView &I)
{
    ConstF c;
    c.n_xi = I.n_xi;
    c.n_eta = I.n_eta;
    c.nx1 = I.n_xi - 1;
    c.ny1 = I.n_eta - 1;
    c.per_xi = PER < 0 ? I.per_xi : (PER & 1);
    c.per_eta = PER < 0 ? I.per_eta : ((PER >> 1) & 1);
    c.bridge = I.bridge;
    c.four = PER < 0 ? (path_kind(I) >> 2) : (PER >> 2);
    c.K = I.K;
    c.fnx1 = (float)(I.n_xi - 1);
    c.fny1 = (float)(I.n_eta - 1);
    c.dt = I.dt_f;
    c.inv_dt = I.inv_dt_f;
    c.inv_tau = I.inv_tau_f;
    c.Lx = I.Lx_f;
    c.Ly = I.Ly_f;
    c.c_rad = I.c_rad_f;
    c.sq2dt = I.sq2dt_f;
    c.delta = I.delta_f;
    c.cdata = (const GLOBAL char *)I.coef_y;
    c.rec0 = I.rec0;
    return c;
}

struct PathF {
    float x, y;   // position in [0,1]^2 (periodic axes wrapped)
    float m;      // distance of (x, y) to the nearest Dirichlet side (1e30 without one)
    float wx, wy; // winding numbers (whole numbers, exact in FP32 below 2^24)
    int k;        // substeps done
};

// Cell index and local coordinate along one axis with `n1` cells.
__device__ __forceinline__ int cell_of(float s, int n1, float &t)
{
    int c = (int)s;
    c = max(0, min(c, n1 - 1));
    t = s - (float)c;
    return c;
}

// Distance of (x, y) to the nearest Dirichlet side; negative when outside.
__device__ __forceinline__ float side_distance(const ConstF &C, float x, float y)
{
    float m = 1.0e30f;
    if (!C.per_xi) m = fminf(m, fminf(x, 1.0f - x));
    if (!C.per_eta) m = fminf(m, fminf(y, 1.0f - y));
    return m;
}

// Bilinear interpolant from the four corner values of a cell.
__device__ __forceinline__ float bilerp(float tx, float ty, float f00, float f10, float f01, float f11)
{
    const float v0 = fmaf(tx, f10 - f00, f00), v1 = fmaf(tx, f11 - f01, f01);
    return fmaf(ty, v1 - v0, v0);
}

// The same interpolant from the corner values along eta = 0 and eta = 1 and
// their differences along xi (f10 - f00 and f11 - f01, rounded as bilerp
// rounds them): the same result in two instructions fewer.
__device__ __forceinline__ float bilerp_d(float tx, float ty, float f00, float d0, float f01, float d1)
{
    const float v0 = fmaf(tx, d0, f00), v1 = fmaf(tx, d1, f01);
    return fmaf(ty, v1 - v0, v0);
}

// Window of the node tables held in LDS by the windowed kernel: nodes
// [i0, i0 + tw) x [j0, j0 + th), (rho, dt rho_xi) interleaved, row stride tw;
// w1 = tw - 1 and h1 = th - 1 cells.  Three-field windows (TAB 4) also hold
// dt rho_eta of the same nodes, row stride tw, from byte `coff` of the
// window on.
struct Win {
    int i0, j0, tw, w1, h1, coff;
};

// One EM substep of the FP32 path (a3-a6).  Returns the exit side (0: xi=0,
// 1: xi=1, 2: eta=0, 3: eta=1), or -1; an exited path keeps the end of the
// substep as its position (path_value_f32 moves it onto the side).
//
// TAB: where the corner values of rho and dt rho_xi come from.  0: the cell
// record; 2: the LDS node table (rho, dt rho_xi interleaved); 3: the LDS
// window when the cell lies inside it, else the cell record; 4: as 3, with
// dt rho_eta at the corners of the cells inside the window from LDS too; 5:
// as 4, for a square window of kWin3Side nodes.
// The values are the same in every case, so the results are identical.
template <int TAB>
__device__ __forceinline__ int substep_f32(PathF &P, const ConstF &C, uint32_t wa, uint32_t wb, uint32_t wc,
                                           float *trace4, const float *tab, const Win &win)
{
    // a3: Box-Muller on two stream words with the hardware log2 / sqrt /
    // sin / cos (sin and cos take revolutions); sqrt(2 dt) is folded into
    // the radius: rad = sqrt(2 dt) sqrt(-2 ln u0).
    const float u0 = uniform_f32(wa);
    const float u1 = uniform_f32(wb);
    const float rad = __builtin_amdgcn_sqrtf(C.c_rad * __builtin_amdgcn_logf(u0));
    const float cs = __builtin_amdgcn_cosf(u1);
    const float sn = __builtin_amdgcn_sinf(u1);

    // a4: bilinear interpolation of (rho, dt rho_xi, dt rho_eta) on the cell.
    // A coordinate lies in [0, 1) on a periodic axis (after the wrap) and in
    // [0, 1] on a Dirichlet one; below 1 its product with the cell count c
    // stays below c (the largest float below 1 times c rounds down, or is
    // exact for a power of two), so the truncation is the cell and v_fract
    // the local coordinate.  Exactly 1 on a Dirichlet side (a path that ends
    // a substep there survives only if its bridge test, whose crossing
    // probability is then 1, rounds below its uniform, or when the bridge is
    // off) takes the last cell at local coordinate 0.
    const float sx = P.x * C.fnx1, sy = P.y * C.fny1;
    const int cx = C.per_xi ? (int)sx : min((int)sx, C.nx1 - 1);
    const int cy = C.per_eta ? (int)sy : min((int)sy, C.ny1 - 1);
    const float tx = __builtin_amdgcn_fractf(sx), ty = __builtin_amdgcn_fractf(sy);
    // 32-bit indices and byte offsets (a grid has at most 8193^2 nodes, 2^26
    // cells): each gather adds one lane offset to the scalar base of the cell
    // data, and the LDS address is one 24-bit multiply-add.  The record
    // offset (rec0 + 48 B per cell, below 2^32) is a sum of 24-bit products,
    // each exact: the cell index itself can exceed 24 bits.
    const uint32_t ci = __umul24((uint32_t)cy, (uint32_t)C.nx1) + (uint32_t)cx;   // cell
    const uint32_t rec = C.rec0 + __umul24((uint32_t)cy, (uint32_t)C.nx1 * 48u) + __umul24((uint32_t)cx, 48u);
    const GLOBAL f32x4 *cell = (const GLOBAL f32x4 *)(C.cdata + rec);
    const GLOBAL f32x4 *coef = (const GLOBAL f32x4 *)(C.cdata + (ci << 4));
    float r00, r10, r01, r11, g00, g10, g01, g11;
    f32x4 G;   // dt rho_eta at corners 00, 10, 01, 11
    if (TAB == 2) {
        const uint32_t off = __umul24((uint32_t)cy, (uint32_t)C.n_xi << 3) + ((uint32_t)cx << 3);
        const float2 *t2 = (const float2 *)((const char *)tab + off);
        const float2 c00 = t2[0], c10 = t2[1], c01 = t2[C.n_xi], c11 = t2[C.n_xi + 1];
        r00 = c00.x, r10 = c10.x, r01 = c01.x, r11 = c11.x;
        g00 = c00.y, g10 = c10.y, g01 = c01.y, g11 = c11.y;
    } else if (TAB >= 3) {
        // Lanes outside the window read the cell record, which keeps its corner
        // values in the window's order (rho, dt rho_xi per node, row by row):
        // both branches load into the same registers, so neither waits for its
        // loads before the join.  The LDS branch comes first, so a record load
        // waits only for LDS reads before it overwrites their registers, never a
        // gather for an LDS read.  The two-field window's dt rho_eta comes from
        // the plane for every lane, through one gather issued ahead of both.
        // TAB 5: a square three-field window of kWin3Side nodes, whose row
        // stride and dt rho_eta offset are then compile-time constants (the
        // row above becomes an immediate offset of the same LDS address)
        const uint32_t tw = TAB == 5 ? (uint32_t)kWin3Side : (uint32_t)win.tw;
        const uint32_t w1 = TAB == 5 ? (uint32_t)kWin3Side - 1u : (uint32_t)win.w1;
        const uint32_t h1 = TAB == 5 ? (uint32_t)kWin3Side - 1u : (uint32_t)win.h1;
        const int rx = cx - win.i0, ry = cy - win.j0;
        const bool outside = ((uint32_t)rx >= w1) | ((uint32_t)ry >= h1);
        if (TAB == 3) G = *coef;
        if (outside) {
            const f32x4 A = cell[0], B = cell[1];
            r00 = A.x, g00 = A.y, r10 = A.z, g10 = A.w;
            r01 = B.x, g01 = B.y, r11 = B.z, g11 = B.w;
            if (TAB >= 4) G = cell[2];
        } else {
            // window node of corner 00 (row stride tw); the row above is tw on
            // (the multiply takes the job's width, equal to kWin3Side for TAB 5,
            // as a scalar operand of one 24-bit multiply-add)
            const uint32_t node = __umul24((uint32_t)ry, (uint32_t)win.tw) + (uint32_t)rx;
            const float2 *t2 = (const float2 *)tab + node;
            const float2 *u2 = t2 + tw;
            const float2 c00 = t2[0], c10 = t2[1], c01 = u2[0], c11 = u2[1];
            r00 = c00.x, r10 = c10.x, r01 = c01.x, r11 = c11.x;
            g00 = c00.y, g10 = c10.y, g01 = c01.y, g11 = c11.y;
            if (TAB >= 4) {
                // dt rho_eta of window node k sits at byte coff + 4 k
                const uint32_t coff = TAB == 5 ? (uint32_t)(kWin3Side * kWin3Side * 8) : (uint32_t)win.coff;
                const float *e0 = (const float *)((const char *)tab + coff) + node;
                const float *e1 = e0 + tw;
                G.x = e0[0];
                G.y = e0[1];
                G.z = e1[0];
                G.w = e1[1];
            }
        }
    } else {
        const f32x4 A = cell[0], B = cell[1];
        r00 = A.x, g00 = A.y, r10 = A.z, g10 = A.w;
        r01 = B.x, g01 = B.y, r11 = B.z, g11 = B.w;
    }
    // the two-field table kernel reads dt rho_eta from the compact plane (its
    // only gather: better L1 reuse), as the two-field window kernel does; the
    // plane holds it in the difference form of bilerp_d, the record (and the
    // three-field window) as corner values
    if (TAB < 3) G = TAB == 2 ? *coef : cell[2];
    const float rho = bilerp(tx, ty, r00, r10, r01, r11);
    const float gx = bilerp(tx, ty, g00, g10, g01, g11);
    const float gy = TAB == 2 || TAB == 3 ? bilerp_d(tx, ty, G.x, G.y, G.z, G.w) : bilerp(tx, ty, G.x, G.y, G.z, G.w);
    const float inv_rho = __builtin_amdgcn_rcpf(rho);

    // a5: Euler-Maruyama, x + (grad rho / rho) dt + sqrt(2 dt) N.
    float nx = fmaf(rad, cs, fmaf(gx, inv_rho, P.x));
    float ny = fmaf(rad, sn, fmaf(gy, inv_rho, P.y));

    // a6: periodic wrap with winding: x - floor(x) by v_fract, which also
    // keeps the rare tiny negative x (where x + 1 rounds to 1) below 1; the
    // winding is summed as a float (no conversion per substep).
    if (C.per_xi) {
        P.wx += floorf(nx);
        nx = __builtin_amdgcn_fractf(nx);
    }
    if (C.per_eta) {
        P.wy += floorf(ny);
        ny = __builtin_amdgcn_fractf(ny);
    }
    if (trace4) {   // diagnostics: position after the wrap, before any exit projection
        trace4[0] = nx;
        trace4[1] = ny;
        trace4[2] = rad * cs / C.sq2dt;
        trace4[3] = rad * sn / C.sq2dt;
    }

    // a6: one distance serves both tests: negative -> the endpoint left a
    // Dirichlet side; below delta at either end -> a bridge crossing may matter.
    const float m = side_distance(C, nx, ny);
    int side = -1;
    if (m < 0.0f) {
        // endpoint outside; several sides out -> corner, first side crossed.
        // The position stays where it is: the value of an exit reads only the
        // coordinate along its side, clamped onto the side there.
        side = !C.per_xi && nx < 0.0f ? 0 : (!C.per_xi && nx > 1.0f ? 1 : (!C.per_eta && ny < 0.0f ? 2 : 3));
    } else if (C.bridge && min(__float_as_int(P.m), __float_as_int(m)) < __float_as_int(C.delta)) {
        // (the minimum of the two distances below delta; on the signed-integer
        // bit patterns, which order non-NaN floats as their values for a
        // positive delta, -0 included, with no NaN quieting of a float min)
        // Brownian bridge between the two inside points: crossing probability
        // exp(-d0 d1 / dt) per side; d0 d1 / dt > 18.5 gives < 2^-26.6, below
        // the smallest uniform even summed over four sides.
        const float big = 1.0e30f;
        const float L2E = 1.4426950408889634f;
        if (!C.four) {
            // Substeps up to 4e-3: per Dirichlet axis only the side with the
            // smaller d0 d1 / dt is evaluated.  The two values of an axis sum
            // to ((s - 1)^2 + 1 - e^2) / (2 dt), s the sum and e the
            // difference of the two coordinates, so the other's is at least
            // 62.5 (1 - e^2): unless the substep moved more than half the
            // domain, its probability is below 1e-20, and the decision is that
            // of all four sides but when the uniform falls that close to q
            // (bit for bit that of the four-side form, where the probability
            // underflows to 0 in FP32).
            float ax = big, ay = big;
            int sx = 0, sy = 2;
            if (!C.per_xi) {
                const float a0 = P.x * nx * C.inv_dt, a1 = (1.0f - P.x) * (1.0f - nx) * C.inv_dt;
                sx = a1 < a0;
                ax = fminf(a0, a1);
            }
            if (!C.per_eta) {
                const float a2 = P.y * ny * C.inv_dt, a3 = (1.0f - P.y) * (1.0f - ny) * C.inv_dt;
                sy = 2 + (a3 < a2);
                ay = fminf(a2, a3);
            }
            if (fminf(ax, ay) < 18.5f) {
                const float px = __builtin_amdgcn_exp2f(-ax * L2E);
                const float py = __builtin_amdgcn_exp2f(-ay * L2E);
                // q = 1 - (1 - px)(1 - py), without cancellation
                const float q = fmaf(-px, py, px + py);
                // the side with the smaller value, the lower index on ties
                if (uniform_f32(wc) < q) side = ay < ax ? sy : sx;
            }
        } else {
            const float a0 = C.per_xi ? big : P.x * nx * C.inv_dt;
            const float a1 = C.per_xi ? big : (1.0f - P.x) * (1.0f - nx) * C.inv_dt;
            const float a2 = C.per_eta ? big : P.y * ny * C.inv_dt;
            const float a3 = C.per_eta ? big : (1.0f - P.y) * (1.0f - ny) * C.inv_dt;
            if (fminf(fminf(a0, a1), fminf(a2, a3)) < 18.5f) {
                const float p0 = __builtin_amdgcn_exp2f(-a0 * L2E);
                const float p1 = __builtin_amdgcn_exp2f(-a1 * L2E);
                const float p2 = __builtin_amdgcn_exp2f(-a2 * L2E);
                const float p3 = __builtin_amdgcn_exp2f(-a3 * L2E);
                // q = 1 - prod(1 - p_s), accumulated without cancellation
                float q = p0;
                q = fmaf(-q, p1, q + p1);
                q = fmaf(-q, p2, q + p2);
                q = fmaf(-q, p3, q + p3);
                if (uniform_f32(wc) < q) {
                    int s = 0;
                    float am = a0;
                    if (a1 < am) { s = 1; am = a1; }
                    if (a2 < am) { s = 2; am = a2; }
                    if (a3 < am) { s = 3; am = a3; }
                    side = s;
                }
            }
        }
    }
    P.x = nx;
    P.y = ny;
    P.m = m;
    return side;
}

// a7 (exit): boundary value, linear along the side and linear in time.
__device__ __forceinline__ float boundary_f32(const GLOBAL float *b0, const GLOBAL float *b1, int n_xi, int n_eta,
                                              int side, int comp, float tang, float w_tn)
{
    const int len = side < 2 ? n_eta : n_xi;
    const int off = side < 2 ? (side * 2 + comp) * n_eta : 4 * n_eta + ((side - 2) * 2 + comp) * n_xi;
    float fr;
    const int c = cell_of(tang * (float)(len - 1), len - 1, fr);
    const uint32_t o = (uint32_t)(off + c);
    const float v0 = fmaf(fr, b0[o + 1] - b0[o], b0[o]);
    const float v1 = fmaf(fr, b1[o + 1] - b1[o], b1[o]);
    return fmaf(w_tn, v0 - v1, v1);   // w_tn v0 + (1 - w_tn) v1
}

// a7 (survivor): Keys cubic convolution (a = -1/2) on the padded mesh.
__device__ __forceinline__ float keys_f32(const GLOBAL float *pad, int n_xi, int nx1, int ny1, float fnx1, float fny1,
                                          float x, float y)
{
    float tx, ty;
    const int cx = cell_of(x * fnx1, nx1, tx);
    const int cy = cell_of(y * fny1, ny1, ty);
    const float wx[4] = {((-0.5f * tx + 1.0f) * tx - 0.5f) * tx, (1.5f * tx - 2.5f) * tx * tx + 1.0f,
                         ((-1.5f * tx + 2.0f) * tx + 0.5f) * tx, (0.5f * tx - 0.5f) * tx * tx};
    const float wy[4] = {((-0.5f * ty + 1.0f) * ty - 0.5f) * ty, (1.5f * ty - 2.5f) * ty * ty + 1.0f,
                         ((-1.5f * ty + 2.0f) * ty + 0.5f) * ty, (0.5f * ty - 0.5f) * ty * ty};
    const int stride = n_xi + 2;
    const GLOBAL float *row = pad + (uint32_t)(cy * stride + cx);   // padded node (cx-1, cy-1)
    float acc = 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const float r = fmaf(wx[3], row[3], fmaf(wx[2], row[2], fmaf(wx[1], row[1], wx[0] * row[0])));
        acc = fmaf(wy[b], r, acc);
        row += stride;
    }
    return acc;
}

// Value of an ended FP32 path (a7), winding offsets included.
__device__ __forceinline__ void path_value_f32(const InstView &I, const ConstF &C, const PathF &P, int side,
                                               float &vx, float &vy)
{
    if (side >= 0) {
        // the exit point: the end of the substep moved onto the side, i.e. its
        // coordinate along the side, clamped to [0, 1] (a corner exit)
        const float w_tn = (float)P.k * C.dt * C.inv_tau;
        const float tang = __builtin_amdgcn_fmed3f(side < 2 ? P.y : P.x, 0.0f, 1.0f);
        vx = boundary_f32(gptr(I.bnd0_f), gptr(I.bnd1_f), C.n_xi, C.n_eta, side, 0, tang, w_tn);
        vy = boundary_f32(gptr(I.bnd0_f), gptr(I.bnd1_f), C.n_xi, C.n_eta, side, 1, tang, w_tn);
    } else {
        vx = keys_f32(gptr(I.xpad_f), C.n_xi, C.nx1, C.ny1, C.fnx1, C.fny1, P.x, P.y);
        vy = keys_f32(gptr(I.ypad_f), C.n_xi, C.nx1, C.ny1, C.fnx1, C.fny1, P.x, P.y);
    }
    if (C.per_xi) vx = fmaf(P.wx, C.Lx, vx);
    if (C.per_eta) vy = fmaf(P.wy, C.Ly, vy);
}

// When a wave leaves its stepping loop for the refill and item bookkeeping
// (LDS table and window kernels): once fewer than `lanes` of its 64 lanes
// still have a path in flight, or after `quarters` groups of four substeps
// (the launch's tuned values; 56 and 16 by default).
struct Refill {
    uint32_t lanes, quarters;
};

// Advances one path by quarters of four substeps: each quarter draws its
// three Philox blocks at once (words 3s..3s+2 for substep s of the quarter,
// block 3 (k / 4) onwards).  The LDS table and window kernels (TAB 2, 3, 4)
// run up to rf.quarters quarters and leave after a quarter once fewer than
// rf.lanes of the wave's 64 lanes still have a path in flight, so the
// caller's refill and item bookkeeping runs only when lanes are idle.  The
// cell-record kernel (TAB 0) is bound by its gathers, where idle lanes cost
// more than the bookkeeping: it runs one quarter per call, so ended lanes are
// refilled at once.  The substeps and their random words do not depend on
// where the loop is left.  Returns the exit side or -1; `ended` is set when
// the path exited or reached K.
template <bool TRACE, int TAB>
__device__ __forceinline__ int group_f32(PathF &P, const ConstF &C, uint32_t path, uint32_t node, uint32_t ctr3,
                                         uint32_t key0, uint32_t key1, bool &ended, double *trace,
                                         const float *tab, const Win &win, const Refill rf)
{
    int side = -1;
    ended = false;
    const uint32_t quarters = TAB > 0 ? rf.quarters : 1u;
#pragma unroll 1
    for (uint32_t q = 0; q < quarters; ++q) {
        if (q > 0 && (uint32_t)__popcll(__ballot(!ended && P.k < C.K)) < rf.lanes) break;
        const uint32_t blk = 3u * ((uint32_t)P.k >> 2);
        const Words4 A = philox4x32_10(blk, path, node, ctr3, key0, key1);
        const Words4 B = philox4x32_10(blk + 1u, path, node, ctr3, key0, key1);
        const Words4 G = philox4x32_10(blk + 2u, path, node, ctr3, key0, key1);
        const uint32_t w[12] = {A.w0, A.w1, A.w2, A.w3, B.w0, B.w1, B.w2, B.w3, G.w0, G.w1, G.w2, G.w3};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (!ended && P.k < C.K) {
                float t4[4];
                side = substep_f32<TAB>(P, C, w[3 * s], w[3 * s + 1], w[3 * s + 2], TRACE ? t4 : nullptr, tab, win);
                if (TRACE) {
                    double *t = trace + 4 * (size_t)P.k;
                    t[0] = t4[0];
                    t[1] = t4[1];
                    t[2] = t4[2];
                    t[3] = t4[3];
                }
                P.k += 1;
                ended = side >= 0;
            }
        }
    }
    ended = ended || P.k >= C.K;
    return side;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Next item of the queue for the whole wave.  Every lane takes part in the
// atomic (lane 0 adds 1, the others 0), so the pop has no lane-conditional
// branch; lane 0's old value is the wave's item.
__device__ __forceinline__ uint32_t pop_item(uint32_t *head, int lane)
{
    const uint32_t old = atomicAdd(head, lane == 0 ? 1u : 0u);
    return __builtin_amdgcn_readfirstlane(old);
}

// Decoded work item (wave-uniform).
struct ItemF {
    uint32_t inst, node, p_begin, count, partial;
};

__device__ __forceinline__ ItemF decode_item(const GLOBAL WorkRange *rg, uint32_t n_ranges, uint32_t it)
{
    // range holding launch item `it` (ranges are sorted by base, base[0] = 0)
    uint32_t lo = 0, hi = n_ranges;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (rg[mid].base <= it)
            lo = mid;
        else
            hi = mid;
    }
    const GLOBAL WorkRange &R = rg[lo];
    const uint32_t chunks = R.chunks, chunk_paths = R.chunk_paths;
    const uint32_t q = R.first + (it - R.base);   // request-wide item, node-major
    const uint32_t node = q / chunks;
    const uint32_t c = q - node * chunks;
    ItemF f;
    f.inst = R.inst;
    f.node = node;
    f.p_begin = c * chunk_paths;
    f.count = min(chunk_paths, R.N - f.p_begin);
    f.partial = f.node * R.chunks + c;
    return f;
}

// End state of a path, kept in three words of its item's LDS slot until
// the item drains (the value of a path is evaluated then, by all lanes at
// once, instead of by the whole wave whenever one lane's path ends):
//   w2 = wx & 0x3fff | (wy & 0x3fff) << 14 | (side + 1) << 28  (side -1: survived)
//   survived: w0, w1 = x, y;  exited: w0 = k (substeps done), w1 = the
//   coordinate along the side (the other one is fixed by the side).
// A path whose winding does not fit 14 bits stores its values instead:
// w2 = 0x80000000, w0, w1 = vx, vy.
constexpr uint32_t kValueStored = 0x80000000u;

__device__ __forceinline__ void store_end(float *b, uint32_t cap, uint32_t slot, const InstView &I, const ConstF &C,
                                          const PathF &P, int side)
{
    uint32_t w0, w1, w2;
    if (P.wx >= -8192.0f && P.wx < 8192.0f && P.wy >= -8192.0f && P.wy < 8192.0f) {
        w2 = ((uint32_t)(int)P.wx & 0x3FFFu) | (((uint32_t)(int)P.wy & 0x3FFFu) << 14) |
             ((uint32_t)(side + 1) << 28);
        if (side >= 0) {
            w0 = (uint32_t)P.k;
            w1 = __float_as_uint(side < 2 ? P.y : P.x);
        } else {
            w0 = __float_as_uint(P.x);
            w1 = __float_as_uint(P.y);
        }
    } else {
        float vx, vy;
        path_value_f32(I, C, P, side, vx, vy);
        w0 = __float_as_uint(vx);
        w1 = __float_as_uint(vy);
        w2 = kValueStored;
    }
    b[slot] = __uint_as_float(w0);
    b[cap + slot] = __uint_as_float(w1);
    b[2u * cap + slot] = __uint_as_float(w2);
}

__device__ __forceinline__ void stored_value(const float *b, uint32_t cap, uint32_t j, const InstView &I,
                                             const ConstF &C, float &vx, float &vy)
{
    const uint32_t w0 = __float_as_uint(b[j]), w1 = __float_as_uint(b[cap + j]);
    const uint32_t w2 = __float_as_uint(b[2u * cap + j]);
    if (w2 & kValueStored) {
        vx = __uint_as_float(w0);
        vy = __uint_as_float(w1);
        return;
    }
    const int side = (int)(w2 >> 28) - 1;
    PathF P;
    P.wx = (float)((int)(w2 << 18) >> 18);   // sign-extend the 14-bit fields
    P.wy = (float)((int)(w2 << 4) >> 18);
    P.m = 0.0f;
    if (side < 0) {
        P.x = __uint_as_float(w0);
        P.y = __uint_as_float(w1);
        P.k = C.K;
    } else {
        P.k = (int)w0;
        P.x = side < 2 ? 0.0f : __uint_as_float(w1);
        P.y = side < 2 ? __uint_as_float(w1) : 0.0f;
    }
    path_value_f32(I, C, P, side, vx, vy);
}

// Values and fixed-order reduction of one drained item: lane l evaluates
// the paths l, l + 64, ... from their end states, v - v_ref is rounded to
// FP32 and summed in FP64, then the lanes' sums and the exit and step counts
// are combined by butterflies; every lane stores the identical totals.
__device__ __forceinline__ void finish_item(const float *buf, uint32_t cap, uint32_t count, int lane, uint32_t exits,
                                            unsigned long long steps, const InstView &I, const ConstF &C, double rx,
                                            double ry, GLOBAL Partial *out)
{
    double s1x = 0.0, s2x = 0.0, s1y = 0.0, s2y = 0.0;
    for (uint32_t j = (uint32_t)lane; j < count; j += 64u) {
        float vx, vy;
        stored_value(buf, cap, j, I, C, vx, vy);
        const double dx = (double)(float)((double)vx - rx), dy = (double)(float)((double)vy - ry);
        s1x += dx;
        s2x = fma(dx, dx, s2x);
        s1y += dy;
        s2y = fma(dy, dy, s2y);
    }
    s1x = wave_sum(s1x);
    s2x = wave_sum(s2x);
    s1y = wave_sum(s1y);
    s2y = wave_sum(s2y);
    const unsigned long long ex = wave_sum_u64((unsigned long long)exits);
    const unsigned long long st = wave_sum_u64(steps);
    out->s1x = s1x;
    out->s2x = s2x;
    out->s1y = s1y;
    out->s2y = s2y;
    out->exits = ex;
    out->steps = st;
}

// Item sources of the persistent kernels.  QueueSrc: the launch-wide queue,
// one atomic per item, decoded through the launch's range table.
struct QueueSrc {
    uint32_t *head;
    const GLOBAL WorkRange *rg;
    uint32_t n_ranges;
    __device__ __forceinline__ uint32_t pop(int lane) { return pop_item(head, lane); }
    __device__ __forceinline__ ItemF decode(uint32_t it) const { return decode_item(rg, n_ranges, it); }
};

// JobSrc: the items q0 .. q0 + count of one range, handed out by a counter
// in LDS that the workgroup's waves share.  The pop is the queue's: every
// lane takes part in the atomic (lane 0 adds 1), so no lane leaves the wave
// loop on a branch of its own.
struct JobSrc {
    uint32_t *next;   // LDS
    WorkRange R;
    uint32_t q0;
    __device__ __forceinline__ uint32_t pop(int lane) { return pop_item(next, lane); }
    __device__ __forceinline__ ItemF decode(uint32_t it) const
    {
        const uint32_t q = q0 + it;   // request-wide item, node-major
        const uint32_t node = q / R.chunks;
        const uint32_t c = q - node * R.chunks;
        ItemF f;
        f.inst = R.inst;
        f.node = node;
        f.p_begin = c * R.chunk_paths;
        f.count = min(R.chunk_paths, R.N - f.p_begin);
        f.partial = node * R.chunks + c;
        return f;
    }
};

// Wave loop of the persistent kernels.  Each wave keeps up to two work items in
// flight: the one whose paths it is handing out and the one whose last
// paths are finishing, so lanes never wait for an item to drain.  A lane
// whose path ended takes the next path when the wave leaves its stepping
// loop (at a four-substep boundary; see group_f32); its end
// state goes to the item's end-state slot at the path's index, and a drained item
// is evaluated (bicubic or boundary value) and reduced by all lanes in a
// fixed order, so the sums do not depend on which lane ran which path, and
// the wave does not run the value code whenever one lane's path ends.
// Items of another instance start once both slots are drained (the
// per-instance constants are wave-uniform).  The loop ends when the source
// has no item left and both slots have drained.
template <int TAB, int PER, class Src>
__device__ __forceinline__ void item_loop(Src &src, uint32_t n_items, const InstView *__restrict__ insts, float *buf,
                                          uint32_t cap, const float *tab, const Win &win, int lane, const Refill rf)
{
    // wave-uniform state
    uint32_t next = src.pop(lane);
    uint32_t cur_inst = 0xFFFFFFFFu;
    const InstView *Ip = insts;
    ConstF C = load_const_f<PER>(insts[0]);
    uint32_t key0 = 0, key1 = 0, ctr3 = 0;
    uint32_t act0 = 0, act1 = 0, cnt0 = 0, cnt1 = 0, rem0 = 0, rem1 = 0;
    uint32_t node0 = 0, node1 = 0, pb0 = 0, pb1 = 0, part0 = 0, part1 = 0;
    float x00 = 0.f, y00 = 0.f, m00 = 0.f, x01 = 0.f, y01 = 0.f, m01 = 0.f;
    double rx0 = 0.0, ry0 = 0.0, rx1 = 0.0, ry1 = 0.0;
    uint32_t cur = 0, issued = 0;
    bool issuing = false;

    // lane state
    bool has = false;
    uint32_t which = 0, slot = 0, path = 0, node = 0;
    PathF P{0.f, 0.f, 0.f, 0.f, 0.f, 0};
    uint32_t ex0 = 0, ex1 = 0;
    unsigned long long st0 = 0, st1 = 0;

    for (;;) {
        // start the next item in the free slot (another instance only when
        // both slots are drained)
        if (!issuing && next < n_items) {
            const ItemF f = src.decode(next);
            if (f.count == 0u) {   // never produced by the host; skipped so that no slot waits on it
                next = src.pop(lane);
                continue;
            }
            const uint32_t tgt = act0 ? (act1 ? 2u : 1u) : 0u;
            const bool same = f.inst == cur_inst;
            if (tgt < 2u && (same || (act0 == 0u && act1 == 0u))) {
                if (!same) {
                    cur_inst = f.inst;
                    Ip = insts + f.inst;
                    C = load_const_f<PER>(*Ip);
                    key0 = Ip->key0;
                    key1 = Ip->key1;
                    ctr3 = Ip->ctr3;
                }
                const int i0 = gptr(Ip->node_i)[f.node], j0 = gptr(Ip->node_j)[f.node];
                const uint32_t rk = gptr(Ip->node_r)[f.node];   // random-stream identity
                const float x0 = (float)((double)i0 / (double)C.nx1);
                const float y0 = (float)((double)j0 / (double)C.ny1);
                const float m0 = side_distance(C, x0, y0);
                const double rx = gptr(Ip->x64)[(uint32_t)(j0 * C.n_xi + i0)];
                const double ry = gptr(Ip->y64)[(uint32_t)(j0 * C.n_xi + i0)];
                if (tgt == 0u) {
                    act0 = 1u; cnt0 = f.count; rem0 = f.count; node0 = rk; pb0 = f.p_begin;
                    part0 = f.partial; x00 = x0; y00 = y0; m00 = m0; rx0 = rx; ry0 = ry;
                } else {
                    act1 = 1u; cnt1 = f.count; rem1 = f.count; node1 = rk; pb1 = f.p_begin;
                    part1 = f.partial; x01 = x0; y01 = y0; m01 = m0; rx1 = rx; ry1 = ry;
                }
                cur = tgt;
                issued = 0;
                issuing = f.count > 0;
                next = src.pop(lane);
            }
        }
        // refill lanes without a path from the item being handed out, in lane order
        if (issuing) {
            const uint32_t count = cur ? cnt1 : cnt0;
            const uint64_t need = __ballot(!has);
            const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
            if (!has && issued + below < count) {
                has = true;
                which = cur;
                slot = issued + below;
                path = (cur ? pb1 : pb0) + slot;
                node = cur ? node1 : node0;
                P.x = cur ? x01 : x00;
                P.y = cur ? y01 : y00;
                P.m = cur ? m01 : m00;
                P.wx = 0.0f;
                P.wy = 0.0f;
                P.k = 0;
            }
            issued = min(count, issued + (uint32_t)__popcll(need));
            issuing = issued < count;
        }
        if (__ballot(has) == 0) {
            if (issuing) continue;
            if (next >= n_items && act0 == 0u && act1 == 0u) break;
            continue;   // both slots drained: the next item starts at the top
        }
        // advance every path until the wave has lanes to refill
        bool ended = false;
        if (has) {
            const int side = group_f32<false, TAB>(P, C, path, node, ctr3, key0, key1, ended, nullptr, tab, win, rf);
            if (ended) {
                store_end(buf + (size_t)which * 3u * cap, cap, slot, *Ip, C, P, side);
                const uint32_t e = side >= 0 ? 1u : 0u;
                if (which) {
                    ex1 += e;
                    st1 += (unsigned long long)P.k;
                } else {
                    ex0 += e;
                    st0 += (unsigned long long)P.k;
                }
                has = false;
            }
        }
        const uint64_t end_mask = __ballot(ended);
        const uint64_t in1 = __ballot(which != 0u);
        rem0 -= (uint32_t)__popcll(end_mask & ~in1);
        rem1 -= (uint32_t)__popcll(end_mask & in1);
        // reduce and write the items whose paths have all ended
        if (act0 && rem0 == 0u && !(issuing && cur == 0u)) {
            finish_item(buf, cap, cnt0, lane, ex0, st0, *Ip, C, rx0, ry0, gptr_rw(Ip->partials) + part0);
            ex0 = 0;
            st0 = 0;
            act0 = 0u;
        }
        if (act1 && rem1 == 0u && !(issuing && cur == 1u)) {
            finish_item(buf + 3u * cap, cap, cnt1, lane, ex1, st1, *Ip, C, rx1, ry1, gptr_rw(Ip->partials) + part1);
            ex1 = 0;
            st1 = 0;
            act1 = 0u;
        }
    }
}

// The wave loop compiled for the path kind `kind` (path_kind).
template <int TAB, class Src>
__device__ __forceinline__ void item_loop_kind(int kind, Src &src, uint32_t n_items, const InstView *__restrict__ insts,
                                               float *buf, uint32_t cap, const float *tab, const Win &win, int lane,
                                               const Refill rf)
{
    switch (kind) {
    case 0: item_loop<TAB, 0>(src, n_items, insts, buf, cap, tab, win, lane, rf); break;
    case 1: item_loop<TAB, 1>(src, n_items, insts, buf, cap, tab, win, lane, rf); break;
    case 2: item_loop<TAB, 2>(src, n_items, insts, buf, cap, tab, win, lane, rf); break;
    case 4: item_loop<TAB, 4>(src, n_items, insts, buf, cap, tab, win, lane, rf); break;
    case 5: item_loop<TAB, 5>(src, n_items, insts, buf, cap, tab, win, lane, rf); break;
    case 6: item_loop<TAB, 6>(src, n_items, insts, buf, cap, tab, win, lane, rf); break;
    default: item_loop<TAB, 3>(src, n_items, insts, buf, cap, tab, win, lane, rf); break;
    }
}

// Queue-driven persistent kernel (one launch-wide queue of items).
// TAB 2: the launch holds one instance (the host guarantees it), whose FP32
// node tables of rho and dt rho_xi the workgroup copies into LDS,
// interleaved; the bilinear interpolation then reads those corner values
// there instead of from the cell record (the same values, so the results are
// identical), which takes two of the three L1 gathers of a substep off the
// texture path.  The table fills the LDS, so the waves keep the
// end states of their items in `ends` (global memory, 6 * cap words per
// wave, room for `end_waves` waves; read back by the same wave only).
// PER >= 0 (single-instance launches): the instance's path kind as
// compile-time constants (see load_const_f); a mismatching instance ends the
// launch at once, untouched.
template <int BLOCK, int TAB, int PER>
__global__ __launch_bounds__(BLOCK) void paths_fp32(const InstView *__restrict__ insts,
                                                    const WorkRange *__restrict__ ranges, uint32_t n_ranges,
                                                    uint32_t n_items, uint32_t *__restrict__ head, uint32_t cap,
                                                    float *__restrict__ ends, uint32_t end_waves, Refill rf)
{
    extern __shared__ float lds[];
    if (PER >= 0 && path_kind(insts[0]) != PER) return;
    const int lane = threadIdx.x & 63;
    const uint32_t wave = blockIdx.x * (uint32_t)(BLOCK / 64) + (threadIdx.x >> 6);
    if (TAB > 0 && (blockIdx.x + 1u) * (uint32_t)(BLOCK / 64) > end_waves) return;   // whole block: no room
    float *buf = TAB > 0 ? ends + (size_t)wave * 6u * cap
                         : lds + (size_t)(threadIdx.x >> 6) * 6u * cap;   // [slot][w0 | w1 | w2][cap]
    float *tab = nullptr;
    if (TAB > 0) {
        tab = lds;
        const int n = insts[0].n_xi * insts[0].n_eta;
        const GLOBAL float *src = gptr(insts[0].rho_f);
        const GLOBAL float *srx = gptr(insts[0].rhox_f);
        float2 *t2 = (float2 *)tab;
        for (int q = threadIdx.x; q < n; q += BLOCK) t2[q] = make_float2(src[q], srx[q]);
        __syncthreads();
    }

    QueueSrc src{head, gptr(ranges), n_ranges};
    const Win none{0, 0, 0, 0, 0, 0};
    item_loop<TAB, PER>(src, n_items, insts, buf, cap, tab, none, lane, rf);
}

// Windowed kernel for launches whose node tables do not fit the LDS whole:
// several instances, or one large grid.  The host splits the launch into
// jobs: the items of one range whose nodes lie in one block of the grid,
// with a window of the monitor tables around that block (the block plus a
// margin, clamped to the grid), blocks in Z order, cut into per-XCD queues
// (JobQueues).  A workgroup (1024 threads, one per CU) pops a job and copies
// its window into LDS: (rho, dt rho_xi) per node (kind 0), and also dt
// rho_eta per node (kind 1).  Its waves run the job's items
// with the wave loop above; a lane whose path has left the window reads the
// cell record instead (TAB 3 and 4 in substep_f32), so the results are those
// of every other kernel.  The waves
// keep their items' end states in `ends` as the table kernel does.
// PER >= 0: every instance of the launch has that path kind (compiled in);
// a job of another kind is skipped, untouched.
template <int PER>
__global__ __launch_bounds__(kTableBlock) void paths_fp32_win(const InstView *__restrict__ insts,
                                                            const WorkRange *__restrict__ ranges,
                                                            const WinJob *__restrict__ jobs, JobQueues qs,
                                                            uint32_t *__restrict__ head, uint32_t cap,
                                                            float *__restrict__ ends, uint32_t end_waves, Refill rf)
{
    constexpr int BLOCK = kTableBlock;
    // The only LDS of this kernel, a static block (so that its address is a
    // compile-time constant, folded into the LDS instructions' offsets): the
    // job and item counters in its first 16 bytes, then the window: (rho,
    // dt rho_xi) per node, and in three-field windows dt rho_eta per node
    // after them.
    __shared__ float lds[(kWinBytes + 16) / sizeof(float)];
    uint32_t *ctl = (uint32_t *)lds;   // [0]: current job, [1]: next item of the job
    float *wtab = lds + 4;
    const int lane = threadIdx.x & 63;
    const uint32_t wave = blockIdx.x * (uint32_t)(BLOCK / 64) + (threadIdx.x >> 6);
    if ((blockIdx.x + 1u) * (uint32_t)(BLOCK / 64) > end_waves) return;   // whole block: no room
    float *buf = ends + (size_t)wave * 6u * cap;   // [slot][w0 | w1 | w2][cap]
    const uint32_t n_jobs = qs.b[kJobQueues];
    for (;;) {
        if (threadIdx.x == 0) {
            // own queue first, then the others in turn; head[q] counts pops of queue q
            uint32_t j = n_jobs;
            for (int t = 0; t < kJobQueues; ++t) {
                const int q = (int)((blockIdx.x + (uint32_t)t) % (uint32_t)kJobQueues);
                const uint32_t k = qs.b[q] + atomicAdd(head + q, 1u);
                if (k < qs.b[q + 1]) {
                    j = k;
                    break;
                }
            }
            ctl[0] = j;
            ctl[1] = 0u;
        }
        __syncthreads();
        const uint32_t job = ctl[0];
        if (job >= n_jobs) break;   // the same for the whole workgroup
        const WinJob J = jobs[job];
        const WorkRange R = ranges[J.range];
        const InstView &I = insts[R.inst];
        const bool ok = PER < 0 || path_kind(I) == PER;
        const int coff = J.tw * J.th * 8;   // three-field windows: dt rho_eta from here
        {
            const GLOBAL float *src = gptr(I.rho_f);
            const GLOBAL float *srx = gptr(I.rhox_f);
            float2 *t2 = (float2 *)wtab;
            const int n = J.tw * J.th;
            for (int q = threadIdx.x; q < n; q += BLOCK) {
                const int r = q / J.tw, c = q - r * J.tw;
                const uint32_t g = (uint32_t)((J.j0 + r) * I.n_xi + J.i0 + c);
                t2[q] = make_float2(src[g], srx[g]);
            }
            if (J.kind == 1) {
                const GLOBAL float *sry = gptr(I.rhoy_f);
                float *t1 = (float *)((char *)wtab + coff);
                for (int q = threadIdx.x; q < n; q += BLOCK) {
                    const int r = q / J.tw, c = q - r * J.tw;
                    t1[q] = sry[(uint32_t)((J.j0 + r) * I.n_xi + J.i0 + c)];
                }
            }
        }
        __syncthreads();
        JobSrc js{ctl + 1, R, J.q0};
        const Win win{J.i0, J.j0, J.tw, J.tw - 1, J.th - 1, coff};
        const uint32_t count = ok ? J.count : 0u;
        const bool square = J.kind == 1 && J.tw == kWin3Side && J.th == kWin3Side;
        if (PER >= 0) {
            if (square)
                item_loop<5, PER>(js, count, insts, buf, cap, wtab, win, lane, rf);
            else if (J.kind == 1)
                item_loop<4, PER>(js, count, insts, buf, cap, wtab, win, lane, rf);
            else
                item_loop<3, PER>(js, count, insts, buf, cap, wtab, win, lane, rf);
        } else {
            // a launch of mixed kinds: a job holds one instance, so its kind is
            // uniform over the workgroup; each kind runs the wave loop
            // compiled for it
            const int kind = path_kind(I);
            if (square)
                item_loop_kind<5>(kind, js, count, insts, buf, cap, wtab, win, lane, rf);
            else if (J.kind == 1)
                item_loop_kind<4>(kind, js, count, insts, buf, cap, wtab, win, lane, rf);
            else
                item_loop_kind<3>(kind, js, count, insts, buf, cap, wtab, win, lane, rf);
        }
        __syncthreads();   // every wave is done with the window
    }
}

// ---------------------------------------------------------------------------
// FP64 plain path
// ---------------------------------------------------------------------------
struct StreamF64 {
    uint32_t path, node, ctr3, key0, key1;
    uint32_t blk;
    Words4 cur;
    __device__ uint32_t word(uint32_t q)
    {
        const uint32_t b = q >> 2;
        if (b != blk) {
            cur = philox4x32_10(b, path, node, ctr3, key0, key1);
            blk = b;
        }
        const uint32_t r = q & 3u;
        return r == 0 ? cur.w0 : (r == 1 ? cur.w1 : (r == 2 ? cur.w2 : cur.w3));
    }
};

__device__ __forceinline__ int cell_of_d(double s, int n1, double &t)
{
    int c = (int)floor(s);
    c = max(0, min(c, n1 - 1));
    t = s - (double)c;
    return c;
}

__device__ __forceinline__ double bilinear_d(const double *f, int n_xi, int cx, int cy, double tx, double ty)
{
    const double *r0 = f + (size_t)cy * n_xi + cx;
    const double *r1 = r0 + n_xi;
    return (1.0 - tx) * (1.0 - ty) * r0[0] + tx * (1.0 - ty) * r0[1] + (1.0 - tx) * ty * r1[0] + tx * ty * r1[1];
}

__device__ __forceinline__ double boundary_d(const double *b0, const double *b1, int n_xi, int n_eta, int side,
                                             int comp, double tang, double w_tn)
{
    const int len = side < 2 ? n_eta : n_xi;
    const int off = side < 2 ? (side * 2 + comp) * n_eta : 4 * n_eta + ((side - 2) * 2 + comp) * n_xi;
    double fr;
    const int c = cell_of_d(tang * (double)(len - 1), len - 1, fr);
    const double v0 = (1.0 - fr) * b0[off + c] + fr * b0[off + c + 1];
    const double v1 = (1.0 - fr) * b1[off + c] + fr * b1[off + c + 1];
    return w_tn * v0 + (1.0 - w_tn) * v1;
}

__device__ __forceinline__ double keys_d(const double *pad, int n_xi, int n_eta, double x, double y)
{
    double tx, ty;
    const int cx = cell_of_d(x * (double)(n_xi - 1), n_xi - 1, tx);
    const int cy = cell_of_d(y * (double)(n_eta - 1), n_eta - 1, ty);
    const double wx[4] = {((-0.5 * tx + 1.0) * tx - 0.5) * tx, (1.5 * tx - 2.5) * tx * tx + 1.0,
                          ((-1.5 * tx + 2.0) * tx + 0.5) * tx, (0.5 * tx - 0.5) * tx * tx};
    const double wy[4] = {((-0.5 * ty + 1.0) * ty - 0.5) * ty, (1.5 * ty - 2.5) * ty * ty + 1.0,
                          ((-1.5 * ty + 2.0) * ty + 0.5) * ty, (0.5 * ty - 0.5) * ty * ty};
    const int stride = n_xi + 2;
    const double *row = pad + (size_t)cy * stride + cx;
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        acc += wy[b] * (wx[0] * row[0] + wx[1] * row[1] + wx[2] * row[2] + wx[3] * row[3]);
        row += stride;
    }
    return acc;
}

struct PathOutD {
    double vx, vy;
    int side;
    int steps;
};

// One whole path in FP64 (a2-a7).
template <bool TRACE>
__device__ __forceinline__ PathOutD run_path_f64(const InstView &I, uint32_t node, uint32_t path, double *trace)
{
    const int nx1 = I.n_xi - 1, ny1 = I.n_eta - 1;
    const double dt = I.dt, sq = sqrt(2.0 * dt);
    StreamF64 S{path, I.node_r[node], I.ctr3, I.key0, I.key1, 0xFFFFFFFFu, Words4{0, 0, 0, 0}};
    double x = (double)I.node_i[node] / (double)nx1;
    double y = (double)I.node_j[node] / (double)ny1;
    long wx = 0, wy = 0;
    PathOutD out{0.0, 0.0, -1, I.K};
    for (int k = 0; k < I.K; ++k) {
        const uint32_t q = 3u * (uint32_t)k;
        const double u0 = uniform_f64(S.word(q));
        const double u1 = uniform_f64(S.word(q + 1u));
        double sn, cs;
        sincospi(2.0 * u1, &sn, &cs);
        const double rad = sqrt(-2.0 * log(u0));
        const double n1 = rad * cs, n2 = rad * sn;

        double tx, ty;
        const int cx = cell_of_d(x * (double)nx1, nx1, tx);
        const int cy = cell_of_d(y * (double)ny1, ny1, ty);
        const double r = bilinear_d(I.rho, I.n_xi, cx, cy, tx, ty);
        const double rx = bilinear_d(I.rho_xi, I.n_xi, cx, cy, tx, ty);
        const double ry = bilinear_d(I.rho_eta, I.n_xi, cx, cy, tx, ty);
        double nx = x + (rx / r) * dt + sq * n1;
        double ny = y + (ry / r) * dt + sq * n2;
        if (I.per_xi) {
            const double f = floor(nx);
            nx -= f;
            wx += (long)f;
            if (nx >= 1.0) { nx -= 1.0; wx += 1; }
        }
        if (I.per_eta) {
            const double f = floor(ny);
            ny -= f;
            wy += (long)f;
            if (ny >= 1.0) { ny -= 1.0; wy += 1; }
        }
        if (TRACE) {
            trace[4 * k + 0] = nx;
            trace[4 * k + 1] = ny;
            trace[4 * k + 2] = n1;
            trace[4 * k + 3] = n2;
        }
        int side = -1;
        if (!I.per_xi) {
            if (nx < 0.0) { side = 0; nx = 0.0; }
            else if (nx > 1.0) { side = 1; nx = 1.0; }
        }
        if (!I.per_eta) {
            if (ny < 0.0) { side = side < 0 ? 2 : side; ny = 0.0; }
            else if (ny > 1.0) { side = side < 0 ? 3 : side; ny = 1.0; }
        }
        if (side < 0 && I.bridge) {
            double p[4] = {0.0, 0.0, 0.0, 0.0};
            if (!I.per_xi) {
                p[0] = exp(-x * nx / dt);
                p[1] = exp(-(1.0 - x) * (1.0 - nx) / dt);
            }
            if (!I.per_eta) {
                p[2] = exp(-y * ny / dt);
                p[3] = exp(-(1.0 - y) * (1.0 - ny) / dt);
            }
            const double q_exit = 1.0 - (1.0 - p[0]) * (1.0 - p[1]) * (1.0 - p[2]) * (1.0 - p[3]);
            if (uniform_f64(S.word(q + 2u)) < q_exit) {
                int s = 0;
                double pm = p[0];
                if (p[1] > pm) { s = 1; pm = p[1]; }
                if (p[2] > pm) { s = 2; pm = p[2]; }
                if (p[3] > pm) { s = 3; pm = p[3]; }
                side = s;
                if (s == 0) nx = 0.0;
                if (s == 1) nx = 1.0;
                if (s == 2) ny = 0.0;
                if (s == 3) ny = 1.0;
            }
        }
        x = nx;
        y = ny;
        if (side >= 0) {
            const double w_tn = (double)(k + 1) * dt / I.tau;
            const double tang = side < 2 ? y : x;
            out.vx = boundary_d(I.bnd0, I.bnd1, I.n_xi, I.n_eta, side, 0, tang, w_tn);
            out.vy = boundary_d(I.bnd0, I.bnd1, I.n_xi, I.n_eta, side, 1, tang, w_tn);
            out.side = side;
            out.steps = k + 1;
            break;
        }
    }
    if (out.side < 0) {
        out.vx = keys_d(I.xpad, I.n_xi, I.n_eta, x, y);
        out.vy = keys_d(I.ypad, I.n_xi, I.n_eta, x, y);
    }
    if (I.per_xi) out.vx += (double)wx * I.Lx;
    if (I.per_eta) out.vy += (double)wy * I.Ly;
    return out;
}

__global__ __launch_bounds__(kFp64Block) void paths_fp64(const InstView *__restrict__ inst, uint32_t n_paths,
                                                         uint32_t chunks, Partial *__restrict__ partials)
{
    const InstView &I = *inst;
    const uint32_t node = blockIdx.x / chunks;
    const uint32_t chunk = blockIdx.x - node * chunks;
    const uint32_t path = chunk * kFp64Block + threadIdx.x;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (path < n_paths) {
        const PathOutD o = run_path_f64<false>(I, node, path, nullptr);
        const int i0 = I.node_i[node], j0 = I.node_j[node];
        const double dx = o.vx - I.x64[(size_t)j0 * I.n_xi + i0];
        const double dy = o.vy - I.y64[(size_t)j0 * I.n_xi + i0];
        v[0] = dx;
        v[1] = dx * dx;
        v[2] = dy;
        v[3] = dy * dy;
        v[4] = o.side >= 0 ? 1.0 : 0.0;
        v[5] = (double)o.steps;
    }
    // fixed-order tree reduction over the block
    __shared__ double red[6][kFp64Block];
#pragma unroll
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int s = kFp64Block / 2; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Partial &o = partials[blockIdx.x];
        o.s1x = red[0][0];
        o.s2x = red[1][0];
        o.s1y = red[2][0];
        o.s2y = red[3][0];
        o.exits = (unsigned long long)red[4][0];
        o.steps = (unsigned long long)red[5][0];
    }
}

// ---------------------------------------------------------------------------
// Finalize (a9)
// ---------------------------------------------------------------------------
__global__ void finalize_kernel(const Partial *__restrict__ partials, const NodeSpan *__restrict__ spans,
                                const InstView *__restrict__ inst, uint32_t M, uint64_t n_paths,
                                double *mean_x, double *mean_y, double *se_x, double *se_y, double *exit_frac,
                                unsigned long long *steps_total)
{
    const uint32_t node = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long my_steps = 0;
    if (node < M) {
        const InstView &I = *inst;
        const NodeSpan sp = spans[node];
        double s1x = 0.0, s2x = 0.0, s1y = 0.0, s2y = 0.0;
        unsigned long long ex = 0;
        for (uint32_t c = 0; c < sp.count; ++c) {
            const Partial &p = partials[sp.first + c];
            s1x += p.s1x;
            s2x += p.s2x;
            s1y += p.s1y;
            s2y += p.s2y;
            ex += p.exits;
            my_steps += p.steps;
        }
        const int i0 = I.node_i[node], j0 = I.node_j[node];
        const uint32_t r = I.node_r[node];
        const double N = (double)n_paths;
        mean_x[r] = I.x64[(size_t)j0 * I.n_xi + i0] + s1x / N;
        mean_y[r] = I.y64[(size_t)j0 * I.n_xi + i0] + s1y / N;
        if (n_paths > 1) {
            const double vx = (s2x - s1x * s1x / N) / (N - 1.0);
            const double vy = (s2y - s1y * s1y / N) / (N - 1.0);
            se_x[r] = sqrt(fmax(vx, 0.0) / N);
            se_y[r] = sqrt(fmax(vy, 0.0) / N);
        } else {
            se_x[r] = __longlong_as_double(0x7FF8000000000000ll);
            se_y[r] = __longlong_as_double(0x7FF8000000000000ll);
        }
        exit_frac[r] = (double)ex / N;
    }
    // one atomic per wave for the executed-step total
    my_steps = wave_sum_u64(my_steps);
    if ((threadIdx.x & 63) == 0 && my_steps) atomicAdd(steps_total, my_steps);
}

// ---------------------------------------------------------------------------
// Table and mesh preparation (a0, a7 set-up)
// ---------------------------------------------------------------------------
__global__ void prep_gradient_kernel(const double *__restrict__ in, int n_xi, int n_eta, int per_xi, int per_eta,
                                     double *rho, double *rx, double *ry)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_xi * n_eta) return;
    int i = idx % n_xi, j = idx / n_xi;
    // the image node of a periodic axis carries node 0's values
    if (per_xi && i == n_xi - 1) i = 0;
    if (per_eta && j == n_eta - 1) j = 0;
    const double hx = 1.0 / (double)(n_xi - 1), hy = 1.0 / (double)(n_eta - 1);
    auto at = [&](int a, int b) { return in[(size_t)b * n_xi + a]; };
    double gx, gy;
    if (per_xi) {
        const int m = n_xi - 1;
        gx = (at((i + 1) % m, j) - at((i + m - 1) % m, j)) / (2.0 * hx);
    } else if (i == 0) {
        gx = (-3.0 * at(0, j) + 4.0 * at(1, j) - at(2, j)) / (2.0 * hx);
    } else if (i == n_xi - 1) {
        gx = (3.0 * at(i, j) - 4.0 * at(i - 1, j) + at(i - 2, j)) / (2.0 * hx);
    } else {
        gx = (at(i + 1, j) - at(i - 1, j)) / (2.0 * hx);
    }
    if (per_eta) {
        const int m = n_eta - 1;
        gy = (at(i, (j + 1) % m) - at(i, (j + m - 1) % m)) / (2.0 * hy);
    } else if (j == 0) {
        gy = (-3.0 * at(i, 0) + 4.0 * at(i, 1) - at(i, 2)) / (2.0 * hy);
    } else if (j == n_eta - 1) {
        gy = (3.0 * at(i, j) - 4.0 * at(i, j - 1) + at(i, j - 2)) / (2.0 * hy);
    } else {
        gy = (at(i, j + 1) - at(i, j - 1)) / (2.0 * hy);
    }
    rho[idx] = at(i, j);
    rx[idx] = gx;
    ry[idx] = gy;
}

__global__ void prep_cells_kernel(const double *__restrict__ rho, const double *__restrict__ rx,
                                  const double *__restrict__ ry, int n_xi, int n_eta, double grad_scale,
                                  float4 *cells, float4 *coef_y)
{
    const int nx1 = n_xi - 1, ny1 = n_eta - 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nx1 * ny1) return;
    const int cx = idx % nx1, cy = idx / nx1;
    const size_t a = (size_t)cy * n_xi + cx, b = a + n_xi;
    const double *f[3] = {rho, rx, ry};
    // rho and dt rho_xi at the four corners, exactly the FP32 node tables'
    // values, in their order: (rho, dt rho_xi) of nodes 00, 10, then of 01, 11
    cells[3 * (size_t)idx] = make_float4((float)rho[a], (float)(grad_scale * rx[a]), (float)rho[a + 1],
                                         (float)(grad_scale * rx[a + 1]));
    cells[3 * (size_t)idx + 1] = make_float4((float)rho[b], (float)(grad_scale * rx[b]), (float)rho[b + 1],
                                             (float)(grad_scale * rx[b + 1]));
    {   // dt rho_eta at the corners, the FP32 node table's values: in the
        // record as corner values, in the plane with the differences along xi
        // (e00, e10 - e00, e01, e11 - e01), rounded in FP32 as bilerp rounds
        // them, so bilerp_d on the plane gives bilerp's value on the record
        const float e00 = (float)(grad_scale * f[2][a]), e10 = (float)(grad_scale * f[2][a + 1]);
        const float e01 = (float)(grad_scale * f[2][b]), e11 = (float)(grad_scale * f[2][b + 1]);
        cells[3 * (size_t)idx + 2] = make_float4(e00, e10, e01, e11);
        coef_y[idx] = make_float4(e00, e10 - e00, e01, e11 - e01);
    }
}

// Weights and node indices that express padded node `a` (in [-1, n]) as a
// combination of real nodes along one axis; `period` receives the number of
// periods crossed on a periodic axis.
__device__ int pad_stencil(int a, int n, int periodic, int idx[3], double wt[3], int &period)
{
    period = 0;
    if (periodic) {
        const int m = n - 1;
        int q = 0;
        while (a < 0) { a += m; --q; }
        while (a >= m) { a -= m; ++q; }
        period = q;
        idx[0] = a;
        wt[0] = 1.0;
        return 1;
    }
    if (a < 0) {
        idx[0] = 0; idx[1] = 1; idx[2] = 2;
        wt[0] = 3.0; wt[1] = -3.0; wt[2] = 1.0;
        return 3;
    }
    if (a > n - 1) {
        idx[0] = n - 1; idx[1] = n - 2; idx[2] = n - 3;
        wt[0] = 3.0; wt[1] = -3.0; wt[2] = 1.0;
        return 3;
    }
    idx[0] = a;
    wt[0] = 1.0;
    return 1;
}

__global__ void prep_mesh_kernel(const double *__restrict__ x, const double *__restrict__ y, int n_xi, int n_eta,
                                 int per_xi, int per_eta, double Lx, double Ly, double *xpad, double *ypad,
                                 float *xpad_f, float *ypad_f)
{
    const int px = n_xi + 2, py = n_eta + 2;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= px * py) return;
    const int a = idx % px - 1, b = idx / px - 1;
    int ia[3], jb[3], qa, qb;
    double wa[3], wb[3];
    const int na = pad_stencil(a, n_xi, per_xi, ia, wa, qa);
    const int nb = pad_stencil(b, n_eta, per_eta, jb, wb, qb);
    double vx = 0.0, vy = 0.0;
    for (int s = 0; s < nb; ++s)
        for (int r = 0; r < na; ++r) {
            const size_t o = (size_t)jb[s] * n_xi + ia[r];
            vx += wb[s] * wa[r] * x[o];
            vy += wb[s] * wa[r] * y[o];
        }
    vx += (double)qa * Lx;   // x winds along xi (periodic axis only: qa = 0 otherwise)
    vy += (double)qb * Ly;   // y winds along eta
    xpad[idx] = vx;
    ypad[idx] = vy;
    xpad_f[idx] = (float)vx;
    ypad_f[idx] = (float)vy;
}

__global__ void to_f32_kernel(const double *__restrict__ in, float *out, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

__global__ void scaled_to_f32_kernel(const double *__restrict__ in, double scale, float *out, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)(scale * in[i]);
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Interpolation of the interface nodes that ran no paths (a10)
// ---------------------------------------------------------------------------
// Keys' cubic-convolution kernel (a = -1/2) at distance d >= 0.
__device__ __forceinline__ double keys_kernel(double d)
{
    if (d <= 1.0) return (1.5 * d - 2.5) * d * d + 1.0;
    if (d < 2.0) return ((-0.5 * d + 2.5) * d - 4.0) * d + 2.0;
    return 0.0;
}

// One thread per interface rank; nodes that ran paths return at once.  A
// node without paths lies on exactly one interface line (line crossings sit
// on multiples of the stride, which divides the subdomain sizes), at
// position t between the known positions base and base + s.  The stencil
// base - s .. base + 2s holds estimates, boundary values at t^{n+1} (line
// ends on a Dirichlet side), Keys' end rule f(-s) = 3f(0) - 3f(s) + f(2s)
// for a position beyond such an end, and periodic images plus the period
// of the winding coordinate across a seam.  Every position the host allows
// is an interface node or a line end; any other reads as NaN.
__global__ void interpolate_kernel(InterpArgs a)
{
    const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (r >= a.M) return;
    const int i = a.node_i[r], j = a.node_j[r];
    const int s = a.stride;
    const bool on_v = i % a.P_xi == 0, on_h = j % a.P_eta == 0;
    if ((on_v && j % s == 0) || (on_h && i % s == 0)) return;
    const bool vert = on_v;
    const int n = vert ? a.n_eta : a.n_xi;
    const bool per = vert ? a.per_eta != 0 : a.per_xi != 0;
    const int t = vert ? j : i;
    const int base = t - t % s;
    const double u = (double)(t - base) / (double)s;
    const double wk[4] = {keys_kernel(1.0 + u), keys_kernel(u), keys_kernel(1.0 - u), keys_kernel(2.0 - u)};

    // stencil terms (position on the line, weight), at most six
    int tp[6];
    double tw[6];
    int nt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int p = base + (k - 1) * s;
        if (!per && p < 0) {
            tp[nt] = 0, tw[nt++] = 3.0 * wk[k];
            tp[nt] = s, tw[nt++] = -3.0 * wk[k];
            tp[nt] = 2 * s, tw[nt++] = wk[k];
        } else if (!per && p > n - 1) {
            tp[nt] = n - 1, tw[nt++] = 3.0 * wk[k];
            tp[nt] = n - 1 - s, tw[nt++] = -3.0 * wk[k];
            tp[nt] = n - 1 - 2 * s, tw[nt++] = wk[k];
        } else {
            tp[nt] = p, tw[nt++] = wk[k];
        }
    }
    const int ne = a.n_eta, nx = a.n_xi;
    const double qnan = __longlong_as_double(0x7FF8000000000000ll);
    int tq[6];   // interface rank of each term's value, -1 for a boundary value
    double vx = 0.0, vy = 0.0;
    for (int e = 0; e < nt; ++e) {
        int p = tp[e];
        double ox = 0.0, oy = 0.0, fx, fy;
        int q = -1;
        if (per) {
            if (p < 0) {
                p += n - 1;
                (vert ? oy : ox) = -(vert ? a.Ly : a.Lx);
            } else if (p > n - 2) {
                p -= n - 1;
                (vert ? oy : ox) = vert ? a.Ly : a.Lx;
            }
        }
        if (!per && (p == 0 || p == n - 1)) {
            const int side = p == 0 ? 0 : 1;
            const int o = vert ? 4 * ne + side * 2 * nx + i : side * 2 * ne + j;
            const int stride_y = vert ? nx : ne;
            fx = a.bnd1[o];
            fy = a.bnd1[o + stride_y];
        } else if (p >= 0 && p < n) {
            q = vert ? a.rank_of[p * nx + i] : a.rank_of[j * nx + p];
            fx = q >= 0 ? a.mean_x[q] + ox : qnan;
            fy = q >= 0 ? a.mean_y[q] + oy : qnan;
        } else {
            fx = fy = qnan;
        }
        tq[e] = q;
        vx += tw[e] * fx;
        vy += tw[e] * fy;
    }
    // variance of the combination: the weights of repeated estimates merged
    double vsx = 0.0, vsy = 0.0;
    for (int e = 0; e < nt; ++e) {
        const int q = tq[e];
        bool first = q >= 0;
        for (int b = 0; b < e; ++b) first = first && tq[b] != q;
        if (!first) continue;
        double W = 0.0;
        for (int b = e; b < nt; ++b)
            if (tq[b] == q) W += tw[b];
        const double sx = a.se_x[q], sy = a.se_y[q];
        vsx += W * W * (sx * sx);
        vsy += W * W * (sy * sy);
    }
    a.mean_x[r] = vx;
    a.mean_y[r] = vy;
    a.se_x[r] = sqrt(vsx);
    a.se_y[r] = sqrt(vsy);
    a.exit_frac[r] = qnan;
}

// ---------------------------------------------------------------------------
// Diagnostics: one path per thread
// ---------------------------------------------------------------------------
__global__ void debug_paths_kernel(const InstView *__restrict__ inst, int fp64, uint32_t node, uint32_t p_begin,
                                   uint32_t count, double *vx, double *vy, int32_t *exited, int32_t *side_out,
                                   int32_t *steps, double *trace)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const InstView &I = *inst;
    const uint32_t path = p_begin + t;
    double *tr = trace ? trace + (size_t)t * 4 * I.K : nullptr;
    if (fp64) {
        const PathOutD o = tr ? run_path_f64<true>(I, node, path, tr) : run_path_f64<false>(I, node, path, nullptr);
        vx[t] = o.vx;
        vy[t] = o.vy;
        exited[t] = o.side >= 0;
        side_out[t] = o.side;
        steps[t] = o.steps;
        return;
    }
    const ConstF C = load_const_f<-1>(I);
    const int i0 = I.node_i[node], j0 = I.node_j[node];
    PathF P{(float)((double)i0 / (double)C.nx1), (float)((double)j0 / (double)C.ny1), 0.0f, 0.0f, 0.0f, 0};
    P.m = side_distance(C, P.x, P.y);
    int side = -1;
    bool ended = false;
    while (!ended) {
        const Win none{0, 0, 0, 0, 0, 0};
        side = tr ? group_f32<true, 0>(P, C, path, I.node_r[node], I.ctr3, I.key0, I.key1, ended, tr, nullptr, none,
                                       Refill{64u, 1u})
                  : group_f32<false, 0>(P, C, path, I.node_r[node], I.ctr3, I.key0, I.key1, ended, nullptr, nullptr,
                                        none, Refill{64u, 1u});
    }
    float fx, fy;
    path_value_f32(I, C, P, side, fx, fy);
    vx[t] = fx;
    vy[t] = fy;
    exited[t] = side >= 0;
    side_out[t] = side;
    steps[t] = P.k;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_prep_gradient(const double *rho_in, int n_xi, int n_eta, int per_xi, int per_eta, double *rho,
                                double *rho_xi, double *rho_eta, hipStream_t s)
{
    const size_t n = (size_t)n_xi * n_eta;
    hipLaunchKernelGGL(prep_gradient_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, rho_in, n_xi, n_eta, per_xi,
                       per_eta, rho, rho_xi, rho_eta);
    return hipGetLastError();
}

hipError_t launch_prep_cells(const double *rho, const double *rho_xi, const double *rho_eta, int n_xi, int n_eta,
                             double grad_scale, float4 *cells, float4 *coef_y, hipStream_t s)
{
    const size_t n = (size_t)(n_xi - 1) * (n_eta - 1);
    hipLaunchKernelGGL(prep_cells_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, rho, rho_xi, rho_eta, n_xi,
                       n_eta, grad_scale, cells, coef_y);
    return hipGetLastError();
}

hipError_t launch_prep_mesh(const double *x, const double *y, int n_xi, int n_eta, int per_xi, int per_eta, double Lx,
                            double Ly, double *xpad, double *ypad, float *xpad_f, float *ypad_f, hipStream_t s)
{
    const size_t n = (size_t)(n_xi + 2) * (n_eta + 2);
    hipLaunchKernelGGL(prep_mesh_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, y, n_xi, n_eta, per_xi,
                       per_eta, Lx, Ly, xpad, ypad, xpad_f, ypad_f);
    return hipGetLastError();
}

hipError_t launch_to_f32(const double *in, float *out, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(to_f32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_scaled_to_f32(const double *in, double scale, float *out, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(scaled_to_f32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, scale, out, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, value, n);
    return hipGetLastError();
}

hipError_t launch_paths_fp32(const InstView *insts, const WorkRange *ranges, uint32_t n_ranges, uint32_t n_items,
                             uint32_t *head, uint32_t cap, int grid, int block, hipStream_t s)
{
    hipError_t e = launch_fill_u32(head, 0u, 1, s);
    if (e != hipSuccess) return e;
    if (n_items == 0) return hipSuccess;
    const size_t lds = paths_fp32_lds_bytes(block, cap);
    switch (block) {
    case 64:
        hipLaunchKernelGGL((paths_fp32<64, 0, -1>), dim3(grid), dim3(64), lds, s, insts, ranges, n_ranges, n_items, head,
                           cap, nullptr, 0u, Refill{64u, 1u});
        break;
    case 128:
        hipLaunchKernelGGL((paths_fp32<128, 0, -1>), dim3(grid), dim3(128), lds, s, insts, ranges, n_ranges, n_items,
                           head, cap, nullptr, 0u, Refill{64u, 1u});
        break;
    case 256:
        hipLaunchKernelGGL((paths_fp32<256, 0, -1>), dim3(grid), dim3(256), lds, s, insts, ranges, n_ranges, n_items,
                           head, cap, nullptr, 0u, Refill{64u, 1u});
        break;
    case 512:
        hipLaunchKernelGGL((paths_fp32<512, 0, -1>), dim3(grid), dim3(512), lds, s, insts, ranges, n_ranges, n_items,
                           head, cap, nullptr, 0u, Refill{64u, 1u});
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t paths_fp32_table_lds_bytes(int level, int n_nodes) { return (size_t)n_nodes * (size_t)level * sizeof(float); }

template <int TAB, int PER>
static void launch_table(int grid, size_t lds, hipStream_t s, const InstView *insts, const WorkRange *ranges,
                         uint32_t n_items, uint32_t *head, uint32_t cap, float *ends, uint32_t end_waves, Refill rf)
{
    hipLaunchKernelGGL((paths_fp32<kTableBlock, TAB, PER>), dim3(grid), dim3(kTableBlock), lds, s, insts, ranges, 1u,
                       n_items, head, cap, ends, end_waves, rf);
}

hipError_t launch_paths_fp32_table(const InstView *insts, const WorkRange *ranges, uint32_t n_items, uint32_t *head,
                                   uint32_t cap, int level, int kind, int n_nodes, int grid, float *ends,
                                   uint32_t end_waves, uint32_t refill_lanes, uint32_t max_quarters, hipStream_t s)
{
    hipError_t e = launch_fill_u32(head, 0u, 1, s);
    if (e != hipSuccess) return e;
    if (n_items == 0) return hipSuccess;
    if ((size_t)grid * (kTableBlock / 64) > end_waves || level != 2 || kind < 0 || kind > 6 ||
        refill_lanes < 1 || refill_lanes > 64 || max_quarters < 1 || max_quarters > 64)
        return hipErrorInvalidValue;
    const size_t lds = paths_fp32_table_lds_bytes(level, n_nodes);
    const Refill rf{refill_lanes, max_quarters};
    switch (kind) {
    case 0: launch_table<2, 0>(grid, lds, s, insts, ranges, n_items, head, cap, ends, end_waves, rf); break;
    case 1: launch_table<2, 1>(grid, lds, s, insts, ranges, n_items, head, cap, ends, end_waves, rf); break;
    case 2: launch_table<2, 2>(grid, lds, s, insts, ranges, n_items, head, cap, ends, end_waves, rf); break;
    case 4: launch_table<2, 4>(grid, lds, s, insts, ranges, n_items, head, cap, ends, end_waves, rf); break;
    case 5: launch_table<2, 5>(grid, lds, s, insts, ranges, n_items, head, cap, ends, end_waves, rf); break;
    case 6: launch_table<2, 6>(grid, lds, s, insts, ranges, n_items, head, cap, ends, end_waves, rf); break;
    default: launch_table<2, 3>(grid, lds, s, insts, ranges, n_items, head, cap, ends, end_waves, rf); break;
    }
    return hipGetLastError();
}

int paths_fp32_table_blocks_per_cu(int level, int n_nodes)
{
    // every periodicity instance has the same launch bounds and LDS use
    int n = 0;
    const size_t lds = paths_fp32_table_lds_bytes(level, n_nodes);
    if (level != 2) return 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, paths_fp32<kTableBlock, 2, 0>, kTableBlock,
                                                                      lds);
    return e == hipSuccess ? n : 0;
}

template <int PER>
static void launch_win(int grid, size_t lds, hipStream_t s, const InstView *insts, const WorkRange *ranges,
                       const WinJob *jobs, const JobQueues &qs, uint32_t *head, uint32_t cap, float *ends,
                       uint32_t end_waves, Refill rf)
{
    hipLaunchKernelGGL((paths_fp32_win<PER>), dim3(grid), dim3(kTableBlock), lds, s, insts, ranges, jobs, qs, head,
                       cap, ends, end_waves, rf);
}

hipError_t launch_paths_fp32_window(const InstView *insts, const WorkRange *ranges, const WinJob *jobs,
                                    const JobQueues &qs, uint32_t *head, uint32_t cap, int kind, size_t lds,
                                    int grid, float *ends, uint32_t end_waves, uint32_t refill_lanes,
                                    uint32_t max_quarters, hipStream_t s)
{
    hipError_t e = launch_fill_u32(head, 0u, kJobQueues, s);
    if (e != hipSuccess) return e;
    if (qs.b[kJobQueues] == 0) return hipSuccess;
    for (int q = 0; q < kJobQueues; ++q)
        if (qs.b[q] > qs.b[q + 1]) return hipErrorInvalidValue;
    if ((size_t)grid * (kTableBlock / 64) > end_waves || kind < -1 || kind > 6 || lds < 32 ||
        lds > kWinBytes || refill_lanes < 1 || refill_lanes > 64 || max_quarters < 1 || max_quarters > 64)
        return hipErrorInvalidValue;
    lds = 0;   // the kernel's LDS is its static block (counters and the largest window)
    const Refill rf{refill_lanes, max_quarters};
    switch (kind) {
    case 0: launch_win<0>(grid, lds, s, insts, ranges, jobs, qs, head, cap, ends, end_waves, rf); break;
    case 1: launch_win<1>(grid, lds, s, insts, ranges, jobs, qs, head, cap, ends, end_waves, rf); break;
    case 2: launch_win<2>(grid, lds, s, insts, ranges, jobs, qs, head, cap, ends, end_waves, rf); break;
    case 3: launch_win<3>(grid, lds, s, insts, ranges, jobs, qs, head, cap, ends, end_waves, rf); break;
    case 4: launch_win<4>(grid, lds, s, insts, ranges, jobs, qs, head, cap, ends, end_waves, rf); break;
    case 5: launch_win<5>(grid, lds, s, insts, ranges, jobs, qs, head, cap, ends, end_waves, rf); break;
    case 6: launch_win<6>(grid, lds, s, insts, ranges, jobs, qs, head, cap, ends, end_waves, rf); break;
    default: launch_win<-1>(grid, lds, s, insts, ranges, jobs, qs, head, cap, ends, end_waves, rf); break;
    }
    return hipGetLastError();
}

int paths_fp32_window_blocks_per_cu(size_t lds)
{
    int n = 0;
    if (lds > kWinBytes) return 0;   // the static block holds windows up to kWinBytes
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, paths_fp32_win<-1>, kTableBlock, 0);
    return e == hipSuccess ? n : 0;
}

size_t paths_fp32_lds_bytes(int block, uint32_t cap) { return (size_t)(block / 64) * 6u * cap * sizeof(float); }

hipError_t launch_paths_fp64(const InstView *inst, uint32_t M, uint32_t n_paths, uint32_t chunks_per_node,
                             Partial *partials, hipStream_t s)
{
    const size_t blocks = (size_t)M * chunks_per_node;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7FFFFFFFu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(paths_fp64, dim3((unsigned)blocks), dim3(kFp64Block), 0, s, inst, n_paths, chunks_per_node,
                       partials);
    return hipGetLastError();
}

hipError_t launch_finalize(const Partial *partials, const NodeSpan *spans, const InstView *inst, uint32_t M,
                           uint64_t n_paths, double *mean_x, double *mean_y, double *se_x, double *se_y,
                           double *exit_frac, unsigned long long *steps_total, hipStream_t s)
{
    if (M == 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(blocks_for(M, 256)), dim3(256), 0, s, partials, spans, inst, M, n_paths,
                       mean_x, mean_y, se_x, se_y, exit_frac, steps_total);
    return hipGetLastError();
}

hipError_t launch_interpolate(const InterpArgs &a, hipStream_t s)
{
    if (a.M <= 0) return hipSuccess;
    hipLaunchKernelGGL(interpolate_kernel, dim3(blocks_for((size_t)a.M, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_debug_paths(const InstView *inst, int fp64, uint32_t node, uint32_t p_begin, uint32_t count,
                              double *vx, double *vy, int32_t *exited, int32_t *side, int32_t *steps, double *trace,
                              hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(debug_paths_kernel, dim3(blocks_for(count, 64)), dim3(64), 0, s, inst, fp64, node, p_begin,
                       count, vx, vy, exited, side, steps, trace);
    return hipGetLastError();
}

int paths_fp32_blocks_per_cu(int block, uint32_t cap)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    const size_t lds = paths_fp32_lds_bytes(block, cap);
    switch (block) {
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, paths_fp32<64, 0, -1>, 64, lds); break;
    case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, paths_fp32<128, 0, -1>, 128, lds); break;
    case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, paths_fp32<256, 0, -1>, 256, lds); break;
    case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, paths_fp32<512, 0, -1>, 512, lds); break;
    default: break;
    }
    return e == hipSuccess ? n : 0;
}

int paths_fp32_attributes(int block, int *vgprs, int *sgprs, int *lds_bytes)
{
    hipFuncAttributes a;
    hipError_t e = hipErrorInvalidValue;
    switch (block) {
    case 64: e = hipFuncGetAttributes(&a, reinterpret_cast<const void *>(paths_fp32<64, 0, -1>)); break;
    case 128: e = hipFuncGetAttributes(&a, reinterpret_cast<const void *>(paths_fp32<128, 0, -1>)); break;
    case 256: e = hipFuncGetAttributes(&a, reinterpret_cast<const void *>(paths_fp32<256, 0, -1>)); break;
    case 512: e = hipFuncGetAttributes(&a, reinterpret_cast<const void *>(paths_fp32<512, 0, -1>)); break;
    default: break;
    }
    if (e != hipSuccess) return -1;
    if (vgprs) *vgprs = a.numRegs;
    if (sgprs) *sgprs = 0;
    if (lds_bytes) *lds_bytes = (int)a.sharedSizeBytes;
    return 0;
}

}  // namespace msdd
