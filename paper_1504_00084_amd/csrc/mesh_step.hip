// Kernels of the mesh step around the interface estimate (FP64):
//   * edge_gen_kernel: the one-dimensional form of the generator (eq. Gen,
//     section 2) along each physical side, which gives the tangential
//     boundary values at t^{n+1};
//   * targets_kernel: Dirichlet data of the decomposed problem at t^{n+1}
//     (physical boundary, interface estimate, images of the seam);
//   * subdomain_lds_kernel: the subdomain solves of section 3.5 (centred
//     differences, forward Euler), one workgroup per subdomain with the
//     subdomain's mesh resident in LDS for all substeps;
//   * fe_sweep_kernel: one forward-Euler substep over the whole grid in
//     global memory; used when a subdomain does not fit in LDS and for the
//     single-domain reference (periodic axes wrap there);
//   * arclength kernels: the monitor rho = sqrt(1 + a |grad u|^2) from nodal u
//     on the new mesh (section 3.6), the physical gradient through the
//     inverse mesh Jacobian;
//   * quality kernels: Q(K) per cell (eq. Q, section 3.7) of two meshes, the
//     ratio R = Q_SD / Q_SDD, its maximum and its mean (fixed-order sums).
//
// Floating-point contraction is off in this file: every update is the plain
// sequence of IEEE operations written below, in that order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msdd_mesh_step.hpp"

#pragma clang fp contract(off)

namespace msdd {

namespace {

__device__ __forceinline__ int side_offset(int side, int comp, int n_xi, int n_eta)
{
    return side < 2 ? (side * 2 + comp) * n_eta : 4 * n_eta + ((side - 2) * 2 + comp) * n_xi;
}

// ---------------------------------------------------------------------------
// 1-D generator along the physical sides
// ---------------------------------------------------------------------------
// Workgroup k advances one side: sides 0, 1 (xi = 0, 1; y runs along eta)
// when xi is a Dirichlet axis, sides 2, 3 (eta = 0, 1; x runs along xi)
// when eta is.  LDS holds the two time levels and the drift coefficients.
__global__ __launch_bounds__(kEdgeBlock) void edge_gen_kernel(const double *__restrict__ rho,
                                                             const double *__restrict__ rho_xi,
                                                             const double *__restrict__ rho_eta, int n_xi,
                                                             int n_eta, int per_xi, int per_eta, double Lx,
                                                             double Ly, double tau, int L_eta, int L_xi,
                                                             double *__restrict__ bnd)
{
    extern __shared__ double sm[];
    const int side = per_xi ? (int)blockIdx.x + 2 : (int)blockIdx.x;
    const bool along_eta = side < 2;
    const int n = along_eta ? n_eta : n_xi;
    const int L = along_eta ? L_eta : L_xi;
    const int periodic = along_eta ? per_eta : per_xi;
    const double period = along_eta ? Ly : Lx;
    const int off = side_offset(side, along_eta ? 1 : 0, n_xi, n_eta);
    double *cur = sm, *nxt = sm + n, *bb = sm + 2 * n;
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        const int g = along_eta ? s * n_xi + (side == 0 ? 0 : n_xi - 1) : (side == 2 ? 0 : n_eta - 1) * n_xi + s;
        cur[s] = bnd[off + s];
        bb[s] = (along_eta ? rho_eta[g] : rho_xi[g]) / rho[g];
    }
    __syncthreads();
    const double h = 1.0 / (double)(n - 1);
    const double two_h = 2.0 * h, hh = h * h;
    const double dt = tau / (double)L;
    for (int l = 0; l < L; ++l) {
        for (int s = threadIdx.x; s < n; s += blockDim.x) {
            double v;
            if (periodic) {
                // node n-1 is the image of node 0: its update is node 0's plus the period
                const int q = s == n - 1 ? 0 : s;
                const double left = q > 0 ? cur[q - 1] : cur[n - 2] - period;
                const double right = cur[q + 1];
                v = cur[q] + dt * (bb[q] * (right - left) / two_h + (right - 2.0 * cur[q] + left) / hh);
                if (s == n - 1) v = v + period;
            } else if (s == 0 || s == n - 1) {
                v = cur[s];
            } else {
                v = cur[s] + dt * (bb[s] * (cur[s + 1] - cur[s - 1]) / two_h +
                                   (cur[s + 1] - 2.0 * cur[s] + cur[s - 1]) / hh);
            }
            nxt[s] = v;
        }
        __syncthreads();
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    for (int s = threadIdx.x; s < n; s += blockDim.x) bnd[off + s] = cur[s];
}

// ---------------------------------------------------------------------------
// Dirichlet data at t^{n+1}
// ---------------------------------------------------------------------------
struct Target {
    double x, y;
    bool dirichlet;
};

__device__ Target target_of(int i, int j, const MeshStepArgs &a)
{
    // with interfaces, an image node on a periodic axis follows its original
    double ox = 0.0, oy = 0.0;
    if (a.with_interfaces) {
        if (a.per_xi && i == a.n_xi - 1) {
            i = 0;
            ox = a.Lx;
        }
        if (a.per_eta && j == a.n_eta - 1) {
            j = 0;
            oy = a.Ly;
        }
    }
    Target t{0.0, 0.0, false};
    if (a.with_interfaces) {
        const int r = a.node_rank[j * a.n_xi + i];
        if (r >= 0) t = Target{a.iface_x[r], a.iface_y[r], true};
    }
    if (!a.per_xi && (i == 0 || i == a.n_xi - 1)) {
        const int side = i == 0 ? 0 : 1;
        t = Target{a.bnd1[side_offset(side, 0, a.n_xi, a.n_eta) + j], a.bnd1[side_offset(side, 1, a.n_xi, a.n_eta) + j],
                   true};
    }
    if (!a.per_eta && (j == 0 || j == a.n_eta - 1)) {   // rows win at corners
        const int side = j == 0 ? 2 : 3;
        t = Target{a.bnd1[side_offset(side, 0, a.n_xi, a.n_eta) + i], a.bnd1[side_offset(side, 1, a.n_xi, a.n_eta) + i],
                   true};
    }
    t.x = t.x + ox;
    t.y = t.y + oy;
    return t;
}

__global__ void targets_kernel(MeshStepArgs a, double *__restrict__ x_new, double *__restrict__ y_new)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n_xi * a.n_eta) return;
    const int i = g % a.n_xi, j = g / a.n_xi;
    const Target t = target_of(i, j, a);
    a.mask[g] = t.dirichlet ? 1 : 0;
    a.tx1[g] = t.x;
    a.ty1[g] = t.y;
    if (t.dirichlet) {
        x_new[g] = t.x;
        y_new[g] = t.y;
    }
}

// ---------------------------------------------------------------------------
// Subdomain solves with the subdomain resident in LDS
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSubBlock) void subdomain_lds_kernel(MeshStepArgs a, double *__restrict__ x_new,
                                                                  double *__restrict__ y_new)
{
    extern __shared__ double sm[];
    const int bi = (int)blockIdx.x % a.sub_xi, bj = (int)blockIdx.x / a.sub_xi;
    const int Px = a.P_xi, Py = a.P_eta;
    const int Bx = Px + 1, By = Py + 1;
    const int i0 = bi * Px, j0 = bj * Py;
    double *sx = sm, *sy = sm + Bx * By;
    const int tid = threadIdx.x;
    for (int q = tid; q < Bx * By; q += kSubBlock) {
        const int g = (j0 + q / Bx) * a.n_xi + i0 + q % Bx;
        sx[q] = a.x0[g];
        sy[q] = a.y0[g];
    }
    // interior nodes owned by this thread: q = tid + r * kSubBlock
    const int nin = (Px - 1) * (Py - 1);
    double bxr[kSubPerThread], byr[kSubPerThread];
    int lq[kSubPerThread];
#pragma unroll
    for (int r = 0; r < kSubPerThread; ++r) {
        const int q = tid + r * kSubBlock;
        lq[r] = -1;
        bxr[r] = 0.0;
        byr[r] = 0.0;
        if (q < nin) {
            const int ca = 1 + q % (Px - 1), cc = 1 + q / (Px - 1);
            const int g = (j0 + cc) * a.n_xi + i0 + ca;
            lq[r] = cc * Bx + ca;
            bxr[r] = a.rho_xi[g] / a.rho[g];
            byr[r] = a.rho_eta[g] / a.rho[g];
        }
    }
    // boundary node of the box owned by this thread (at most one)
    const int nb = 2 * Bx + 2 * (By - 2);
    int bq = -1;
    double bx0 = 0.0, by0 = 0.0, bx1 = 0.0, by1 = 0.0;
    if (tid < nb) {
        int ca, cc;
        if (tid < Bx) {
            ca = tid;
            cc = 0;
        } else if (tid < 2 * Bx) {
            ca = tid - Bx;
            cc = By - 1;
        } else if (tid < 2 * Bx + By - 2) {
            ca = 0;
            cc = 1 + tid - 2 * Bx;
        } else {
            ca = Bx - 1;
            cc = 1 + tid - 2 * Bx - (By - 2);
        }
        const int g = (j0 + cc) * a.n_xi + i0 + ca;
        bq = cc * Bx + ca;
        bx0 = a.x0[g];
        by0 = a.y0[g];
        bx1 = a.tx1[g];
        by1 = a.ty1[g];
    }
    const double hx = 1.0 / (double)(a.n_xi - 1), hy = 1.0 / (double)(a.n_eta - 1);
    const double two_hx = 2.0 * hx, two_hy = 2.0 * hy, hxx = hx * hx, hyy = hy * hy;
    const double dt = a.tau / (double)a.L;
    __syncthreads();
    double nxr[kSubPerThread], nyr[kSubPerThread];
    for (int l = 0; l < a.L; ++l) {
        const double th1 = (double)(l + 1) / (double)a.L;
#pragma unroll
        for (int r = 0; r < kSubPerThread; ++r) {
            nxr[r] = 0.0;
            nyr[r] = 0.0;
            if (lq[r] >= 0) {
                const int q = lq[r];
                {
                    const double c = sx[q], e = sx[q + 1], w = sx[q - 1], n = sx[q + Bx], s = sx[q - Bx];
                    nxr[r] = c + dt * (bxr[r] * (e - w) / two_hx + byr[r] * (n - s) / two_hy +
                                       (e - 2.0 * c + w) / hxx + (n - 2.0 * c + s) / hyy);
                }
                {
                    const double c = sy[q], e = sy[q + 1], w = sy[q - 1], n = sy[q + Bx], s = sy[q - Bx];
                    nyr[r] = c + dt * (bxr[r] * (e - w) / two_hx + byr[r] * (n - s) / two_hy +
                                       (e - 2.0 * c + w) / hxx + (n - 2.0 * c + s) / hyy);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSubPerThread; ++r) {
            if (lq[r] >= 0) {
                sx[lq[r]] = nxr[r];
                sy[lq[r]] = nyr[r];
            }
        }
        if (bq >= 0) {
            sx[bq] = (1.0 - th1) * bx0 + th1 * bx1;
            sy[bq] = (1.0 - th1) * by0 + th1 * by1;
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < kSubPerThread; ++r) {
        if (lq[r] >= 0) {
            const int q = lq[r];
            const int g = (j0 + q / Bx) * a.n_xi + i0 + q % Bx;
            x_new[g] = sx[q];
            y_new[g] = sy[q];
        }
    }
}

// ---------------------------------------------------------------------------
// One forward-Euler substep over the whole grid in global memory
// ---------------------------------------------------------------------------
__device__ __forceinline__ double nb_value(const double *f, int i, int j, const MeshStepArgs &a, double L_xi,
                                           double L_eta)
{
    double off = 0.0;
    if (a.per_xi) {
        if (i < 0) {
            i += a.n_xi - 1;
            off -= L_xi;
        } else if (i > a.n_xi - 1) {
            i -= a.n_xi - 1;
            off += L_xi;
        }
    }
    if (a.per_eta) {
        if (j < 0) {
            j += a.n_eta - 1;
            off -= L_eta;
        } else if (j > a.n_eta - 1) {
            j -= a.n_eta - 1;
            off += L_eta;
        }
    }
    return f[j * a.n_xi + i] + off;
}

__device__ __forceinline__ double stencil(const double *f, int i, int j, const MeshStepArgs &a, double L_xi,
                                          double L_eta, double bx, double by, double dt, double two_hx,
                                          double two_hy, double hxx, double hyy)
{
    const double c = f[j * a.n_xi + i];
    const double e = nb_value(f, i + 1, j, a, L_xi, L_eta), w = nb_value(f, i - 1, j, a, L_xi, L_eta);
    const double n = nb_value(f, i, j + 1, a, L_xi, L_eta), s = nb_value(f, i, j - 1, a, L_xi, L_eta);
    return c + dt * (bx * (e - w) / two_hx + by * (n - s) / two_hy + (e - 2.0 * c + w) / hxx + (n - 2.0 * c + s) / hyy);
}

__global__ void fe_sweep_kernel(MeshStepArgs a, const double *__restrict__ cx, const double *__restrict__ cy,
                                double *__restrict__ nx, double *__restrict__ ny, double th1)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n_xi * a.n_eta) return;
    if (a.mask[g]) {
        nx[g] = (1.0 - th1) * a.x0[g] + th1 * a.tx1[g];
        ny[g] = (1.0 - th1) * a.y0[g] + th1 * a.ty1[g];
        return;
    }
    int i = g % a.n_xi, j = g / a.n_xi;
    // an image node (periodic axis, not Dirichlet) repeats its original's update plus the period
    double ox = 0.0, oy = 0.0;
    if (a.per_xi && i == a.n_xi - 1) {
        i = 0;
        ox = a.Lx;
    }
    if (a.per_eta && j == a.n_eta - 1) {
        j = 0;
        oy = a.Ly;
    }
    const int s = j * a.n_xi + i;
    const double hx = 1.0 / (double)(a.n_xi - 1), hy = 1.0 / (double)(a.n_eta - 1);
    const double bx = a.rho_xi[s] / a.rho[s], by = a.rho_eta[s] / a.rho[s];
    const double dt = a.tau / (double)a.L;
    const double vx = stencil(cx, i, j, a, a.Lx, 0.0, bx, by, dt, 2.0 * hx, 2.0 * hy, hx * hx, hy * hy);
    const double vy = stencil(cy, i, j, a, 0.0, a.Ly, bx, by, dt, 2.0 * hx, 2.0 * hy, hx * hx, hy * hy);
    nx[g] = ox != 0.0 ? vx + ox : vx;
    ny[g] = oy != 0.0 ? vy + oy : vy;
}

// ---------------------------------------------------------------------------
// Arc-length monitor from nodal u
// ---------------------------------------------------------------------------
// Difference along one axis in units of the node index: centred inside,
// one-sided second order at Dirichlet ends, wrapped (plus `period` for the
// winding coordinate) on a periodic axis.  `stride` steps along the axis.
__device__ __forceinline__ double axis_diff(const double *f, int base, int k, int n, int stride, int periodic,
                                            double period)
{
    if (periodic) {
        double left, right;
        if (k == 0 || k == n - 1) {
            left = f[base + (n - 2) * stride] - period;
            right = f[base + stride];
        } else {
            left = f[base + (k - 1) * stride];
            right = f[base + (k + 1) * stride];
        }
        return 0.5 * (right - left);
    }
    if (k == 0) return 0.5 * (-3.0 * f[base] + 4.0 * f[base + stride] - f[base + 2 * stride]);
    if (k == n - 1)
        return 0.5 * (3.0 * f[base + (n - 1) * stride] - 4.0 * f[base + (n - 2) * stride] + f[base + (n - 3) * stride]);
    return 0.5 * (f[base + (k + 1) * stride] - f[base + (k - 1) * stride]);
}

__global__ void arclength_grad_kernel(const double *__restrict__ u, const double *__restrict__ x,
                                      const double *__restrict__ y, int n_xi, int n_eta, int per_xi, int per_eta,
                                      double Lx, double Ly, double *__restrict__ g_out,
                                      unsigned long long *__restrict__ gmax_bits, unsigned int *__restrict__ bad)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_xi * n_eta) return;
    const int i = g % n_xi, j = g / n_xi;
    const double hx = 1.0 / (double)(n_xi - 1), hy = 1.0 / (double)(n_eta - 1);
    const int row = j * n_xi, col = i;
    const double u_xi = axis_diff(u, row, i, n_xi, 1, per_xi, 0.0) / hx;
    const double x_xi = axis_diff(x, row, i, n_xi, 1, per_xi, Lx) / hx;
    const double y_xi = axis_diff(y, row, i, n_xi, 1, per_xi, 0.0) / hx;
    const double u_eta = axis_diff(u, col, j, n_eta, n_xi, per_eta, 0.0) / hy;
    const double x_eta = axis_diff(x, col, j, n_eta, n_xi, per_eta, 0.0) / hy;
    const double y_eta = axis_diff(y, col, j, n_eta, n_xi, per_eta, Ly) / hy;
    const double jac = x_xi * y_eta - x_eta * y_xi;
    const double ux = (u_xi * y_eta - u_eta * y_xi) / jac;
    const double uy = (u_eta * x_xi - u_xi * x_eta) / jac;
    const double gg = ux * ux + uy * uy;
    g_out[g] = gg;
    if (!(gg >= 0.0) || gg > 1.0e300) {   // NaN / infinite: vanishing Jacobian or bad input
        atomicOr(bad, 1u);
        return;
    }
    // non-negative doubles order like their bit patterns
    atomicMax(gmax_bits, (unsigned long long)__double_as_longlong(gg));
}

__global__ void arclength_rho_kernel(const double *__restrict__ g_in, int n, double alpha, int normalize,
                                     const unsigned long long *__restrict__ gmax_bits, double *__restrict__ rho)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double a = alpha;
    if (normalize) {
        const double gmax = __longlong_as_double((long long)*gmax_bits);
        a = gmax > 0.0 ? alpha / gmax : 0.0;
    }
    rho[k] = sqrt(1.0 + a * g_in[k]);
}

// ---------------------------------------------------------------------------
// Mesh quality
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cell_q(const double *x, const double *y, int i, int j, int n_xi, double hx, double hy)
{
    const int g00 = j * n_xi + i, g10 = g00 + 1, g01 = g00 + n_xi, g11 = g01 + 1;
    const double x_xi = 0.5 * ((x[g10] - x[g00]) + (x[g11] - x[g01])) / hx;
    const double y_xi = 0.5 * ((y[g10] - y[g00]) + (y[g11] - y[g01])) / hx;
    const double x_eta = 0.5 * ((x[g01] - x[g00]) + (x[g11] - x[g10])) / hy;
    const double y_eta = 0.5 * ((y[g01] - y[g00]) + (y[g11] - y[g10])) / hy;
    const double tr = x_xi * x_xi + y_xi * y_xi + x_eta * x_eta + y_eta * y_eta;
    const double det = fabs(x_xi * y_eta - x_eta * y_xi);
    return 0.5 * tr / det;
}

// R per cell; per-block maximum and sum (fixed tree order) into partials.
__global__ __launch_bounds__(kQualityBlock) void quality_kernel(const double *__restrict__ xs,
                                                               const double *__restrict__ ys,
                                                               const double *__restrict__ xd,
                                                               const double *__restrict__ yd, int n_xi, int n_eta,
                                                               double *__restrict__ r_cells,
                                                               double *__restrict__ part_max,
                                                               double *__restrict__ part_sum)
{
    __shared__ double smax[kQualityBlock], ssum[kQualityBlock];
    const int nc = (n_xi - 1) * (n_eta - 1);
    const int c = blockIdx.x * kQualityBlock + threadIdx.x;
    double r = 0.0, mx = 0.0;
    if (c < nc) {
        const int i = c % (n_xi - 1), j = c / (n_xi - 1);
        const double hx = 1.0 / (double)(n_xi - 1), hy = 1.0 / (double)(n_eta - 1);
        r = cell_q(xs, ys, i, j, n_xi, hx, hy) / cell_q(xd, yd, i, j, n_xi, hx, hy);
        mx = r;
        if (r_cells) r_cells[c] = r;
    }
    smax[threadIdx.x] = mx;
    ssum[threadIdx.x] = r;
    __syncthreads();
    for (int w = kQualityBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            ssum[threadIdx.x] = ssum[threadIdx.x] + ssum[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_max[blockIdx.x] = smax[0];
        part_sum[blockIdx.x] = ssum[0];
    }
}

// One workgroup: partials in block order -> (max, mean).
__global__ __launch_bounds__(kQualityBlock) void quality_final_kernel(const double *__restrict__ part_max,
                                                                     const double *__restrict__ part_sum,
                                                                     int n_parts, int n_cells,
                                                                     double *__restrict__ out)
{
    __shared__ double smax[kQualityBlock], ssum[kQualityBlock];
    double mx = 0.0, sm = 0.0;
    for (int k = threadIdx.x; k < n_parts; k += kQualityBlock) {
        mx = fmax(mx, part_max[k]);
        sm = sm + part_sum[k];
    }
    smax[threadIdx.x] = mx;
    ssum[threadIdx.x] = sm;
    __syncthreads();
    for (int w = kQualityBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            ssum[threadIdx.x] = ssum[threadIdx.x] + ssum[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = smax[0];
        out[1] = ssum[0] / (double)n_cells;
    }
}

inline unsigned blocks_of(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// Piecewise-linear transfer of a nodal field between meshes (MᵏP, section 5)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int floor_div(int a, int m) { return a >= 0 ? a / m : -((-a + m - 1) / m); }

// Old-mesh node at grid indices (ii, jj) that may lie beyond a periodic
// seam: wrapped into range, with the period added to the winding coordinate.
__device__ __forceinline__ void old_node(const TransferArgs &a, int ii, int jj, double &x, double &y, double &f)
{
    double ox = 0.0, oy = 0.0;
    if (a.per_xi) {
        const int q = floor_div(ii, a.n_xi - 1);
        ii -= q * (a.n_xi - 1);
        ox = (double)q * a.Lx;
    }
    if (a.per_eta) {
        const int q = floor_div(jj, a.n_eta - 1);
        jj -= q * (a.n_eta - 1);
        oy = (double)q * a.Ly;
    }
    const size_t k = (size_t)jj * a.n_xi + ii;
    x = a.x_old[k] + ox;
    y = a.y_old[k] + oy;
    f = a.f_old[k];
}

// Barycentric test of point p against triangle (A, B, C): the smallest
// coordinate and the linear interpolant of the vertex values.
__device__ __forceinline__ void tri_test(double px, double py, double ax, double ay, double af, double bx, double by,
                                         double bf, double cx, double cy, double cf, double &lmin, double &val)
{
    const double e1x = bx - ax, e1y = by - ay, e2x = cx - ax, e2y = cy - ay;
    const double det = e1x * e2y - e1y * e2x;
    const double dx = px - ax, dy = py - ay;
    const double lb = (dx * e2y - dy * e2x) / det;
    const double lc = (e1x * dy - e1y * dx) / det;
    const double la = 1.0 - lb - lc;
    lmin = fmin(fmin(la, lb), lc);
    val = la * af + lb * bf + lc * cf;
}

// One thread per new node.  The search starts with the 4 x 4 old cells
// around the node's own grid position (a mesh step moves a node by about a
// cell at most) and doubles the window until a triangle contains the point
// (smallest coordinate >= -1e-10: a point on a shared edge or a rounding
// error outside the mesh) or the window covers the whole mesh (with its
// periodic images), so every thread ends.
__global__ void transfer_p1_kernel(TransferArgs a)
{
    const int idx = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (idx >= a.n_xi * a.n_eta) return;
    int i = idx % a.n_xi, j = idx / a.n_xi;
    if (a.per_xi && i == a.n_xi - 1) i = 0;     // image node: node 0's value
    if (a.per_eta && j == a.n_eta - 1) j = 0;
    const double px = a.x_new[(size_t)j * a.n_xi + i], py = a.y_new[(size_t)j * a.n_xi + i];
    const int cxm = a.n_xi - 2, cym = a.n_eta - 2;   // last cell index per axis
    double best = -INFINITY, bval = 0.0;
    for (int w = 2;; w *= 2) {
        int i0 = i - w, i1 = i + w - 1, j0 = j - w, j1 = j + w - 1;
        if (!a.per_xi) {
            i0 = max(i0, 0);
            i1 = min(i1, cxm);
        }
        if (!a.per_eta) {
            j0 = max(j0, 0);
            j1 = min(j1, cym);
        }
        for (int cj = j0; cj <= j1; ++cj) {
            for (int ci = i0; ci <= i1; ++ci) {
                double ax, ay, af, bx, by, bf, cx, cy, cf, dx, dy, df;
                old_node(a, ci, cj, ax, ay, af);
                old_node(a, ci + 1, cj, bx, by, bf);
                old_node(a, ci + 1, cj + 1, cx, cy, cf);
                old_node(a, ci, cj + 1, dx, dy, df);
                double l, v;
                tri_test(px, py, ax, ay, af, bx, by, bf, cx, cy, cf, l, v);
                if (l > best) {
                    best = l;
                    bval = v;
                }
                tri_test(px, py, ax, ay, af, cx, cy, cf, dx, dy, df, l, v);
                if (l > best) {
                    best = l;
                    bval = v;
                }
            }
        }
        if (best >= -1e-10) break;
        const bool all_xi = a.per_xi ? w >= 2 * (a.n_xi - 1) : (i0 == 0 && i1 == cxm);
        const bool all_eta = a.per_eta ? w >= 2 * (a.n_eta - 1) : (j0 == 0 && j1 == cym);
        if (all_xi && all_eta) break;
    }
    a.f_new[idx] = bval;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
size_t edge_gen_lds_bytes(int n_max) { return (size_t)3 * (size_t)n_max * sizeof(double); }

hipError_t launch_edge_gen(const double *rho, const double *rho_xi, const double *rho_eta, int n_xi, int n_eta,
                           int per_xi, int per_eta, double Lx, double Ly, double tau, int L_eta, int L_xi,
                           double *bnd, hipStream_t s)
{
    const int sides = (per_xi ? 0 : 2) + (per_eta ? 0 : 2);
    if (sides == 0) return hipSuccess;
    const int n_max = per_xi ? n_xi : (per_eta ? n_eta : (n_xi > n_eta ? n_xi : n_eta));
    hipLaunchKernelGGL(edge_gen_kernel, dim3(sides), dim3(kEdgeBlock), edge_gen_lds_bytes(n_max), s, rho, rho_xi,
                       rho_eta, n_xi, n_eta, per_xi, per_eta, Lx, Ly, tau, L_eta, L_xi, bnd);
    return hipGetLastError();
}

hipError_t launch_targets(const MeshStepArgs &a, double *x_new, double *y_new, hipStream_t s)
{
    const size_t n = (size_t)a.n_xi * a.n_eta;
    hipLaunchKernelGGL(targets_kernel, dim3(blocks_of(n, 256)), dim3(256), 0, s, a, x_new, y_new);
    return hipGetLastError();
}

size_t subdomain_lds_bytes(int P_xi, int P_eta) { return (size_t)2 * (P_xi + 1) * (P_eta + 1) * sizeof(double); }

bool subdomain_fits_lds(int P_xi, int P_eta)
{
    const long nin = (long)(P_xi - 1) * (P_eta - 1);
    const long nb = 2L * (P_xi + 1) + 2L * (P_eta - 1);
    return P_xi >= 2 && P_eta >= 2 && nin <= (long)kSubBlock * kSubPerThread && nb <= kSubBlock &&
           subdomain_lds_bytes(P_xi, P_eta) <= kSubLdsMax;
}

hipError_t launch_subdomain_lds(const MeshStepArgs &a, double *x_new, double *y_new, hipStream_t s)
{
    hipLaunchKernelGGL(subdomain_lds_kernel, dim3(a.sub_xi * a.sub_eta), dim3(kSubBlock),
                       subdomain_lds_bytes(a.P_xi, a.P_eta), s, a, x_new, y_new);
    return hipGetLastError();
}

hipError_t launch_fe_sweep(const MeshStepArgs &a, const double *cx, const double *cy, double *nx, double *ny,
                           double th1, hipStream_t s)
{
    const size_t n = (size_t)a.n_xi * a.n_eta;
    hipLaunchKernelGGL(fe_sweep_kernel, dim3(blocks_of(n, 256)), dim3(256), 0, s, a, cx, cy, nx, ny, th1);
    return hipGetLastError();
}

hipError_t launch_arclength(const double *u, const double *x, const double *y, int n_xi, int n_eta, int per_xi,
                            int per_eta, double Lx, double Ly, double alpha, int normalize, double *g_scratch,
                            unsigned long long *gmax_bits, unsigned int *bad, double *rho, hipStream_t s)
{
    const size_t n = (size_t)n_xi * n_eta;
    hipLaunchKernelGGL(arclength_grad_kernel, dim3(blocks_of(n, 256)), dim3(256), 0, s, u, x, y, n_xi, n_eta, per_xi,
                       per_eta, Lx, Ly, g_scratch, gmax_bits, bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(arclength_rho_kernel, dim3(blocks_of(n, 256)), dim3(256), 0, s, g_scratch, (int)n, alpha,
                       normalize, gmax_bits, rho);
    return hipGetLastError();
}

hipError_t launch_transfer_p1(const TransferArgs &a, hipStream_t s)
{
    const size_t n = (size_t)a.n_xi * a.n_eta;
    hipLaunchKernelGGL(transfer_p1_kernel, dim3(blocks_of(n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

int quality_parts(int n_xi, int n_eta) { return (int)blocks_of((size_t)(n_xi - 1) * (n_eta - 1), kQualityBlock); }

hipError_t launch_quality(const double *xs, const double *ys, const double *xd, const double *yd, int n_xi,
                          int n_eta, double *r_cells, double *part_max, double *part_sum, double *out2,
                          hipStream_t s)
{
    const int parts = quality_parts(n_xi, n_eta);
    hipLaunchKernelGGL(quality_kernel, dim3(parts), dim3(kQualityBlock), 0, s, xs, ys, xd, yd, n_xi, n_eta, r_cells,
                       part_max, part_sum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(quality_final_kernel, dim3(1), dim3(kQualityBlock), 0, s, part_max, part_sum, parts,
                       (n_xi - 1) * (n_eta - 1), out2);
    return hipGetLastError();
}

}  // namespace msdd
