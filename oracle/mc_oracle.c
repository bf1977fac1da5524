/*
 * Plain FP64 CPU oracle for the Monte-Carlo interface-node estimate of the
 * linearised parabolic mesh generator of Bihlo, Haynes & Walsh,
 * "Stochastic domain decomposition for time dependent adaptive mesh
 * generation" (arXiv:1504.00084).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with
 * the GPU path.  It is deliberately slow and literal: one path at a time,
 * every step written in the order of the method, FP64 throughout, sums taken
 * serially in path order.  The only parallelism is a pool of threads that
 * each take whole interface nodes.
 *
 * What it computes (paper section 3):
 *   - the mesh generator (Gen), eq. (ParabolicWinslowGeneratorPeriodicDomain):
 *       x_t = (grad rho / rho) . grad x + lap x   (same for y),
 *     with rho frozen at t^n (section 3.2, MP linearisation);
 *   - its Dirichlet stochastic representation, eq. (...StochasticSolutionA):
 *       x = E[x0(Phi(t)) 1{exit > t}] + E[f(t - exit, Phi(exit)) 1{exit < t}],
 *     and the periodic (Kac-Feynman) one, eq. (StochasticSolutionPeriodic...),
 *     driven by the SDE dPhi = (grad rho / rho) dt + sqrt(2) dW
 *     (eq. ...StochasticSolutionB);
 *   - the Euler-Maruyama scheme of section 3.4, eq.
 *     (WinslowGeneratorSDEDiscretization), with K substeps dt_s = tau / K,
 *     finite-difference grad rho, bilinear interpolation of rho and grad rho,
 *     bicubic interpolation of the mesh at the step start for survivors,
 *     a linear Brownian-bridge boundary test per substep for Dirichlet
 *     sides, no boundary test on periodic axes, and the arithmetic mean over
 *     N paths (section 3.4).
 *
 * Readings taken where the paper is silent (each one is listed with its
 * reason in the design notes of the repository):
 *   R1 bicubic = Keys cubic convolution, a = -1/2, Keys' end rule for ghosts;
 *   R2 grad rho: central differences inside, second-order one-sided at
 *      Dirichlet edges, wrapped on periodic axes;
 *   R3 the three fields rho, rho_xi, rho_eta are interpolated, then divided;
 *   R4 bridge: crossing probability exp(-d0 d1 / dt_s) per Dirichlet side
 *      (Brownian bridge of variance 2 dt_s), sides combined as independent,
 *      exit side = largest probability (lower index on ties), exit time =
 *      end of the substep, exit point = new position moved onto the side;
 *   R5 boundary data linear in time between the arrays at t^n and t^{n+1};
 *   R6 a periodic axis has n nodes with node n-1 the image of node 0; the
 *      mesh is quasi-periodic, x(xi+1) = x(xi) + Lx, y(eta+1) = y(eta) + Ly;
 *   R7 the periodic seam is an interface;
 *   R8 paths that wrap carry a winding number that adds w*L at evaluation;
 *   R13 random numbers: Philox4x32-10 (Salmon et al., SC'11), stream
 *      layout below, uniforms ((r >> 9) + 1/2) 2^-23, Box-Muller normals;
 *   R14 unbiased variance from shifted sums.
 *
 * Stream layout (R13).  Path p of interface node `node` (its rank in the
 * row-major interface enumeration), instance id I and mesh step S owns the
 * word sequence w_0, w_1, ... where w_q is word (q mod 4) of the Philox
 * block with counter (q div 4, p, node, I<<16 | S&0xffff) and key
 * (seed & 0xffffffff, seed >> 32).  Substep k uses w_{3k}, w_{3k+1}
 * (Box-Muller -> the two normals) and w_{3k+2} (the bridge uniform).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Problem description (the oracle's own; no header is shared with the GPU) */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_xi, n_eta;           /* grid nodes per axis                  */
    int32_t sub_xi, sub_eta;       /* subdomains per axis                  */
    int32_t periodic_xi, periodic_eta;
    double Lx, Ly;                 /* physical extents                     */
    double tau;                    /* mesh time step Delta t               */
    int32_t K;                     /* Euler-Maruyama substeps              */
    int32_t bridge;                /* 1: Brownian-bridge test on           */
    uint64_t seed;
    uint32_t instance_id;
    uint32_t mesh_step;
} oracle_problem;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror and  */
/* Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).             */
/* One round maps (x0,x1,x2,x3) under key (k0,k1) to                        */
/*   (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0)),       */
/* and the key is bumped by the Weyl constants between rounds.              */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = M0 * (uint64_t)x0;
        uint64_t prod1 = M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform in (0,1): ((r >> 9) + 1/2) * 2^-23.  The 24-bit odd numerator is
 * exact in binary32 as well as binary64. */
double oracle_uniform(uint32_t r)
{
    return ((double)(r >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* Box-Muller: two uniforms -> two independent standard normals. */
void oracle_box_muller(uint32_t r0, uint32_t r1, double *n1, double *n2)
{
    const double two_pi = 6.283185307179586476925286766559;
    double u0 = oracle_uniform(r0);
    double u1 = oracle_uniform(r1);
    double radius = sqrt(-2.0 * log(u0));
    *n1 = radius * cos(two_pi * u1);
    *n2 = radius * sin(two_pi * u1);
}

/* Word q of the stream of one path (stream layout R13). */
uint32_t oracle_stream_word(const oracle_problem *P, int32_t node, int64_t path, int64_t q)
{
    uint32_t ctr[4], key[2], r[4];
    ctr[0] = (uint32_t)(q / 4);
    ctr[1] = (uint32_t)path;
    ctr[2] = (uint32_t)node;
    ctr[3] = (P->instance_id << 16) | (P->mesh_step & 0xFFFFu);
    key[0] = (uint32_t)(P->seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(P->seed >> 32);
    oracle_philox4x32_10(ctr, key, r);
    return r[q % 4];
}

/* The two standard normals that drive substep k of path `path` at `node`. */
void oracle_normals(const oracle_problem *P, int32_t node, int64_t path, int32_t k,
                    double *n1, double *n2)
{
    uint32_t a = oracle_stream_word(P, node, path, 3 * (int64_t)k);
    uint32_t b = oracle_stream_word(P, node, path, 3 * (int64_t)k + 1);
    oracle_box_muller(a, b, n1, n2);
}

/* The uniform that drives the bridge test of substep k. */
double oracle_bridge_uniform(const oracle_problem *P, int32_t node, int64_t path, int32_t k)
{
    return oracle_uniform(oracle_stream_word(P, node, path, 3 * (int64_t)k + 2));
}

/* ------------------------------------------------------------------------ */
/* Grid helpers                                                              */
/* ------------------------------------------------------------------------ */

/* Index of a node along an axis after periodic wrapping over the n-1
 * distinct nodes; `*period` receives how many periods were crossed. */
static int wrap_index(int i, int n, int *period)
{
    int m = n - 1;
    int q = (i >= 0) ? i / m : -((-i + m - 1) / m);
    *period = q;
    return i - q * m;
}

/* Cell containing coordinate a in [0,1] along an axis with n nodes, and the
 * local coordinate in that cell.  Dirichlet: the last node belongs to the
 * last cell.  Periodic: cell index may come out as n-1 by rounding; the
 * callers wrap it. */
static void locate(double a, int n, int periodic, int *cell, double *frac)
{
    double s = a * (double)(n - 1);
    int c = (int)floor(s);
    if (!periodic && c > n - 2) c = n - 2;
    if (!periodic && c < 0) c = 0;
    *cell = c;
    *frac = s - (double)c;
}

/* ------------------------------------------------------------------------ */
/* (a0) Finite-difference gradient of the frozen monitor (section 3.4:      */
/* grad rho by finite differences; stencils by reading R2).                  */
/* ------------------------------------------------------------------------ */
void oracle_monitor_gradient(int32_t n_xi, int32_t n_eta, int32_t per_xi, int32_t per_eta,
                             const double *rho, double *rho_xi, double *rho_eta)
{
    double h_xi = 1.0 / (double)(n_xi - 1), h_eta = 1.0 / (double)(n_eta - 1);
    for (int j = 0; j < n_eta; ++j) {
        for (int i = 0; i < n_xi; ++i) {
            double d;
            /* xi direction */
            if (per_xi) {
                int pd, ii = wrap_index(i, n_xi, &pd);
                int ip = wrap_index(ii + 1, n_xi, &pd), im = wrap_index(ii - 1, n_xi, &pd);
                d = (rho[j * n_xi + ip] - rho[j * n_xi + im]) / (2.0 * h_xi);
            } else if (i == 0) {
                d = (-3.0 * rho[j * n_xi + 0] + 4.0 * rho[j * n_xi + 1] - rho[j * n_xi + 2]) / (2.0 * h_xi);
            } else if (i == n_xi - 1) {
                d = (3.0 * rho[j * n_xi + i] - 4.0 * rho[j * n_xi + i - 1] + rho[j * n_xi + i - 2]) / (2.0 * h_xi);
            } else {
                d = (rho[j * n_xi + i + 1] - rho[j * n_xi + i - 1]) / (2.0 * h_xi);
            }
            rho_xi[j * n_xi + i] = d;
            /* eta direction */
            if (per_eta) {
                int pd, jj = wrap_index(j, n_eta, &pd);
                int jp = wrap_index(jj + 1, n_eta, &pd), jm = wrap_index(jj - 1, n_eta, &pd);
                d = (rho[jp * n_xi + i] - rho[jm * n_xi + i]) / (2.0 * h_eta);
            } else if (j == 0) {
                d = (-3.0 * rho[0 * n_xi + i] + 4.0 * rho[1 * n_xi + i] - rho[2 * n_xi + i]) / (2.0 * h_eta);
            } else if (j == n_eta - 1) {
                d = (3.0 * rho[j * n_xi + i] - 4.0 * rho[(j - 1) * n_xi + i] + rho[(j - 2) * n_xi + i]) / (2.0 * h_eta);
            } else {
                d = (rho[(j + 1) * n_xi + i] - rho[(j - 1) * n_xi + i]) / (2.0 * h_eta);
            }
            rho_eta[j * n_xi + i] = d;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* (a1) Interface nodes (section 3.5 with reading R7): node (i,j) lies on   */
/* an artificial interface when i is a multiple of (n_xi-1)/sub_xi or j is  */
/* a multiple of (n_eta-1)/sub_eta, and it is not on the physical boundary.  */
/* Order: row-major in (j, i).  Returns the count; fills i_out/j_out when   */
/* they are not NULL.                                                        */
/* ------------------------------------------------------------------------ */
int32_t oracle_interface_nodes(const oracle_problem *P, int32_t *i_out, int32_t *j_out)
{
    int32_t pxi = (P->n_xi - 1) / P->sub_xi, peta = (P->n_eta - 1) / P->sub_eta;
    int32_t count = 0;
    for (int j = 0; j < P->n_eta; ++j) {
        for (int i = 0; i < P->n_xi; ++i) {
            int on_boundary;
            if (P->periodic_xi) {
                if (i == P->n_xi - 1) continue;   /* image of node 0 */
            }
            if (P->periodic_eta) {
                if (j == P->n_eta - 1) continue;
            }
            on_boundary = (!P->periodic_xi && (i == 0 || i == P->n_xi - 1)) ||
                          (!P->periodic_eta && (j == 0 || j == P->n_eta - 1));
            if (on_boundary) continue;
            if (i % pxi == 0 || j % peta == 0) {
                if (i_out) i_out[count] = i;
                if (j_out) j_out[count] = j;
                ++count;
            }
        }
    }
    return count;
}

/* ------------------------------------------------------------------------ */
/* (a4) Bilinear interpolation of rho, rho_xi, rho_eta at (xi, eta)          */
/* (section 3.4: bilinear interpolation of rho and grad rho).               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_xi, n_eta, per_xi, per_eta;
    const double *rho, *rho_xi, *rho_eta;
} monitor_table;

static double table_node(const double *f, const monitor_table *T, int i, int j)
{
    int pd;
    if (T->per_xi) i = wrap_index(i, T->n_xi, &pd);
    if (T->per_eta) j = wrap_index(j, T->n_eta, &pd);
    return f[j * T->n_xi + i];
}

static double bilinear_field(const double *f, const monitor_table *T, int ci, int cj, double tx, double ty)
{
    double f00 = table_node(f, T, ci, cj), f10 = table_node(f, T, ci + 1, cj);
    double f01 = table_node(f, T, ci, cj + 1), f11 = table_node(f, T, ci + 1, cj + 1);
    return (1.0 - tx) * (1.0 - ty) * f00 + tx * (1.0 - ty) * f10 + (1.0 - tx) * ty * f01 + tx * ty * f11;
}

static void bilinear3(const monitor_table *T, double xi, double eta, double *r, double *rx, double *ry)
{
    int ci, cj;
    double tx, ty;
    locate(xi, T->n_xi, T->per_xi, &ci, &tx);
    locate(eta, T->n_eta, T->per_eta, &cj, &ty);
    *r = bilinear_field(T->rho, T, ci, cj, tx, ty);
    *rx = bilinear_field(T->rho_xi, T, ci, cj, tx, ty);
    *ry = bilinear_field(T->rho_eta, T, ci, cj, tx, ty);
}

/* Partial derivatives in (xi, eta) of the bilinear interpolant inside cell
 * (ci, cj) at local coordinates (tx, ty). */
static void bilinear_field_grad(const double *f, const monitor_table *T, int ci, int cj, double tx, double ty,
                                double *f_xi, double *f_eta)
{
    double f00 = table_node(f, T, ci, cj), f10 = table_node(f, T, ci + 1, cj);
    double f01 = table_node(f, T, ci, cj + 1), f11 = table_node(f, T, ci + 1, cj + 1);
    *f_xi = (double)(T->n_xi - 1) * ((1.0 - ty) * (f10 - f00) + ty * (f11 - f01));
    *f_eta = (double)(T->n_eta - 1) * ((1.0 - tx) * (f01 - f00) + tx * (f11 - f10));
}

/* Jacobian of one Euler-Maruyama substep's deterministic part,
 * I + dt grad(b), b = (rho_xi / rho, rho_eta / rho) interpolated as in
 * bilinear3, at (xi, eta): row-major a[4]. */
static void substep_jacobian(const monitor_table *T, double xi, double eta, double dt, double a[4])
{
    int ci, cj;
    double tx, ty, r, gx, gy, r_xi, r_eta, gx_xi, gx_eta, gy_xi, gy_eta;
    locate(xi, T->n_xi, T->per_xi, &ci, &tx);
    locate(eta, T->n_eta, T->per_eta, &cj, &ty);
    r = bilinear_field(T->rho, T, ci, cj, tx, ty);
    gx = bilinear_field(T->rho_xi, T, ci, cj, tx, ty);
    gy = bilinear_field(T->rho_eta, T, ci, cj, tx, ty);
    bilinear_field_grad(T->rho, T, ci, cj, tx, ty, &r_xi, &r_eta);
    bilinear_field_grad(T->rho_xi, T, ci, cj, tx, ty, &gx_xi, &gx_eta);
    bilinear_field_grad(T->rho_eta, T, ci, cj, tx, ty, &gy_xi, &gy_eta);
    /* d(g / r) = (dg r - g dr) / r^2 */
    a[0] = 1.0 + dt * (gx_xi * r - gx * r_xi) / (r * r);
    a[1] = dt * (gx_eta * r - gx * r_eta) / (r * r);
    a[2] = dt * (gy_xi * r - gy * r_xi) / (r * r);
    a[3] = 1.0 + dt * (gy_eta * r - gy * r_eta) / (r * r);
}

void oracle_bilinear(int32_t n_xi, int32_t n_eta, int32_t per_xi, int32_t per_eta,
                     const double *rho, const double *rho_xi, const double *rho_eta,
                     double xi, double eta, double out[3])
{
    monitor_table T = {n_xi, n_eta, per_xi, per_eta, rho, rho_xi, rho_eta};
    bilinear3(&T, xi, eta, &out[0], &out[1], &out[2]);
}

/* ------------------------------------------------------------------------ */
/* (a7) Bicubic interpolation of the mesh at the step start (section 3.4),  */
/* read as Keys' cubic convolution (R. Keys, IEEE TASSP 29, 1981) with      */
/* a = -1/2 and Keys' boundary rule f(-1) = 3 f(0) - 3 f(1) + f(2) (and its  */
/* mirror at the far end) on Dirichlet axes.  Periodic axes wrap the index  */
/* and add the quasi-periodic offset (R6).                                  */
/* ------------------------------------------------------------------------ */
static double keys_kernel(double s)
{
    const double a = -0.5;
    s = fabs(s);
    if (s <= 1.0) return (a + 2.0) * s * s * s - (a + 3.0) * s * s + 1.0;
    if (s < 2.0) return a * s * s * s - 5.0 * a * s * s + 8.0 * a * s - 4.0 * a;
    return 0.0;
}

typedef struct {
    int32_t n_xi, n_eta, per_xi, per_eta;
    const double *f;
    double off_xi, off_eta;  /* value added per period crossed along each axis */
} mesh_field;

/* Node value at integer (i, j) with i in [-1, n_xi], j in [-1, n_eta]:
 * ghosts on Dirichlet axes, wrapping with offsets on periodic axes. */
static double mesh_node(const mesh_field *F, int i, int j)
{
    if (!F->per_xi && i < 0)
        return 3.0 * mesh_node(F, 0, j) - 3.0 * mesh_node(F, 1, j) + mesh_node(F, 2, j);
    if (!F->per_xi && i > F->n_xi - 1) {
        int e = F->n_xi - 1;
        return 3.0 * mesh_node(F, e, j) - 3.0 * mesh_node(F, e - 1, j) + mesh_node(F, e - 2, j);
    }
    if (!F->per_eta && j < 0)
        return 3.0 * mesh_node(F, i, 0) - 3.0 * mesh_node(F, i, 1) + mesh_node(F, i, 2);
    if (!F->per_eta && j > F->n_eta - 1) {
        int e = F->n_eta - 1;
        return 3.0 * mesh_node(F, i, e) - 3.0 * mesh_node(F, i, e - 1) + mesh_node(F, i, e - 2);
    }
    double offset = 0.0;
    int pd;
    if (F->per_xi) {
        i = wrap_index(i, F->n_xi, &pd);
        offset += pd * F->off_xi;
    }
    if (F->per_eta) {
        j = wrap_index(j, F->n_eta, &pd);
        offset += pd * F->off_eta;
    }
    return F->f[j * F->n_xi + i] + offset;
}

static double keys_bicubic(const mesh_field *F, double xi, double eta)
{
    int ci, cj;
    double tx, ty, sum = 0.0;
    locate(xi, F->n_xi, F->per_xi, &ci, &tx);
    locate(eta, F->n_eta, F->per_eta, &cj, &ty);
    for (int b = -1; b <= 2; ++b)
        for (int a = -1; a <= 2; ++a)
            sum += keys_kernel(tx - a) * keys_kernel(ty - b) * mesh_node(F, ci + a, cj + b);
    return sum;
}

double oracle_keys_bicubic(int32_t n_xi, int32_t n_eta, int32_t per_xi, int32_t per_eta,
                           const double *f, double off_xi, double off_eta, double xi, double eta)
{
    mesh_field F = {n_xi, n_eta, per_xi, per_eta, f, off_xi, off_eta};
    return keys_bicubic(&F, xi, eta);
}

/* ------------------------------------------------------------------------ */
/* (a6) Brownian-bridge crossing probability for one side (reading R4): a   */
/* bridge of variance 2 dt between points at distances d0, d1 >= 0 from a   */
/* straight side crosses it with probability exp(-d0 d1 / dt).              */
/* ------------------------------------------------------------------------ */
double oracle_bridge_probability(double d0, double d1, double dt)
{
    return exp(-d0 * d1 / dt);
}

/* ------------------------------------------------------------------------ */
/* Boundary value at an exit point (eq. StochasticSolutionA, second term,   */
/* with reading R5).  Boundary arrays: side 0 (xi=0) and side 1 (xi=1) hold */
/* n_eta entries per component, side 2 (eta=0) and side 3 (eta=1) hold n_xi */
/* entries; layout [side0 x][side0 y][side1 x][side1 y][side2 x][side2 y]   */
/* [side3 x][side3 y].                                                       */
/* ------------------------------------------------------------------------ */
static const double *side_component(const oracle_problem *P, const double *bnd, int side, int comp, int *len)
{
    if (side < 2) {
        *len = P->n_eta;
        return bnd + (size_t)(side * 2 + comp) * P->n_eta;
    }
    *len = P->n_xi;
    return bnd + (size_t)4 * P->n_eta + (size_t)((side - 2) * 2 + comp) * P->n_xi;
}

static double side_linear(const double *arr, int len, double t)
{
    double s = t * (double)(len - 1);
    int c = (int)floor(s);
    if (c > len - 2) c = len - 2;
    if (c < 0) c = 0;
    double fr = s - (double)c;
    return (1.0 - fr) * arr[c] + fr * arr[c + 1];
}

static double boundary_value(const oracle_problem *P, const double *bnd_t0, const double *bnd_t1,
                             int side, int comp, double tangential, double elapsed)
{
    int len;
    const double *a0 = side_component(P, bnd_t0, side, comp, &len);
    const double *a1 = side_component(P, bnd_t1, side, comp, &len);
    double v0 = side_linear(a0, len, tangential);   /* at t^n     */
    double v1 = side_linear(a1, len, tangential);   /* at t^{n+1} */
    /* the path runs backward from t^{n+1}; after `elapsed` it sits at
     * t^{n+1} - elapsed, where linear interpolation in time gives: */
    return (elapsed / P->tau) * v0 + (1.0 - elapsed / P->tau) * v1;
}

/* ------------------------------------------------------------------------ */
/* One path (section 3.4): Euler-Maruyama with bridge test, wrap, and the   */
/* terminal or boundary value.                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    double vx, vy;
    int32_t exited;     /* 1 if the path left through a Dirichlet side */
    int32_t side;       /* exit side or -1 */
    int32_t steps;      /* substeps executed */
} path_outcome;

typedef struct {
    const oracle_problem *P;
    monitor_table T;
    mesh_field X, Y;
    const double *bnd_t0, *bnd_t1;
    int32_t track;       /* sensitivity only (oracle_path_amplification): when set, */
    double amp;          /* run_path leaves the path's rounding amplification here */
} solve_context;

/* trace (optional): per substep, 4 doubles (xi, eta after the step, before
 * any exit projection) -- used by the tiny brute-force comparison. */
static path_outcome run_path(solve_context *C, int32_t node, int32_t i0, int32_t j0, int64_t path,
                             double *trace)
{
    const oracle_problem *P = C->P;
    const double dt = P->tau / (double)P->K;
    const double sq = sqrt(2.0 * dt);
    double xi = (double)i0 / (double)(P->n_xi - 1);
    double eta = (double)j0 / (double)(P->n_eta - 1);
    long w_xi = 0, w_eta = 0;
    path_outcome out = {0.0, 0.0, 0, -1, 0};
    double S[3] = {0.0, 0.0, 0.0};   /* sensitivity only: symmetric 2x2 (xx, xy, yy) */
    if (C->track) C->amp = 0.0;       /* (the estimate's threads share C and never write it) */

    for (int k = 0; k < P->K; ++k) {
        double n1, n2, r, rx, ry;
        oracle_normals(P, node, path, k, &n1, &n2);
        if (C->track) {   /* S <- A S A^T + I, A the Jacobian of this substep */
            double a[4];
            substep_jacobian(&C->T, xi, eta, dt, a);
            double t0 = a[0] * S[0] + a[1] * S[1], t1 = a[0] * S[1] + a[1] * S[2];
            double t2 = a[2] * S[0] + a[3] * S[1], t3 = a[2] * S[1] + a[3] * S[2];
            S[0] = t0 * a[0] + t1 * a[1] + 1.0;
            S[1] = t0 * a[2] + t1 * a[3];
            S[2] = t2 * a[2] + t3 * a[3] + 1.0;
            double amp = sqrt(0.5 * (S[0] + S[2]));
            if (amp > C->amp) C->amp = amp;
        }
        bilinear3(&C->T, xi, eta, &r, &rx, &ry);
        double nxi = xi + (rx / r) * dt + sq * n1;
        double neta = eta + (ry / r) * dt + sq * n2;

        if (P->periodic_xi) {
            double m = floor(nxi);
            nxi -= m;
            w_xi += (long)m;
            if (nxi >= 1.0) { nxi -= 1.0; w_xi += 1; }
        }
        if (P->periodic_eta) {
            double m = floor(neta);
            neta -= m;
            w_eta += (long)m;
            if (neta >= 1.0) { neta -= 1.0; w_eta += 1; }
        }
        if (trace) {
            trace[4 * k + 0] = nxi;
            trace[4 * k + 1] = neta;
            trace[4 * k + 2] = n1;
            trace[4 * k + 3] = n2;
        }

        /* endpoint outside a Dirichlet side: exit; several sides out -> the
         * corner, side = first crossed in the order xi=0, xi=1, eta=0, eta=1 */
        int side = -1;
        if (!P->periodic_xi) {
            if (nxi < 0.0) { side = 0; nxi = 0.0; }
            else if (nxi > 1.0) { side = 1; nxi = 1.0; }
        }
        if (!P->periodic_eta) {
            if (neta < 0.0) { if (side < 0) side = 2; neta = 0.0; }
            else if (neta > 1.0) { if (side < 0) side = 3; neta = 1.0; }
        }

        /* Brownian-bridge test when both ends are inside */
        if (side < 0 && P->bridge) {
            double p[4] = {0.0, 0.0, 0.0, 0.0};
            if (!P->periodic_xi) {
                p[0] = oracle_bridge_probability(xi, nxi, dt);
                p[1] = oracle_bridge_probability(1.0 - xi, 1.0 - nxi, dt);
            }
            if (!P->periodic_eta) {
                p[2] = oracle_bridge_probability(eta, neta, dt);
                p[3] = oracle_bridge_probability(1.0 - eta, 1.0 - neta, dt);
            }
            double stay = (1.0 - p[0]) * (1.0 - p[1]) * (1.0 - p[2]) * (1.0 - p[3]);
            double q = 1.0 - stay;
            double u2 = oracle_bridge_uniform(P, node, path, k);
            if (u2 < q) {
                int best = 0;
                for (int s = 1; s < 4; ++s)
                    if (p[s] > p[best]) best = s;
                side = best;
                if (side == 0) nxi = 0.0;
                if (side == 1) nxi = 1.0;
                if (side == 2) neta = 0.0;
                if (side == 3) neta = 1.0;
            }
        }

        if (side >= 0) {
            double elapsed = (double)(k + 1) * dt;
            double tangential = (side < 2) ? neta : nxi;
            out.vx = boundary_value(P, C->bnd_t0, C->bnd_t1, side, 0, tangential, elapsed);
            out.vy = boundary_value(P, C->bnd_t0, C->bnd_t1, side, 1, tangential, elapsed);
            if (P->periodic_xi) out.vx += (double)w_xi * P->Lx;
            if (P->periodic_eta) out.vy += (double)w_eta * P->Ly;
            out.exited = 1;
            out.side = side;
            out.steps = k + 1;
            return out;
        }
        xi = nxi;
        eta = neta;
    }

    /* survivor: mesh at t^n, bicubic, plus winding offsets */
    out.vx = keys_bicubic(&C->X, xi, eta);
    out.vy = keys_bicubic(&C->Y, xi, eta);
    if (P->periodic_xi) out.vx += (double)w_xi * P->Lx;
    if (P->periodic_eta) out.vy += (double)w_eta * P->Ly;
    out.steps = P->K;
    return out;
}

/* ------------------------------------------------------------------------ */
/* Per-node estimate (section 3.4: arithmetic mean over N repetitions;      */
/* reading R14 for the standard error).                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    solve_context C;
    int32_t n_nodes;
    const int32_t *node_rank;    /* ranks to solve                  */
    const int32_t *node_i, *node_j;
    int64_t n_paths;
    double *mean_x, *mean_y, *se_x, *se_y, *exit_frac;
    int64_t *steps_per_node;
    int32_t next;                /* shared work counter              */
} solve_job;

static void solve_one_node(solve_job *J, int idx)
{
    const oracle_problem *P = J->C.P;
    int32_t node = J->node_rank[idx];
    int32_t i0 = J->node_i[idx], j0 = J->node_j[idx];
    double ref_x = J->C.X.f[j0 * P->n_xi + i0];
    double ref_y = J->C.Y.f[j0 * P->n_xi + i0];
    double s1x = 0.0, s2x = 0.0, s1y = 0.0, s2y = 0.0;
    int64_t exits = 0, steps = 0;
    for (int64_t p = 0; p < J->n_paths; ++p) {
        path_outcome o = run_path(&J->C, node, i0, j0, p, NULL);
        double dx = o.vx - ref_x, dy = o.vy - ref_y;
        s1x += dx;
        s2x += dx * dx;
        s1y += dy;
        s2y += dy * dy;
        exits += o.exited;
        steps += o.steps;
    }
    double N = (double)J->n_paths;
    J->mean_x[idx] = ref_x + s1x / N;
    J->mean_y[idx] = ref_y + s1y / N;
    if (J->n_paths > 1) {
        double vx = (s2x - s1x * s1x / N) / (N - 1.0);
        double vy = (s2y - s1y * s1y / N) / (N - 1.0);
        J->se_x[idx] = sqrt((vx > 0.0 ? vx : 0.0) / N);
        J->se_y[idx] = sqrt((vy > 0.0 ? vy : 0.0) / N);
    } else {
        J->se_x[idx] = NAN;
        J->se_y[idx] = NAN;
    }
    J->exit_frac[idx] = (double)exits / N;
    if (J->steps_per_node) J->steps_per_node[idx] = steps;
}

static void *solve_worker(void *arg)
{
    solve_job *J = (solve_job *)arg;
    for (;;) {
        int idx = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
        if (idx >= J->n_nodes) break;
        solve_one_node(J, idx);
    }
    return NULL;
}

static void build_context(const oracle_problem *P, const double *rho, double *rho_xi, double *rho_eta,
                          const double *x_cur, const double *y_cur, const double *bnd_t0,
                          const double *bnd_t1, solve_context *C)
{
    oracle_monitor_gradient(P->n_xi, P->n_eta, P->periodic_xi, P->periodic_eta, rho, rho_xi, rho_eta);
    C->P = P;
    C->T.n_xi = P->n_xi; C->T.n_eta = P->n_eta;
    C->T.per_xi = P->periodic_xi; C->T.per_eta = P->periodic_eta;
    C->T.rho = rho; C->T.rho_xi = rho_xi; C->T.rho_eta = rho_eta;
    C->X.n_xi = P->n_xi; C->X.n_eta = P->n_eta;
    C->X.per_xi = P->periodic_xi; C->X.per_eta = P->periodic_eta;
    C->X.f = x_cur; C->X.off_xi = P->Lx; C->X.off_eta = 0.0;
    C->Y = C->X;
    C->Y.f = y_cur; C->Y.off_xi = 0.0; C->Y.off_eta = P->Ly;
    C->bnd_t0 = bnd_t0;
    C->bnd_t1 = bnd_t1;
    C->track = 0;
    C->amp = 0.0;
}

/*
 * Estimate (x, y) at t^{n+1} at the interface nodes whose ranks are listed
 * in node_rank[0..n_nodes) (ranks into the row-major interface enumeration;
 * NULL means all nodes, in order).  Arrays: rho, x_cur, y_cur are n_eta*n_xi
 * row-major; bnd_t0 / bnd_t1 as described at boundary_value().  Outputs have
 * n_nodes entries.  steps_per_node may be NULL.  Returns 0, or -1 on a bad
 * argument or allocation failure.
 */
int32_t oracle_solve(const oracle_problem *P, const double *rho, const double *x_cur, const double *y_cur,
                     const double *bnd_t0, const double *bnd_t1, int64_t n_paths,
                     int32_t n_nodes, const int32_t *node_rank, int32_t n_threads,
                     double *mean_x, double *mean_y, double *se_x, double *se_y, double *exit_frac,
                     int64_t *steps_per_node)
{
    if (!P || P->n_xi < 4 || P->n_eta < 4 || P->K < 1 || P->tau <= 0.0 || n_paths < 1) return -1;
    int32_t total = oracle_interface_nodes(P, NULL, NULL);
    int32_t *all_i = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    int32_t *all_j = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    int32_t *ranks = NULL, *sel_i = NULL, *sel_j = NULL;
    double *rho_xi = (double *)malloc(sizeof(double) * (size_t)P->n_xi * P->n_eta);
    double *rho_eta = (double *)malloc(sizeof(double) * (size_t)P->n_xi * P->n_eta);
    int32_t rc = -1;
    if (!all_i || !all_j || !rho_xi || !rho_eta) goto done;
    oracle_interface_nodes(P, all_i, all_j);
    if (!node_rank) n_nodes = total;
    ranks = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_nodes > 0 ? n_nodes : 1));
    sel_i = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_nodes > 0 ? n_nodes : 1));
    sel_j = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_nodes > 0 ? n_nodes : 1));
    if (!ranks || !sel_i || !sel_j) goto done;
    for (int q = 0; q < n_nodes; ++q) {
        int r = node_rank ? node_rank[q] : q;
        if (r < 0 || r >= total) goto done;
        ranks[q] = r;
        sel_i[q] = all_i[r];
        sel_j[q] = all_j[r];
    }

    solve_job J;
    memset(&J, 0, sizeof(J));
    build_context(P, rho, rho_xi, rho_eta, x_cur, y_cur, bnd_t0, bnd_t1, &J.C);
    J.n_nodes = n_nodes;
    J.node_rank = ranks;
    J.node_i = sel_i;
    J.node_j = sel_j;
    J.n_paths = n_paths;
    J.mean_x = mean_x; J.mean_y = mean_y; J.se_x = se_x; J.se_y = se_y;
    J.exit_frac = exit_frac;
    J.steps_per_node = steps_per_node;
    J.next = 0;

    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t tid[256];
    int started = 0;
    for (int t = 1; t < n_threads; ++t) {
        if (pthread_create(&tid[started], NULL, solve_worker, &J) == 0) ++started;
    }
    solve_worker(&J);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    rc = 0;
done:
    free(all_i); free(all_j); free(ranks); free(sel_i); free(sel_j);
    free(rho_xi); free(rho_eta);
    return rc;
}

/*
 * Per-path outcomes of one node for paths [p_begin, p_end): value, exit flag,
 * exit side and executed substeps, plus (if trace != NULL) the per-substep
 * position after wrapping and the two normals, 4 doubles per substep, K
 * substeps per path (unused entries after an exit are left untouched).
 */
int32_t oracle_paths(const oracle_problem *P, const double *rho, const double *x_cur, const double *y_cur,
                     const double *bnd_t0, const double *bnd_t1, int32_t node_rank,
                     int64_t p_begin, int64_t p_end, double *vx, double *vy, int32_t *exited,
                     int32_t *side, int32_t *steps, double *trace)
{
    if (!P || P->n_xi < 4 || P->n_eta < 4 || P->K < 1 || P->tau <= 0.0) return -1;
    int32_t total = oracle_interface_nodes(P, NULL, NULL);
    if (node_rank < 0 || node_rank >= total) return -1;
    int32_t *all_i = (int32_t *)malloc(sizeof(int32_t) * (size_t)total);
    int32_t *all_j = (int32_t *)malloc(sizeof(int32_t) * (size_t)total);
    double *rho_xi = (double *)malloc(sizeof(double) * (size_t)P->n_xi * P->n_eta);
    double *rho_eta = (double *)malloc(sizeof(double) * (size_t)P->n_xi * P->n_eta);
    if (!all_i || !all_j || !rho_xi || !rho_eta) {
        free(all_i); free(all_j); free(rho_xi); free(rho_eta);
        return -1;
    }
    oracle_interface_nodes(P, all_i, all_j);
    solve_context C;
    build_context(P, rho, rho_xi, rho_eta, x_cur, y_cur, bnd_t0, bnd_t1, &C);
    for (int64_t p = p_begin; p < p_end; ++p) {
        int64_t q = p - p_begin;
        path_outcome o = run_path(&C, node_rank, all_i[node_rank], all_j[node_rank], p,
                                  trace ? trace + (size_t)q * 4 * P->K : NULL);
        vx[q] = o.vx;
        vy[q] = o.vy;
        exited[q] = o.exited;
        side[q] = o.side;
        steps[q] = o.steps;
    }
    free(all_i); free(all_j); free(rho_xi); free(rho_eta);
    return 0;
}

/*
 * Sensitivity of each path to rounding, not an estimate.  A perturbation
 * e_k of the position after substep k (k = 1..s, s the substeps the path
 * ran), independent between substeps with unit variance per coordinate,
 * reaches the position after substep k as a deviation of covariance S_k:
 * S_1 = I, S_{k+1} = A_k S_k A_k^T + I with A_k = I + dt grad b the
 * Jacobian of substep k at the position before it (linearised).
 * amp[q] = max over k of sqrt(trace(S_k) / 2): the largest standard
 * deviation the path reaches per unit per-substep perturbation, sqrt(s)
 * where there is no drift.  The maximum over time, not the end value: a
 * deviation grown large in a steep stretch leaves the linear regime and
 * need not shrink again where the linearisation would contract it.
 */
int32_t oracle_path_amplification(const oracle_problem *P, const double *rho, const double *x_cur,
                                  const double *y_cur, const double *bnd_t0, const double *bnd_t1,
                                  int32_t node_rank, int64_t p_begin, int64_t p_end, double *amp)
{
    if (!P || P->n_xi < 4 || P->n_eta < 4 || P->K < 1 || P->tau <= 0.0) return -1;
    int32_t total = oracle_interface_nodes(P, NULL, NULL);
    if (node_rank < 0 || node_rank >= total) return -1;
    int32_t *all_i = (int32_t *)malloc(sizeof(int32_t) * (size_t)total);
    int32_t *all_j = (int32_t *)malloc(sizeof(int32_t) * (size_t)total);
    double *rho_xi = (double *)malloc(sizeof(double) * (size_t)P->n_xi * P->n_eta);
    double *rho_eta = (double *)malloc(sizeof(double) * (size_t)P->n_xi * P->n_eta);
    if (!all_i || !all_j || !rho_xi || !rho_eta) {
        free(all_i); free(all_j); free(rho_xi); free(rho_eta);
        return -1;
    }
    oracle_interface_nodes(P, all_i, all_j);
    solve_context C;
    build_context(P, rho, rho_xi, rho_eta, x_cur, y_cur, bnd_t0, bnd_t1, &C);
    C.track = 1;
    for (int64_t p = p_begin; p < p_end; ++p) {
        run_path(&C, node_rank, all_i[node_rank], all_j[node_rank], p, NULL);
        amp[p - p_begin] = C.amp;
    }
    free(all_i); free(all_j); free(rho_xi); free(rho_eta);
    return 0;
}
