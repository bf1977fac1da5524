// Device-side interface of the mesh-step kernels (mesh_step.hip): the 1-D
// edge generator, the Dirichlet targets of the decomposed problem, the
// subdomain solves (LDS-resident or global sweeps), the arc-length monitor,
// the mesh-quality ratio and the piecewise-linear monitor transfer of the
// MᵏP variant.  All FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace msdd {

constexpr int kEdgeBlock = 256;
constexpr int kSubBlock = 1024;                 // one workgroup per subdomain
constexpr int kSubPerThread = 4;                // interior nodes per thread (registers; up to 65x65 subdomains)
constexpr size_t kSubLdsMax = 160u * 1024u;     // LDS of one CU on gfx950
constexpr int kQualityBlock = 256;

// Everything the targets / subdomain / sweep kernels read; device pointers.
struct MeshStepArgs {
    int n_xi, n_eta, sub_xi, sub_eta, P_xi, P_eta;
    int per_xi, per_eta, with_interfaces, L;
    double Lx, Ly, tau;
    const double *x0, *y0;                 // mesh at t^n [n_eta][n_xi]
    const double *bnd1;                    // boundary arrays at t^{n+1}
    const double *iface_x, *iface_y;       // interface estimate at t^{n+1}, by rank
    const int32_t *node_rank;              // [n_eta][n_xi]: interface rank or -1
    const double *rho, *rho_xi, *rho_eta;  // FP64 node tables of the frozen monitor
    double *tx1, *ty1;                     // Dirichlet values at t^{n+1} (written by the targets kernel)
    uint8_t *mask;                         // 1 on Dirichlet nodes
};

size_t edge_gen_lds_bytes(int n_max);
hipError_t launch_edge_gen(const double *rho, const double *rho_xi, const double *rho_eta, int n_xi, int n_eta,
                           int per_xi, int per_eta, double Lx, double Ly, double tau, int L_eta, int L_xi,
                           double *bnd, hipStream_t s);
hipError_t launch_targets(const MeshStepArgs &a, double *x_new, double *y_new, hipStream_t s);
size_t subdomain_lds_bytes(int P_xi, int P_eta);
bool subdomain_fits_lds(int P_xi, int P_eta);
hipError_t launch_subdomain_lds(const MeshStepArgs &a, double *x_new, double *y_new, hipStream_t s);
hipError_t launch_fe_sweep(const MeshStepArgs &a, const double *cx, const double *cy, double *nx, double *ny,
                           double th1, hipStream_t s);
hipError_t launch_arclength(const double *u, const double *x, const double *y, int n_xi, int n_eta, int per_xi,
                            int per_eta, double Lx, double Ly, double alpha, int normalize, double *g_scratch,
                            unsigned long long *gmax_bits, unsigned int *bad, double *rho, hipStream_t s);
// MᵏP monitor update (section 5): f at the nodes of a new mesh from the
// piecewise-linear interpolant of nodal values on an old mesh of the same
// grid.  Each old cell (i, j)-(i+1, j+1) is split along its diagonal from
// node (i, j) to node (i+1, j+1); a point takes the linear interpolant of
// the triangle that contains it (outside the old mesh: of the triangle
// whose smallest barycentric coordinate is largest).  Periodic axes extend
// the old mesh by its images (+Lx along xi, +Ly along eta); image nodes of
// the new mesh take node 0's value.
struct TransferArgs {
    int n_xi, n_eta, per_xi, per_eta;
    double Lx, Ly;
    const double *x_old, *y_old, *f_old;   // [n_eta][n_xi]
    const double *x_new, *y_new;
    double *f_new;
};
hipError_t launch_transfer_p1(const TransferArgs &a, hipStream_t s);

int quality_parts(int n_xi, int n_eta);
hipError_t launch_quality(const double *xs, const double *ys, const double *xd, const double *yd, int n_xi,
                          int n_eta, double *r_cells, double *part_max, double *part_sum, double *out2,
                          hipStream_t s);

}  // namespace msdd
