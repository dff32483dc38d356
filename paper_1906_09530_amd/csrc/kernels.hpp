// Device-side parameter block and kernel launchers of the solver.
#pragma once

#include <hip/hip_runtime.h>

namespace cplbm {

constexpr int kMaxStages = 8;      // parallel cyclic reduction stages
constexpr int kBlockThreads = 1024;
constexpr int kElemsPerThread = 4;
constexpr int kBlockElems = kBlockThreads * kElemsPerThread;  // line elements per block (LDS)

// Everything a kernel needs, passed by value.
struct KParams {
    int nx, ny, bc_y, eos;
    int rows_per_block;  // row passes: whole rows per block
    int cols_per_block;  // column pass: whole columns per block
    int nstage;          // reduction stages of the line solve
    int kappa_zero;      // kappa == 0: the Laplacian is not needed
    double a, b, RT, A;  // EOS constants; A = a alpha(T)
    double k2, kappa, inv_tau, mu_cap, wall_ux;
    double cfd_a2, cfd_b4;  // a/2 and b/4 of Eq. 37 (h = 1)
    double pcr_c[kMaxStages], pcr_g[kMaxStages];
};

// Pass A over rows: rho = sum f, d/dx rho, d2/dx2 rho.  Writes rho, dxx.
hipError_t launch_rows_rho(const KParams &p, const double *f, double *rho, double *dxx,
                           hipStream_t s);
// Pass B over columns: d/dy rho, d2/dy2 rho, mu (Eq. 33), d/dy mu, F_y (Eq. 12).
hipError_t launch_cols_mu(const KParams &p, const double *rho, const double *dxx, double *mu,
                          double *fy, hipStream_t s);
// Pass C over rows: d/dx rho, d/dx mu, F_x, collision and streaming f -> fout.
hipError_t launch_rows_collide(const KParams &p, const double *f, const double *mu,
                               const double *fy, double *fout, hipStream_t s);
// Pass C in observation mode: rho, v = u + F/(2 rho), F_x (any output may be null).
hipError_t launch_rows_observe(const KParams &p, const double *f, const double *mu,
                               const double *fy, double *rho, double *vx, double *vy,
                               double *fx, hipStream_t s);
// f = feq(rho0, u0) (u0 pointers may be null: rest).
hipError_t launch_init_feq(const KParams &p, const double *rho0, const double *ux0,
                           const double *uy0, double *f, hipStream_t s);
// rho of f compared with prev: per-block max |rho - prev| and a non-finite
// flag into partial[2*block]; prev <- rho.  Then one block folds the partials
// into out[0] (max) and out[1] (flag).
hipError_t launch_rho_delta(const KParams &p, const double *f, double *prev, double *partial,
                            int nblocks, double *out, hipStream_t s);
int rho_delta_blocks(const KParams &p);

}  // namespace cplbm
