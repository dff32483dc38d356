/* Host driver of the oracle for the address and undefined-behaviour
 * sanitizers: a few steps of every collision, force and wall option on small
 * meshes (periodic and between walls, sliding, wetting), the convergence
 * loop and the observables.  Exits 0 when every field stays finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/cplbm_oracle.c"

static int run_case(int nx, int ny, int bc_y, int eos, int collision, int force, int wetting,
                    double alpha)
{
    orc_params p = {0};
    p.nx = nx;
    p.ny = ny;
    p.bc_y = bc_y;
    p.eos = eos;
    p.wall_ux = bc_y ? 0.01 : 0.0;
    p.a = eos == EOS_CS ? 1.0 : 2.0 / 49.0;
    p.b = eos == EOS_CS ? 4.0 : 2.0 / 21.0;
    p.R = 1.0;
    p.T = eos == EOS_CS ? 0.066 : 0.044;
    p.alpha_T = 1.3;
    p.kappa = force ? 0.0 : 0.05;
    p.tau = 0.9;
    p.k = 0.2;
    p.mu_cap = 6.0;
    p.cfd_alpha = alpha;
    p.collision = collision;
    p.force = force;
    p.s_e = 1.64;
    p.s_eps = 1.54;
    p.s_q = 1.2;
    p.wetting = wetting;
    p.mu_wall = -0.05;
    size_t N = (size_t)nx * ny;
    double *rho = malloc(sizeof(double) * N * 3), *ux = rho + N, *uy = rho + 2 * N;
    double *f = malloc(sizeof(double) * 9 * N);
    double lo = eos == EOS_CS ? 0.01 : 0.05, hi = eos == EOS_CS ? 0.35 : 7.0;
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            double r = hypot(x - nx / 2.0, y - ny / 2.0);
            rho[(size_t)y * nx + x] = lo + (hi - lo) * 0.5 * (1.0 - tanh((r - nx / 4.0) / 2.0));
            ux[(size_t)y * nx + x] = 0.0;
            uy[(size_t)y * nx + x] = 0.0;
        }
    orc_init(&p, rho, ux, uy, f);
    orc_run(&p, f, 3);
    int64_t steps = 0;
    double delta = 0.0;
    orc_run_until_converged(&p, f, 1e-30, 2, 4, &steps, &delta);
    double *o = malloc(sizeof(double) * 6 * N);
    orc_moments(&p, f, o, o + N, o + 2 * N, o + 3 * N, o + 4 * N, o + 5 * N);
    int ok = 1;
    for (size_t i = 0; i < 6 * N; i++) ok &= isfinite(o[i]);
    free(o);
    free(f);
    free(rho);
    return ok;
}

int main(void)
{
    int ok = 1;
    ok &= run_case(12, 10, 0, EOS_CS, 0, 0, 0, 1.0 / 3.0);
    ok &= run_case(9, 7, 1, EOS_PR, 1, 0, 0, 0.25);
    ok &= run_case(8, 12, 1, EOS_CS, 0, 0, 1, 1.0 / 3.0);
    ok &= run_case(10, 8, 1, EOS_CS, 1, 1, 0, 1.0 / 3.0);
    ok &= run_case(3, 5, 0, EOS_RKS, 0, 0, 0, 1.0 / 3.0);
    double M[81], Mi[81];
    orc_mrt_matrix(M);
    orc_mrt_inverse(Mi);
    printf(ok ? "sanitized oracle: ok\n" : "sanitized oracle: non-finite\n");
    return ok ? 0 : 1;
}
