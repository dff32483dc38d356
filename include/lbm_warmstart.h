/*
 * lbm_warmstart.h -- C ABI of the learned warm start of libcplbm.
 *
 * The paper initialises a static drop with a tanh profile between the
 * Maxwell densities and zero velocity (Sec. 5.3, Eq. 41).  This extension
 * proposes the initial density and velocity with a small network instead,
 * trained on converged drops that the solver itself produced, so that the
 * solver reaches its convergence criterion in fewer steps.  The velocity
 * matters: a drop relaxes towards a steady state that carries the small
 * parasitic currents of the discretisation, and a start at rest takes as
 * long to build them up as the tanh start does, whatever its density.  The
 * solver, its criterion and its converged fields are unchanged: the network
 * only chooses the starting point, and the tanh start remains the fallback.
 *
 * Network (FP32 parameters, one flat array of LBM_MLP_PARAMS floats, in this
 * order): W1 [128][7], b1 [128], W2 [128][128], b2 [128], W3 [3][128], b3 [3];
 *     a1 = tanh(W1 x + b1), a2 = tanh(W2 a1 + b2), y = W3 a2 + b3.
 * Training minimises the mean over samples of sum_j (y_j - t_j)^2 with Adam
 * (Kingma and Ba, ICLR 2015, bias-corrected moments), FP32 throughout.
 * Inference runs either in FP32 or with the 128 x 128 product in bfloat16 on
 * the matrix cores (FP32 accumulation; bfloat16 = binary32 rounded to
 * nearest, ties to even, upper 16 bits).
 *
 * Warm-start features of a node of a drop of radius R centred at (cx, cy):
 * f = (T/Tc, R / 256, kappa, k, r - R, cos 4 theta, sin 4 theta), r the plain
 * distance to the centre in mesh nodes and theta the polar angle about it
 * (0 at the centre), normalised as x_i = (f_i - c_i) / s_i with
 * c = (0.5, 0.25, 0.1, 0.25, 0, 0, 0) and s = (0.25, 0.1, 0.1, 0.1, 8, 1, 1).
 * The angle enters as 4 theta: a drop centred in a square periodic mesh
 * keeps the square's symmetry.  Outputs: the normalised log density
 *     y0 = (ln rho - ln rho_g) / (ln rho_l - ln rho_g),
 * (rho_g, rho_l) the Maxwell pair at T (Sec. 5.1), and the radial and
 * azimuthal fluid velocity in units of 1e-3, y1 = 1e3 v_r, y2 = 1e3 v_theta
 * (v = u + F/(2 rho), the velocity the solver reports, Eq. 5).
 *
 * Memory: x, t, y, order, rho, ux and uy arguments are device pointers; params,
 * grad and losses are host pointers.  Work is enqueued on the stream given
 * at creation (NULL: the default stream); calls that return host data
 * synchronise it.  Errors as in lbm.h; lbm_mlp_last_error() explains.
 */
#ifndef CPLBM_LBM_WARMSTART_H
#define CPLBM_LBM_WARMSTART_H

#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_MLP_PARAMS 17923

typedef struct lbm_mlp lbm_mlp;

/* Create a network on the current device from LBM_MLP_PARAMS host floats
 * (the initial parameters are the caller's: random draws are inputs).
 * Adam's moments start at zero. */
lbm_status lbm_mlp_create(const float *params, void *hip_stream, lbm_mlp **out);

/* Copy the parameters out (host), or replace them (host; resets Adam). */
lbm_status lbm_mlp_get_params(lbm_mlp *m, float *params);
lbm_status lbm_mlp_set_params(lbm_mlp *m, const float *params);

/* y[n][3] = network(x[n][7]) on the device; bf16 != 0 takes the matrix-core
 * path.  Not synchronised. */
lbm_status lbm_mlp_forward(lbm_mlp *m, const float *x, int64_t n, float *y, int bf16);

/* Loss over samples (x[n][7], t[n][3]) and its gradient with respect to the
 * parameters (host outputs, either may be NULL). */
lbm_status lbm_mlp_loss_grad(lbm_mlp *m, const float *x, const float *t, int64_t n, float *loss,
                             float *grad);

/* iters Adam steps on minibatches of `batch` samples: step j uses samples
 * order[j*batch .. (j+1)*batch) of (x, t), which hold nsamples rows (the
 * order is the caller's, e.g. a seeded shuffle).  Hyperparameters as in
 * Adam's paper.  losses (host, iters floats, may be NULL) receives each
 * minibatch's loss before its update.  An index outside [0, nsamples)
 * makes the call fail with LBM_E_INVALID (the parameters are then
 * unspecified). */
lbm_status lbm_mlp_train(lbm_mlp *m, const float *x, const float *t, int64_t nsamples,
                         const int32_t *order, int64_t batch, int64_t iters, float lr,
                         float beta1, float beta2, float eps, float *losses);

/* Adam steps taken since creation or the last set_params. */
int64_t lbm_mlp_steps(const lbm_mlp *m);

/* Warm-start fields of a static drop (radius, centre (cx, cy) in mesh
 * nodes) for the parameters p (periodic mesh, any EOS; features use p->T_r,
 * p->kappa, p->k), from the network (bf16 != 0: matrix-core inference, else
 * FP32; within the reach of lbm_mlp_set_reach, by default everywhere): rho
 * (device, ny*nx doubles, layout of lbm.h), mass matched --
 * target_mass - sum(rho) is added in proportion to
 * max((rho - rho_g)(rho_l - rho), 0), which vanishes in both bulks, so that
 * sum(rho) = target_mass to round-off -- and the fluid velocity v (ux, uy:
 * device, ny*nx doubles each, both NULL to skip).  Start a solver from rho
 * (lbm_init or lbm_batch_create) and then give it v with lbm_set_velocity or
 * lbm_batch_set_velocity.  The network is evaluated at each node and at its
 * mirror features (sin 4 theta negated) and the fields are symmetrised --
 * density and radial velocity even, azimuthal velocity odd under the
 * square's reflections -- so that the proposal carries no net momentum and
 * keeps its centre.  LBM_E_DOMAIN when the matched density would not be
 * positive (the caller then falls back to the tanh start).  Synchronises. */
lbm_status lbm_warm_start_drop(lbm_mlp *m, const lbm_params *p, double cx, double cy,
                               double radius, double target_mass, int bf16, double *rho,
                               double *ux, double *uy);

/* Distance from the interface (r - R, mesh nodes) up to which the warm-start
 * fields of m use the network, for a network whose training meshes did not
 * reach as far from the drop as the meshes it is used on (extension of the
 * Sec. 5.3 drop start, Eq. 41).  With w = 1 for r - R <= reach - 10, 0 for
 * r - R >= reach + 10 and linear in r between, lbm_warm_start_drop forms
 * ln rho = ln rho_g + w y0 (ln rho_l - ln rho_g) and the velocity w v before
 * mass matching: the Maxwell gas at rest beyond reach + 10.  Default
 * +infinity (w = 1 everywhere).  LBM_E_INVALID unless reach > 0 (NaN
 * included); +infinity restores the default.  No device call. */
lbm_status lbm_mlp_set_reach(lbm_mlp *m, double reach);

void lbm_mlp_destroy(lbm_mlp *m);

/* Reason for the last failure of m, or of the last failed lbm_mlp_create
 * when m is NULL. */
const char *lbm_mlp_last_error(const lbm_mlp *m);

#ifdef __cplusplus
}
#endif

#endif /* CPLBM_LBM_WARMSTART_H */
