// Device side of the learned warm start (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace cplbm {
namespace mlp {

constexpr int kInputs = 7, kHidden = 128, kOutputs = 3;
constexpr int kParams = kHidden * kInputs + kHidden + kHidden * kHidden + kHidden +
                        kOutputs * kHidden + kOutputs;

// A static drop whose initial density the network proposes.
struct WsDrop {
    int nx, ny;
    double cx, cy, radius, T_r, kappa, k;
    double rho_g, rho_l, ln_rho_g, ln_rho_l;  // Maxwell pair of the drop's EOS and T
    double radius_ref;                        // feature 2 is radius / radius_ref
    double u_scale;                           // velocity outputs are in units of u_scale
    double reach;  // network within reach of the interface, Maxwell gas beyond (k_ws_map)
    double center[kInputs], scale[kInputs];   // x_i = (f_i - center_i) / scale_i
};

// Workspace floats of a training step with `batch` samples.
size_t train_ws_floats(int batch);
// One gradient evaluation on `batch` samples (rows idx[0..batch) of x, t,
// which hold nsrc rows, or the first batch rows when idx is null) into g; the
// mean squared error into *loss_dev when not null; then, when m is not null,
// one Adam update of w with the bias corrections c1 = 1/(1 - b1^step),
// c2 = 1/(1 - b2^step).  An index outside [0, nsrc) sets *bad = 1 (and
// sample 0 is used in its place).
hipError_t train_step(float *w, float *g, float *m, float *v, const float *x, const float *t,
                      int nsrc, const int32_t *idx, int batch, float lr, float b1, float b2,
                      float eps, float c1, float c2, float *ws, int *bad, float *loss_dev,
                      hipStream_t s);
// y[n][3] of x[n][7]: FP32 throughout, or the hidden product in BF16 (matrix cores).
hipError_t forward_f32(const float *w, const float *x, int n, float *y, int *bad, hipStream_t s);
hipError_t forward_bf16(const float *w, const float *x, int n, float *y, hipStream_t s);
// Warm-start fields of drop d: features of every node and of its mirror
// image into x (2*nx*ny*7 floats), network outputs into y (2*nx*ny*3 floats;
// BF16 matrix-core or FP32 inference), then rho (FP64, ny*nx) mass matched
// to target_mass and the fluid velocity (ux, uy, both null or both not),
// symmetric under the square's reflections.  part holds
// 2 * ws_field_blocks(nx*ny) doubles; c receives the mass-matching
// coefficient; *bad is set when a matched density is not positive and
// finite.
int ws_field_blocks(int nodes);
hipError_t warm_start_field(const float *w, const WsDrop &d, bool bf16, double target_mass,
                            float *x, float *y, double *rho, double *ux, double *uy,
                            double *part, double *c, int *bad, hipStream_t s);

}  // namespace mlp
}  // namespace cplbm
