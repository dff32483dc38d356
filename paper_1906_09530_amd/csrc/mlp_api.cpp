// C ABI of the learned warm start (include/lbm_warmstart.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm_warmstart.h"
#include "mlp.hpp"

using namespace cplbm;

static_assert(mlp::kParams == LBM_MLP_PARAMS, "parameter count");

struct lbm_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // device, kParams each
    float *loss = nullptr;                                         // device scratch loss
    int *bad = nullptr;                                            // device index flag
    float *ws = nullptr;  // training workspace
    size_t ws_floats = 0;
    double *field = nullptr;  // warm-start partial sums and the correction
    size_t field_doubles = 0;
    float *fxy = nullptr;  // warm-start features and outputs
    size_t fxy_floats = 0;
    int64_t steps = 0;
    double reach = INFINITY;  // of the warm-start fields (lbm_mlp_set_reach)
    std::string err;
};

namespace {

thread_local std::string g_mlp_error;

lbm_status mfail(lbm_mlp *m, lbm_status s, const std::string &msg)
{
    if (m)
        m->err = msg;
    else
        g_mlp_error = msg;
    return s;
}

#define MHIP_OR(m, call)                                                                       \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return mfail((m), LBM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

lbm_status menter(lbm_mlp *m)
{
    if (!m) return LBM_E_INVALID;
    MHIP_OR(m, hipSetDevice(m->device));
    return LBM_OK;
}

lbm_status reserve_ws(lbm_mlp *m, int batch)
{
    const size_t need = mlp::train_ws_floats(batch);
    if (need <= m->ws_floats) return LBM_OK;
    MHIP_OR(m, hipStreamSynchronize(m->stream));
    if (m->ws) MHIP_OR(m, hipFree(m->ws));
    m->ws = nullptr;
    m->ws_floats = 0;
    MHIP_OR(m, hipMalloc(&m->ws, need * sizeof(float)));
    m->ws_floats = need;
    return LBM_OK;
}

lbm_status reset_adam(lbm_mlp *m)
{
    MHIP_OR(m, hipMemsetAsync(m->m, 0, sizeof(float) * mlp::kParams, m->stream));
    MHIP_OR(m, hipMemsetAsync(m->v, 0, sizeof(float) * mlp::kParams, m->stream));
    m->steps = 0;
    return LBM_OK;
}

// the device index flag: clear before, read after
lbm_status check_bad(lbm_mlp *m)
{
    int bad = 0;
    MHIP_OR(m, hipMemcpyAsync(&bad, m->bad, sizeof(int), hipMemcpyDeviceToHost, m->stream));
    MHIP_OR(m, hipStreamSynchronize(m->stream));
    if (bad) return mfail(m, LBM_E_INVALID, "a sample index lies outside the sample set");
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_mlp_create(const float *params, void *hip_stream, lbm_mlp **out)
{
    if (!out) return mfail(nullptr, LBM_E_INVALID, "out is NULL");
    *out = nullptr;
    g_mlp_error.clear();
    if (!params) return mfail(nullptr, LBM_E_INVALID, "params is NULL");
    for (int i = 0; i < mlp::kParams; ++i)
        if (!std::isfinite(params[i]))
            return mfail(nullptr, LBM_E_INVALID, "parameters must be finite");
    lbm_mlp *m = new (std::nothrow) lbm_mlp();
    if (!m) return mfail(nullptr, LBM_E_NOMEM, "host allocation failed");
    auto give_up = [&](lbm_status st, const std::string &msg) {
        lbm_mlp_destroy(m);
        return mfail(nullptr, st, msg);
    };
    if (hipGetDevice(&m->device) != hipSuccess) return give_up(LBM_E_DEVICE, "no HIP device");
    m->stream = (hipStream_t)hip_stream;
    float **bufs[] = {&m->w, &m->g, &m->m, &m->v};
    for (float **b : bufs)
        if (hipMalloc(b, sizeof(float) * mlp::kParams) != hipSuccess)
            return give_up(LBM_E_NOMEM, "hipMalloc failed");
    if (hipMalloc(&m->loss, sizeof(float)) != hipSuccess ||
        hipMalloc(&m->bad, sizeof(int)) != hipSuccess)
        return give_up(LBM_E_NOMEM, "hipMalloc failed");
    if (lbm_mlp_set_params(m, params) != LBM_OK) return give_up(LBM_E_DEVICE, m->err);
    *out = m;
    return LBM_OK;
}

lbm_status lbm_mlp_get_params(lbm_mlp *m, float *params)
{
    lbm_status st = menter(m);
    if (st != LBM_OK) return st;
    if (!params) return mfail(m, LBM_E_INVALID, "params is NULL");
    MHIP_OR(m, hipMemcpyAsync(params, m->w, sizeof(float) * mlp::kParams, hipMemcpyDeviceToHost,
                              m->stream));
    MHIP_OR(m, hipStreamSynchronize(m->stream));
    return LBM_OK;
}

lbm_status lbm_mlp_set_params(lbm_mlp *m, const float *params)
{
    lbm_status st = menter(m);
    if (st != LBM_OK) return st;
    if (!params) return mfail(m, LBM_E_INVALID, "params is NULL");
    MHIP_OR(m, hipMemcpyAsync(m->w, params, sizeof(float) * mlp::kParams, hipMemcpyHostToDevice,
                              m->stream));
    if ((st = reset_adam(m)) != LBM_OK) return st;
    MHIP_OR(m, hipStreamSynchronize(m->stream));
    return LBM_OK;
}

lbm_status lbm_mlp_forward(lbm_mlp *m, const float *x, int64_t n, float *y, int bf16)
{
    lbm_status st = menter(m);
    if (st != LBM_OK) return st;
    if (n < 0 || n > INT32_MAX / 8 || (n > 0 && (!x || !y)))
        return mfail(m, LBM_E_INVALID, "bad sample count or NULL buffer");
    MHIP_OR(m, bf16 ? mlp::forward_bf16(m->w, x, (int)n, y, m->stream)
                    : mlp::forward_f32(m->w, x, (int)n, y, m->bad, m->stream));
    return LBM_OK;
}

lbm_status lbm_mlp_loss_grad(lbm_mlp *m, const float *x, const float *t, int64_t n, float *loss,
                             float *grad)
{
    lbm_status st = menter(m);
    if (st != LBM_OK) return st;
    if (n <= 0 || n > (1 << 24) || !x || !t)
        return mfail(m, LBM_E_INVALID, "need 1 <= n <= 2^24 samples and device x, t");
    if ((st = reserve_ws(m, (int)n)) != LBM_OK) return st;
    MHIP_OR(m, hipMemsetAsync(m->bad, 0, sizeof(int), m->stream));
    MHIP_OR(m, mlp::train_step(m->w, m->g, nullptr, nullptr, x, t, (int)n, nullptr, (int)n, 0.f,
                               0.f, 0.f, 0.f, 0.f, 0.f, m->ws, m->bad, m->loss, m->stream));
    if (loss)
        MHIP_OR(m, hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
    if (grad)
        MHIP_OR(m, hipMemcpyAsync(grad, m->g, sizeof(float) * mlp::kParams, hipMemcpyDeviceToHost,
                                  m->stream));
    return check_bad(m);
}

lbm_status lbm_mlp_train(lbm_mlp *m, const float *x, const float *t, int64_t nsamples,
                         const int32_t *order, int64_t batch, int64_t iters, float lr,
                         float beta1, float beta2, float eps, float *losses)
{
    lbm_status st = menter(m);
    if (st != LBM_OK) return st;
    if (nsamples <= 0 || nsamples > INT32_MAX || batch <= 0 || batch > (1 << 20) || iters < 0 ||
        !x || !t || !order)
        return mfail(m, LBM_E_INVALID, "bad sizes or NULL buffer");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return mfail(m, LBM_E_INVALID, "need lr > 0, 0 <= beta < 1, eps > 0");
    if ((st = reserve_ws(m, (int)batch)) != LBM_OK) return st;
    float *dloss = nullptr;
    if (losses && iters > 0) MHIP_OR(m, hipMalloc(&dloss, sizeof(float) * iters));
    MHIP_OR(m, hipMemsetAsync(m->bad, 0, sizeof(int), m->stream));
    hipError_t e = hipSuccess;
    for (int64_t it = 0; it < iters && e == hipSuccess; ++it) {
        const int64_t step = m->steps + 1;
        const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
        const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
        e = mlp::train_step(m->w, m->g, m->m, m->v, x, t, (int)nsamples, order + it * batch,
                            (int)batch, lr, beta1, beta2, eps, c1, c2, m->ws, m->bad,
                            dloss ? dloss + it : nullptr, m->stream);
        if (e == hipSuccess) m->steps = step;
    }
    if (e == hipSuccess && dloss)
        e = hipMemcpyAsync(losses, dloss, sizeof(float) * iters, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (dloss) (void)hipFree(dloss);
    if (e != hipSuccess)
        return mfail(m, LBM_E_DEVICE, std::string("training: ") + hipGetErrorString(e));
    return check_bad(m);
}

int64_t lbm_mlp_steps(const lbm_mlp *m) { return m ? m->steps : -1; }

lbm_status lbm_mlp_set_reach(lbm_mlp *m, double reach)
{
    if (!m) return LBM_E_INVALID;
    if (!(reach > 0)) return mfail(m, LBM_E_INVALID, "reach must be > 0 (or +infinity)");
    m->reach = reach;
    return LBM_OK;
}

lbm_status lbm_warm_start_drop(lbm_mlp *m, const lbm_params *p, double cx, double cy,
                               double radius, double target_mass, int bf16, double *rho,
                               double *ux, double *uy)
{
    lbm_status st = menter(m);
    if (st != LBM_OK) return st;
    if (!p || !rho) return mfail(m, LBM_E_INVALID, "params or rho is NULL");
    if ((ux == nullptr) != (uy == nullptr))
        return mfail(m, LBM_E_INVALID, "ux and uy must both be given or both be NULL");
    if (p->nx < 1 || p->ny < 1 || (int64_t)p->nx * p->ny > (1 << 25))
        return mfail(m, LBM_E_INVALID, "bad mesh size");
    if (!(std::isfinite(cx) && std::isfinite(cy) && radius > 0 && std::isfinite(radius) &&
          target_mass > 0 && std::isfinite(target_mass)))
        return mfail(m, LBM_E_INVALID, "need a finite centre, radius > 0 and target mass > 0");
    double g = 0, l = 0;
    st = lbm_maxwell(p, &g, &l);
    if (st != LBM_OK) return mfail(m, st, "no coexistence densities at this temperature");
    mlp::WsDrop d{};
    d.nx = p->nx;
    d.ny = p->ny;
    d.cx = cx;
    d.cy = cy;
    d.radius = radius;
    d.T_r = p->T_r;
    d.kappa = p->kappa;
    d.k = p->k;
    d.rho_g = g;
    d.rho_l = l;
    d.ln_rho_g = std::log(g);
    d.ln_rho_l = std::log(l);
    d.radius_ref = 256.0;
    d.u_scale = 1e-3;
    d.reach = m->reach;
    const double center[mlp::kInputs] = {0.5, 0.25, 0.1, 0.25, 0.0, 0.0, 0.0};
    const double scale[mlp::kInputs] = {0.25, 0.1, 0.1, 0.1, 8.0, 1.0, 1.0};
    for (int i = 0; i < mlp::kInputs; ++i) {
        d.center[i] = center[i];
        d.scale[i] = scale[i];
    }
    const size_t N = (size_t)d.nx * d.ny;
    const size_t need = 2 * (size_t)mlp::ws_field_blocks((int)N) + 1;
    const size_t need_f = 2 * N * (mlp::kInputs + mlp::kOutputs);
    if (need > m->field_doubles || need_f > m->fxy_floats) {
        MHIP_OR(m, hipStreamSynchronize(m->stream));
        if (m->field) MHIP_OR(m, hipFree(m->field));
        if (m->fxy) MHIP_OR(m, hipFree(m->fxy));
        m->field = nullptr;
        m->fxy = nullptr;
        m->field_doubles = m->fxy_floats = 0;
        MHIP_OR(m, hipMalloc(&m->field, need * sizeof(double)));
        MHIP_OR(m, hipMalloc(&m->fxy, need_f * sizeof(float)));
        m->field_doubles = need;
        m->fxy_floats = need_f;
    }
    float *x = m->fxy, *y = m->fxy + 2 * N * mlp::kInputs;
    MHIP_OR(m, hipMemsetAsync(m->bad, 0, sizeof(int), m->stream));
    MHIP_OR(m, mlp::warm_start_field(m->w, d, bf16 != 0, target_mass, x, y, rho, ux, uy,
                                     m->field + 1, m->field, m->bad, m->stream));
    int bad = 0;
    MHIP_OR(m, hipMemcpyAsync(&bad, m->bad, sizeof(int), hipMemcpyDeviceToHost, m->stream));
    MHIP_OR(m, hipStreamSynchronize(m->stream));
    if (bad)
        return mfail(m, LBM_E_DOMAIN,
                     "the proposed density is too far from the target mass to match it");
    return LBM_OK;
}

void lbm_mlp_destroy(lbm_mlp *m)
{
    if (!m) return;
    (void)hipSetDevice(m->device);
    (void)hipStreamSynchronize(m->stream);
    void *ptrs[] = {m->w, m->g, m->m, m->v, m->loss, m->bad, m->ws, m->field, m->fxy};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete m;
}

const char *lbm_mlp_last_error(const lbm_mlp *m)
{
    return m ? m->err.c_str() : g_mlp_error.c_str();
}

}  // extern "C"
