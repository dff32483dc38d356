// C ABI of the solver (include/lbm.h): context, memory, validation, the
// time-step sequence and the convergence loop.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "kernels.hpp"
#include "setup.hpp"
#include "thermo.hpp"

using namespace cplbm;

struct lbm_ctx {
    lbm_params prm{};
    KParams kp{};
    hipStream_t stream = nullptr;
    int device = 0;
    bool owns_mem = false;
    void *mem = nullptr;
    size_t N = 0;
    double *f[2] = {nullptr, nullptr};
    double *g[2] = {nullptr, nullptr};  // density groups of f[0], f[1]
    int cur = 0;  // f[cur], g[cur] hold the current state
    double *rho = nullptr, *mux = nullptr, *mu = nullptr, *fy = nullptr;
    double *prev = nullptr, *obs = nullptr, *partial = nullptr, *red = nullptr;
    int red_blocks = 1;
    int64_t steps = 0;
    lbm_status sticky = LBM_OK;
    std::string err;
    // runs of graph_steps steps (even; 0: none) replay a captured graph, one
    // per starting buffer, captured on the context's own capture stream
    int64_t graph_steps = 0;
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    size_t lds_max = 0;  // LDS one workgroup may use on the device (bytes)
};

namespace {

thread_local std::string g_init_error;

constexpr int kMaxLine = kMaxBlockElems;  // longest line a block holds in LDS
// longer lines: rows over windowed segments (a whole number of 4-node
// chunks), columns on the factorised solve with 8- or 16-node chunks
constexpr int kMaxRow = 1 << 20;
constexpr int kMaxCol = 1 << 20;
constexpr int kDefaultStripWidth = 4;     // columns per block before tuning
constexpr int kDefaultChunk = 4;          // column nodes per thread before tuning
constexpr size_t kGraphDefaultMaxNodes = 512 * 512;  // graph-replayed runs by default
constexpr int64_t kGraphDefaultSteps = 100;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct Layout {
    size_t f, g, field, partial, red, total;
};

Layout layout_for(const lbm_params *p, int red_blocks)
{
    Layout L;
    const size_t N = (size_t)p->nx * p->ny;
    L.f = align256(9 * N * sizeof(double));
    L.g = align256(3 * N * sizeof(double));
    L.field = align256(N * sizeof(double));
    L.partial = align256(2 * (size_t)red_blocks * sizeof(double));
    L.red = align256(2 * sizeof(double));
    // f A/B, g A/B, rho, mux, mu, fy, prev, 3 observation planes, partials,
    // result
    L.total = 2 * L.f + 2 * L.g + 8 * L.field + L.partial + L.red;
    return L;
}

lbm_status fail(lbm_ctx *c, lbm_status s, const std::string &msg)
{
    if (c)
        c->err = msg;
    else
        g_init_error = msg;
    return s;
}

#define HIP_OR(c, call)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((c), LBM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool finite(double v) { return std::isfinite(v); }

lbm_status validate(const lbm_params *p, std::string *why)
{
    auto bad = [&](const char *m) {
        *why = m;
        return LBM_E_INVALID;
    };
    if (!p) return bad("params is NULL");
    if (p->nx < 8 || p->ny < 8 || p->nx > kMaxRow || p->ny > kMaxCol)
        return bad("nx and ny must lie in [8, 1048576]");
    if (p->nx > kMaxLine && p->nx % kIirRowChunk != 0)
        return bad("rows longer than 4096 nodes must be a multiple of 4");
    if (p->ny > kMaxLine && p->ny % 8 != 0)
        return bad("columns longer than 4096 nodes must be a multiple of 8");
    if (p->bc_y != 0 && p->bc_y != 1) return bad("bc_y must be 0 or 1");
    if (p->eos < LBM_EOS_VDW || p->eos > LBM_EOS_CS) return bad("unknown EOS");
    if (!(finite(p->a) && p->a > 0 && finite(p->b) && p->b > 0 && finite(p->R) && p->R > 0))
        return bad("a, b, R must be positive and finite");
    if (!finite(p->omega)) return bad("omega must be finite");
    if (!(finite(p->T_r) && p->T_r > 0)) return bad("T_r must be positive");
    if (!(finite(p->kappa) && p->kappa >= 0)) return bad("kappa must be >= 0");
    if (!(finite(p->tau) && p->tau > 0.5)) return bad("tau must exceed 1/2");
    if (!(finite(p->k) && p->k > 0)) return bad("k must be positive");
    if (std::isnan(p->mu_cap)) return bad("mu_cap is NaN");
    if (!finite(p->wall_ux)) return bad("wall_ux must be finite");
    if (std::fabs(p->cfd_alpha - 1.0 / 3.0) > 1e-15 && std::fabs(p->cfd_alpha - 0.25) > 1e-15)
        return bad("cfd_alpha must be 1/3 or 1/4");
    if (p->collision != LBM_COLLISION_BGK && p->collision != LBM_COLLISION_MRT)
        return bad("collision must be LBM_COLLISION_BGK or LBM_COLLISION_MRT");
    if (p->force != LBM_FORCE_CP && p->force != LBM_FORCE_SC)
        return bad("force must be LBM_FORCE_CP or LBM_FORCE_SC");
    if (p->wetting != 0 && p->wetting != 1) return bad("wetting must be 0 or 1");
    if (p->wetting && !p->bc_y) return bad("wetting walls need bc_y = 1");
    if (p->wetting && p->force != LBM_FORCE_CP)
        return bad("wetting walls act on the chemical potential (LBM_FORCE_CP)");
    if (p->wetting && !finite(p->mu_wall)) return bad("mu_wall must be finite");
    if (p->collision == LBM_COLLISION_MRT) {
        for (double r : {p->s_e, p->s_eps, p->s_q})
            if (!(finite(r) && r > 0 && r < 2)) return bad("MRT rates must lie in (0, 2)");
    }
    return LBM_OK;
}

Eos eos_of(const lbm_params *p)
{
    return Eos{p->eos, (long double)p->a, (long double)p->b, (long double)p->R,
               (long double)p->omega};
}

// Device parameter block: temperature, alpha(T), compact-scheme and
// reduction-stage coefficients, block shapes.
bool make_kparams(const lbm_params *p, KParams *kp, std::string *why)
{
    Eos e = eos_of(p);
    long double Tc, rc, pc;
    if (!eos_critical(e, &Tc, &rc, &pc)) {
        *why = "critical point not found";
        return false;
    }
    const long double T = (long double)p->T_r * Tc;
    KParams k{};
    k.nx = p->nx;
    k.ny = p->ny;
    k.bc_y = p->bc_y;
    k.eos = p->eos;
    k.kappa_zero = p->kappa == 0.0;
    k.a = p->a;
    k.b = p->b;
    k.RT = (double)((long double)p->R * T);
    const long double A = (long double)p->a * eos_alpha(e, T, Tc);
    k.A = (double)A;
    if (p->eos == LBM_EOS_PR)
        k.eos_c1 = (double)(A / (2.0L * sqrtl(2.0L) * (long double)p->b));
    else
        k.eos_c1 = (double)(A / (long double)p->b);
    k.k2 = p->k * p->k;
    k.kappa = p->kappa;
    k.inv_tau = 1.0 / p->tau;
    k.mu_cap = p->mu_cap;
    k.wall_ux = p->wall_ux;
    k.sc = p->force == LBM_FORCE_SC;
    k.wet = p->bc_y && p->wetting;
    k.mu_wall = k.wet ? p->k * p->k * p->mu_wall : 0.0;
    k.mrt = p->collision == LBM_COLLISION_MRT;
    // MRT: s_k / |M_k|^2 of (e, eps, q_x, q_y, p_xx, p_xy), |M_k|^2 = 36, 36,
    // 12, 12, 4, 4 for the orthogonal moment basis of Eq. 4
    const double rates[6] = {p->s_e, p->s_eps, p->s_q, p->s_q, 1.0 / p->tau, 1.0 / p->tau};
    const double norms[6] = {36.0, 36.0, 12.0, 12.0, 4.0, 4.0};
    for (int i = 0; i < 6; ++i) k.mrt_w[i] = k.mrt ? rates[i] / norms[i] : 0.0;
    const long double al = std::fabs(p->cfd_alpha - 0.25) < 1e-15 ? 0.25L : 1.0L / 3.0L;
    k.cfd_a2 = (double)(2.0L * (al + 2.0L) / 3.0L / 2.0L);  // a/2, Eq. 38
    k.cfd_b4 = (double)((4.0L * al - 1.0L) / 3.0L / 4.0L);  // b/4, Eq. 38
    long double c = al;
    int s = 0;
    while (s < kMaxStages) {
        long double g = 1.0L / (1.0L - 2.0L * c * c);
        k.pcr_c[s] = (double)c;
        k.pcr_g[s] = (double)g;
        ++s;
        c = -c * c * g;
        if (std::fabs((double)c) < 1e-18) break;
    }
    k.nstage = s;
    if (s > 6) {  // the compare-only index folding assumes offsets <= 32
        *why = "too many reduction stages";
        return false;
    }
    // factorised inverse: q is the root of al q^2 + q + al = 0 with |q| < 1
    const long double q = (-1.0L + sqrtl(1.0L - 4.0L * al * al)) / (2.0L * al);
    k.iir_q = (double)q;
    k.iir_inv_q = (double)(1.0L / q);
    k.iir_K = (double)(1.0L / (1.0L + 2.0L * al * q));
    long double qp = 1.0L;
    for (int i = 0; i < 17; ++i) {
        k.iir_qp[i] = (double)qp;
        qp *= q;
    }
    set_row_shape(&k);
    k.row_keep = 1;
    // planes f[9][ny][nx] (the layout of lbm_get_state); a context switches
    // to rows interleaved
    set_state_layout(&k, false);
    set_col_shape(&k, kDefaultStripWidth, kDefaultChunk);
    // wide meshes with long columns: 16-column strips streamed down the
    // columns (at 4096 x 2048 and 16384 x 8192 they take half the time of
    // whole-column strips or tiles; the autotuner decides elsewhere)
    if (k.nx >= 4096 && k.ny >= 2048 && set_col_stream(&k, 16)) {
        *kp = k;
        return true;
    }
    // columns longer than one workgroup's reduction holds: tiles with
    // windows, 4 columns wide
    if (k.ny > kMaxLine && !set_col_tiles(&k, kDefaultStripWidth, 8)) {
        *why = "no column solve holds columns of this length";
        return false;
    }
    *kp = k;
    return true;
}

lbm_status check_density(const lbm_params *p, const double *rho, const double *ux,
                         const double *uy, size_t N, std::string *why)
{
    // the pseudopotential model has no upper limit of mu to fall back on
    const bool cap_off = (std::isinf(p->mu_cap) && p->mu_cap > 0) || p->force == LBM_FORCE_SC;
    for (size_t n = 0; n < N; ++n) {
        const double r = rho[n];
        if (!(finite(r) && r > 0)) {
            *why = "initial density must be positive and finite";
            return LBM_E_DOMAIN;
        }
        if (cap_off) {
            const bool outside = p->eos == LBM_EOS_CS ? p->b * r * 0.25 >= 1.0 : p->b * r >= 1.0;
            if (outside) {
                *why = "initial density outside the EOS domain and no upper limit of mu";
                return LBM_E_DOMAIN;
            }
        }
        if ((ux && !finite(ux[n])) || (uy && !finite(uy[n]))) {
            *why = "initial velocity must be finite";
            return LBM_E_DOMAIN;
        }
    }
    return LBM_OK;
}

void carve(lbm_ctx *c, int red_blocks)
{
    Layout L = layout_for(&c->prm, red_blocks);
    char *m = (char *)c->mem;
    c->f[0] = (double *)m;
    m += L.f;
    c->f[1] = (double *)m;
    m += L.f;
    c->g[0] = (double *)m;
    m += L.g;
    c->g[1] = (double *)m;
    m += L.g;
    double **fields[] = {&c->rho, &c->mux, &c->mu, &c->fy, &c->prev};
    for (double **q : fields) {
        *q = (double *)m;
        m += L.field;
    }
    c->obs = (double *)m;
    m += 3 * L.field;
    c->partial = (double *)m;
    m += L.partial;
    c->red = (double *)m;
}

// One step = pass A, pass B, pass C.
lbm_status enqueue_steps_on(lbm_ctx *c, int64_t n, hipStream_t st)
{
    for (int64_t s = 0; s < n; ++s) {
        const double *fc = c->f[c->cur];
        double *fn = c->f[1 - c->cur];
        HIP_OR(c, launch_rows_rho(c->kp, fc, c->g[c->cur], c->rho, c->mux, st));
        HIP_OR(c, launch_cols_mu(c->kp, c->rho, c->mux, c->mu, c->fy, st));
        HIP_OR(c, launch_rows_collide(c->kp, fc, c->mu, c->fy, fn, c->g[1 - c->cur], c->rho, st));
        c->cur = 1 - c->cur;
        c->steps += 1;
    }
    return LBM_OK;
}

// Graphs hold the pass shapes they were captured with: drop them whenever
// those change.
void drop_graphs(lbm_ctx *c)
{
    for (hipGraphExec_t &g : c->gexec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

// graph_steps steps from the current buffer as one graph launch on the
// context's stream (an even count, so the state returns to the same buffer).
lbm_status enqueue_graph(lbm_ctx *c)
{
    hipGraphExec_t &ex = c->gexec[c->cur];
    if (!ex) {
        if (!c->cap) HIP_OR(c, hipStreamCreate(&c->cap));
        const int cur0 = c->cur;
        const int64_t steps0 = c->steps;
        hipGraph_t g = nullptr;
        HIP_OR(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
        const lbm_status st = enqueue_steps_on(c, c->graph_steps, c->cap);
        const hipError_t e = hipStreamEndCapture(c->cap, &g);
        c->cur = cur0;
        c->steps = steps0;
        if (st != LBM_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return st != LBM_OK ? st
                                : fail(c, LBM_E_DEVICE, std::string("graph capture failed: ") +
                                                            hipGetErrorString(e));
        }
        const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) {
            ex = nullptr;
            return fail(c, LBM_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
        }
    }
    HIP_OR(c, hipGraphLaunch(ex, c->stream));
    c->steps += c->graph_steps;
    return LBM_OK;
}

lbm_status enqueue_steps(lbm_ctx *c, int64_t n)
{
    const int64_t G = c->graph_steps;
    if (G > 0) {
        for (; n >= G; n -= G) {
            const lbm_status st = enqueue_graph(c);
            if (st != LBM_OK) return st;
        }
    }
    return enqueue_steps_on(c, n, c->stream);
}

// rho, mu and F_y of the current state into the context's field buffers.
lbm_status enqueue_fields(lbm_ctx *c)
{
    const double *fc = c->f[c->cur];
    HIP_OR(c, launch_rows_rho(c->kp, fc, c->g[c->cur], c->rho, c->mux, c->stream));
    HIP_OR(c, launch_cols_mu(c->kp, c->rho, c->mux, c->mu, c->fy, c->stream));
    return LBM_OK;
}

lbm_status copy_out(lbm_ctx *c, double *dst, const double *src, size_t n, int on_device)
{
    if (!dst) return LBM_OK;
    HIP_OR(c, hipMemcpyAsync(dst, src, n * sizeof(double),
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             c->stream));
    return LBM_OK;
}

// Copy a state between planes f[9][ny][nx] (the layout of lbm_get_state) and
// the context's layout (to_planes: from the context into planes).
lbm_status copy_state(lbm_ctx *c, double *dst, const double *src, bool to_planes,
                      hipMemcpyKind kind)
{
    const size_t nx = c->kp.nx, ny = c->kp.ny, N = nx * ny, row = nx * sizeof(double);
    if (c->kp.fq == N) {
        HIP_OR(c, hipMemcpyAsync(dst, src, 9 * N * sizeof(double), kind, c->stream));
        return LBM_OK;
    }
    const size_t pitch = c->kp.fr * sizeof(double);
    for (int q = 0; q < 9; ++q) {
        if (to_planes)
            HIP_OR(c, hipMemcpy2DAsync(dst + q * N, row, src + q * c->kp.fq, pitch, row, ny, kind,
                                       c->stream));
        else
            HIP_OR(c, hipMemcpy2DAsync(dst + q * c->kp.fq, pitch, src + q * N, row, row, ny, kind,
                                       c->stream));
    }
    return LBM_OK;
}

// Collision pass variant (fast rows only): 0 one pass reading f twice,
// 1 one pass holding f in registers (rows of up to 1024 nodes), 2 one pass
// over row segments holding f in registers, F_x from a window around each
// segment (rows longer than one segment; the only variant for rows longer
// than one workgroup holds).
bool collision_variant(KParams *kp, int variant)
{
    const bool rows256 = kp->rows_per_block * (kp->nx / kIirRowChunk) <= 256;
    if (kp->row_win && variant != 2) return false;
    switch (variant) {
    case 0: kp->row_keep = 0; kp->row_split = 0; return true;
    case 1:
        if (!kp->use_iir_rows || !rows256) return false;
        kp->row_keep = 1;
        kp->row_split = 0;
        return true;
    case 2:
        if (!iir_split_ok(*kp)) return false;
        kp->row_keep = 1;
        kp->row_split = 1;
        return true;
    default: return false;
    }
}

lbm_status enter(lbm_ctx *c)
{
    if (!c) return LBM_E_INVALID;
    if (c->sticky != LBM_OK) return c->sticky;
    HIP_OR(c, hipSetDevice(c->device));
    return LBM_OK;
}

}  // namespace

namespace cplbm {

lbm_status setup_params(const lbm_params *p, KParams *kp, std::string *why)
{
    lbm_status st = validate(p, why);
    if (st != LBM_OK) return st;
    if (!make_kparams(p, kp, why)) return LBM_E_INVALID;
    return LBM_OK;
}

void set_global_error(const std::string &msg) { g_init_error = msg; }

}  // namespace cplbm

extern "C" {

lbm_status lbm_critical_point(const lbm_params *p, double *T_c, double *rho_c, double *p_c)
{
    if (!p || p->eos < LBM_EOS_VDW || p->eos > LBM_EOS_CS || !(p->a > 0 && p->b > 0 && p->R > 0))
        return fail(nullptr, LBM_E_INVALID, "invalid EOS parameters");
    long double Tc, rc, pc;
    if (!eos_critical(eos_of(p), &Tc, &rc, &pc))
        return fail(nullptr, LBM_E_INVALID, "critical point not found");
    if (T_c) *T_c = (double)Tc;
    if (rho_c) *rho_c = (double)rc;
    if (p_c) *p_c = (double)pc;
    return LBM_OK;
}

lbm_status lbm_maxwell(const lbm_params *p, double *rho_g, double *rho_l)
{
    if (!p || p->eos < LBM_EOS_VDW || p->eos > LBM_EOS_CS || !(p->a > 0 && p->b > 0 && p->R > 0))
        return fail(nullptr, LBM_E_INVALID, "invalid EOS parameters");
    if (!(p->T_r > 0 && p->T_r < 1)) return fail(nullptr, LBM_E_INVALID, "T_r must lie in (0, 1)");
    long double g, l;
    if (!eos_maxwell(eos_of(p), (long double)p->T_r, &g, &l))
        return fail(nullptr, LBM_E_INVALID, "Maxwell construction failed");
    if (rho_g) *rho_g = (double)g;
    if (rho_l) *rho_l = (double)l;
    return LBM_OK;
}

lbm_status lbm_eos_values(const lbm_params *p, double rho, double *p0, double *mu0)
{
    if (!p || p->eos < LBM_EOS_VDW || p->eos > LBM_EOS_CS || !(p->a > 0 && p->b > 0 && p->R > 0))
        return fail(nullptr, LBM_E_INVALID, "invalid EOS parameters");
    if (!(p->T_r > 0)) return fail(nullptr, LBM_E_INVALID, "T_r must be positive");
    const Eos e = eos_of(p);
    long double Tc, rc, pc;
    if (!eos_critical(e, &Tc, &rc, &pc)) return fail(nullptr, LBM_E_INVALID, "critical point not found");
    const long double T = (long double)p->T_r * Tc;
    const long double A = (long double)p->a * eos_alpha(e, T, Tc);
    const long double r = rho;
    if (!(r > 0 && r < eos_rho_max(e))) return fail(nullptr, LBM_E_DOMAIN, "rho outside the EOS domain");
    if (p0) *p0 = (double)eos_p0(e, T, A, r);
    if (mu0) *mu0 = (double)eos_mu0(e, T, A, r);
    return LBM_OK;
}

size_t lbm_workspace_bytes(const lbm_params *p)
{
    std::string why;
    if (validate(p, &why) != LBM_OK) return 0;
    KParams kp;
    if (!make_kparams(p, &kp, &why)) return 0;
    return layout_for(p, rho_delta_blocks(kp)).total;
}

lbm_status lbm_init(const lbm_params *p, const double *rho0, const double *ux0, const double *uy0,
                    int src_on_device, void *hip_stream, void *device_ws, lbm_ctx **out)
{
    if (!out) return fail(nullptr, LBM_E_INVALID, "out is NULL");
    *out = nullptr;
    g_init_error.clear();
    std::string why;
    lbm_status st = validate(p, &why);
    if (st != LBM_OK) return fail(nullptr, st, why);
    if (!rho0) return fail(nullptr, LBM_E_INVALID, "rho0 is NULL");
    KParams kp;
    if (!make_kparams(p, &kp, &why)) return fail(nullptr, LBM_E_INVALID, why);
    const size_t N = (size_t)p->nx * p->ny;

    // validate the initial fields on the host
    std::vector<double> h_rho, h_ux, h_uy;
    const double *vr = rho0, *vx = ux0, *vy = uy0;
    if (src_on_device) {
        h_rho.resize(N);
        if (hipMemcpy(h_rho.data(), rho0, N * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(nullptr, LBM_E_DEVICE, "reading rho0 from the device failed");
        vr = h_rho.data();
        if (ux0) {
            h_ux.resize(N);
            if (hipMemcpy(h_ux.data(), ux0, N * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
                return fail(nullptr, LBM_E_DEVICE, "reading ux0 from the device failed");
            vx = h_ux.data();
        }
        if (uy0) {
            h_uy.resize(N);
            if (hipMemcpy(h_uy.data(), uy0, N * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
                return fail(nullptr, LBM_E_DEVICE, "reading uy0 from the device failed");
            vy = h_uy.data();
        }
    }
    st = check_density(p, vr, vx, vy, N, &why);
    if (st != LBM_OK) return fail(nullptr, st, why);

    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_E_NOMEM, "host allocation failed");
    c->prm = *p;
    c->kp = kp;
    // each row's nine populations side by side: every pass then reads and
    // writes one contiguous block per row instead of nine planes far apart
    set_state_layout(&c->kp, true);
    c->N = N;
    c->stream = (hipStream_t)hip_stream;
    c->red_blocks = rho_delta_blocks(kp);
    // small meshes, whose kernels take a few microseconds, replay runs of
    // steps from graphs by default
    c->graph_steps = N <= kGraphDefaultMaxNodes ? kGraphDefaultSteps : 0;
    int lds_max = 0;
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) !=
            hipSuccess) {
        delete c;
        return fail(nullptr, LBM_E_DEVICE, "no HIP device");
    }
    c->lds_max = (size_t)lds_max;
    const size_t bytes = layout_for(p, c->red_blocks).total;
    if (device_ws) {
        if (((uintptr_t)device_ws & 255) != 0) {
            delete c;
            return fail(nullptr, LBM_E_INVALID, "device_ws must be 256-byte aligned");
        }
        c->mem = device_ws;
    } else {
        if (hipMalloc(&c->mem, bytes) != hipSuccess) {
            delete c;
            return fail(nullptr, LBM_E_NOMEM, "hipMalloc of the workspace failed");
        }
        c->owns_mem = true;
    }
    carve(c, c->red_blocks);

    // initial fields to the device (the observation planes serve as staging)
    const double *d_rho = rho0, *d_ux = ux0, *d_uy = uy0;
    hipError_t e = hipSuccess;
    if (!src_on_device) {
        e = hipMemcpyAsync(c->obs, rho0, N * sizeof(double), hipMemcpyHostToDevice, c->stream);
        d_rho = c->obs;
        if (e == hipSuccess && ux0) {
            e = hipMemcpyAsync(c->obs + N, ux0, N * sizeof(double), hipMemcpyHostToDevice, c->stream);
            d_ux = c->obs + N;
        }
        if (e == hipSuccess && uy0) {
            e = hipMemcpyAsync(c->obs + 2 * N, uy0, N * sizeof(double), hipMemcpyHostToDevice,
                               c->stream);
            d_uy = c->obs + 2 * N;
        }
    }
    if (e == hipSuccess) e = launch_init_feq(c->kp, d_rho, d_ux, d_uy, c->f[0], c->stream);
    if (e == hipSuccess) e = launch_density_groups(c->kp, c->f[0], c->g[0], c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        std::string m = std::string("initialisation on the device failed: ") + hipGetErrorString(e);
        lbm_destroy(c);
        return fail(nullptr, LBM_E_DEVICE, m);
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *c, int64_t nsteps)
{
    lbm_status st = enter(c);
    if (st != LBM_OK) return st;
    if (nsteps < 0) return fail(c, LBM_E_INVALID, "nsteps must be >= 0");
    return enqueue_steps(c, nsteps);
}

lbm_status lbm_moments(lbm_ctx *c, double *rho, double *vx, double *vy, int dst_on_device)
{
    lbm_status st = enter(c);
    if (st != LBM_OK) return st;
    if ((st = enqueue_fields(c)) != LBM_OK) return st;
    const size_t N = c->N;
    HIP_OR(c, launch_rows_observe(c->kp, c->f[c->cur], c->mu, c->fy, c->rho, c->obs,
                                  c->obs + N, c->obs + 2 * N, nullptr, c->stream));
    if ((st = copy_out(c, rho, c->obs, N, dst_on_device)) != LBM_OK) return st;
    if ((st = copy_out(c, vx, c->obs + N, N, dst_on_device)) != LBM_OK) return st;
    if ((st = copy_out(c, vy, c->obs + 2 * N, N, dst_on_device)) != LBM_OK) return st;
    HIP_OR(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_force_fields(lbm_ctx *c, double *mu, double *Fx, double *Fy, int dst_on_device)
{
    lbm_status st = enter(c);
    if (st != LBM_OK) return st;
    if ((st = enqueue_fields(c)) != LBM_OK) return st;
    const size_t N = c->N;
    HIP_OR(c, launch_rows_observe(c->kp, c->f[c->cur], c->mu, c->fy, c->rho, nullptr, nullptr,
                                  nullptr, c->obs, c->stream));
    if ((st = copy_out(c, mu, c->mu, N, dst_on_device)) != LBM_OK) return st;
    if ((st = copy_out(c, Fx, c->obs, N, dst_on_device)) != LBM_OK) return st;
    if ((st = copy_out(c, Fy, c->fy, N, dst_on_device)) != LBM_OK) return st;
    HIP_OR(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_run_until_converged(lbm_ctx *c, double tol, int64_t check_every, int64_t max_steps,
                                   int64_t *steps_done, double *last_delta)
{
    lbm_status st = enter(c);
    if (st != LBM_OK) return st;
    if (check_every <= 0 || max_steps < 0 || !(tol >= 0))
        return fail(c, LBM_E_INVALID, "check_every > 0, max_steps >= 0, tol >= 0 required");
    double res[2] = {0.0, 0.0};
    HIP_OR(c, launch_rho_delta(c->kp, c->f[c->cur], c->prev, c->partial, c->red_blocks, c->red,
                               c->stream));
    int64_t done = 0;
    double delta = INFINITY;
    st = LBM_NOT_CONVERGED;
    while (done < max_steps) {
        int64_t n = check_every;
        if (done + n > max_steps) n = max_steps - done;
        lbm_status s2 = enqueue_steps(c, n);
        if (s2 != LBM_OK) return s2;
        done += n;
        HIP_OR(c, launch_rho_delta(c->kp, c->f[c->cur], c->prev, c->partial, c->red_blocks,
                                   c->red, c->stream));
        HIP_OR(c, hipMemcpyAsync(res, c->red, sizeof(res), hipMemcpyDeviceToHost, c->stream));
        HIP_OR(c, hipStreamSynchronize(c->stream));
        delta = res[0];
        if (res[1] != 0.0) {
            c->sticky = LBM_E_NONFINITE;
            c->err = "non-finite density after " + std::to_string(c->steps) + " steps";
            delta = NAN;
            st = LBM_E_NONFINITE;
            break;
        }
        if (n == check_every && delta < tol) {
            st = LBM_OK;
            break;
        }
    }
    if (steps_done) *steps_done = done;
    if (last_delta) *last_delta = delta;
    return st;
}

lbm_status lbm_get_state(lbm_ctx *c, double *f, int dst_on_device)
{
    lbm_status st = enter(c);
    if (st != LBM_OK) return st;
    if (!f) return fail(c, LBM_E_INVALID, "f is NULL");
    if ((st = copy_state(c, f, c->f[c->cur], true,
                         dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost)) !=
        LBM_OK)
        return st;
    HIP_OR(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_set_state(lbm_ctx *c, const double *f, int src_on_device)
{
    lbm_status st = enter(c);
    if (st != LBM_OK) return st;
    if (!f) return fail(c, LBM_E_INVALID, "f is NULL");
    if ((st = copy_state(c, c->f[c->cur], f, false,
                         src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice)) !=
        LBM_OK)
        return st;
    HIP_OR(c, launch_density_groups(c->kp, c->f[c->cur], c->g[c->cur], c->stream));
    HIP_OR(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_set_velocity(lbm_ctx *c, const double *vx, const double *vy, int src_on_device)
{
    lbm_status st = enter(c);
    if (st != LBM_OK) return st;
    const size_t N = c->N;
    double *fx = c->obs, *ux = c->obs + N, *uy = c->obs + 2 * N;
    const hipMemcpyKind kind = src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if ((st = enqueue_fields(c)) != LBM_OK) return st;
    HIP_OR(c, launch_rows_observe(c->kp, c->f[c->cur], c->mu, c->fy, c->rho, nullptr, nullptr,
                                  nullptr, fx, c->stream));
    if (vx)
        HIP_OR(c, hipMemcpyAsync(ux, vx, N * sizeof(double), kind, c->stream));
    else
        HIP_OR(c, hipMemsetAsync(ux, 0, N * sizeof(double), c->stream));
    if (vy)
        HIP_OR(c, hipMemcpyAsync(uy, vy, N * sizeof(double), kind, c->stream));
    else
        HIP_OR(c, hipMemsetAsync(uy, 0, N * sizeof(double), c->stream));
    HIP_OR(c, launch_bare_velocity(c->kp, c->rho, fx, c->fy, ux, uy, c->stream));
    HIP_OR(c, launch_init_feq(c->kp, c->rho, ux, uy, c->f[c->cur], c->stream));
    HIP_OR(c, launch_density_groups(c->kp, c->f[c->cur], c->g[c->cur], c->stream));
    HIP_OR(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_time_passes(lbm_ctx *c, int64_t nsteps, double *ms_per_pass)
{
    lbm_status st = enter(c);
    if (st != LBM_OK) return st;
    if (nsteps <= 0 || !ms_per_pass) return fail(c, LBM_E_INVALID, "nsteps > 0 and an output required");
    // Each pass is idempotent on the state: passes A and B rewrite the same
    // scalar planes from the same inputs and pass C writes only the spare
    // state buffers.  So each is timed over nsteps back-to-back launches
    // between two events, which keeps per-launch event overhead out of the
    // average.
    hipEvent_t e0, e1;
    HIP_OR(c, hipEventCreate(&e0));
    HIP_OR(c, hipEventCreate(&e1));
    const double *fc = c->f[c->cur], *gc = c->g[c->cur];
    double *fn = c->f[1 - c->cur], *gn = c->g[1 - c->cur];
    hipError_t err = launch_rows_rho(c->kp, fc, gc, c->rho, c->mux, c->stream);
    if (err == hipSuccess) err = launch_cols_mu(c->kp, c->rho, c->mux, c->mu, c->fy, c->stream);
    for (int q = 0; q < 3 && err == hipSuccess; ++q) {
        err = hipEventRecord(e0, c->stream);
        for (int64_t s = 0; s < nsteps && err == hipSuccess; ++s) {
            if (q == 0) err = launch_rows_rho(c->kp, fc, gc, c->rho, c->mux, c->stream);
            if (q == 1) err = launch_cols_mu(c->kp, c->rho, c->mux, c->mu, c->fy, c->stream);
            if (q == 2)
                err = launch_rows_collide(c->kp, fc, c->mu, c->fy, fn, gn, c->rho, c->stream);
        }
        if (err == hipSuccess) err = hipEventRecord(e1, c->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        ms_per_pass[q] = ms / (double)nsteps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess)
        return fail(c, LBM_E_DEVICE, std::string("pass timing failed: ") + hipGetErrorString(err));
    return LBM_OK;
}

lbm_status lbm_time_step_kernels(lbm_ctx *c, int64_t nsteps, double *ms, int *count)
{
    lbm_status st = enter(c);
    if (st != LBM_OK) return st;
    if (nsteps <= 0 || !ms || !count)
        return fail(c, LBM_E_INVALID, "nsteps > 0 and outputs required");
    const int K = 3;
    std::vector<hipEvent_t> ev((size_t)nsteps * (K + 1), nullptr);
    hipError_t err = hipSuccess;
    for (size_t i = 0; i < ev.size() && err == hipSuccess; ++i) err = hipEventCreate(&ev[i]);
    for (int64_t s = 0; s < nsteps && err == hipSuccess; ++s) {
        hipEvent_t *e = &ev[(size_t)s * (K + 1)];
        const double *fc = c->f[c->cur];
        double *fn = c->f[1 - c->cur], *gn = c->g[1 - c->cur];
        err = hipEventRecord(e[0], c->stream);
        if (err == hipSuccess) err = launch_rows_rho(c->kp, fc, c->g[c->cur], c->rho, c->mux, c->stream);
        if (err == hipSuccess) err = hipEventRecord(e[1], c->stream);
        if (err == hipSuccess) err = launch_cols_mu(c->kp, c->rho, c->mux, c->mu, c->fy, c->stream);
        if (err == hipSuccess) err = hipEventRecord(e[2], c->stream);
        if (err == hipSuccess)
            err = launch_rows_collide(c->kp, fc, c->mu, c->fy, fn, gn, c->rho, c->stream);
        if (err == hipSuccess) err = hipEventRecord(e[3], c->stream);
        c->cur = 1 - c->cur;
        c->steps += 1;
    }
    if (err == hipSuccess) err = hipEventSynchronize(ev.back());
    for (int k = 0; k < K; ++k) ms[k] = 0.0;
    for (int64_t s = 0; s < nsteps && err == hipSuccess; ++s) {
        hipEvent_t *e = &ev[(size_t)s * (K + 1)];
        for (int k = 0; k < K && err == hipSuccess; ++k) {
            float t = 0.f;
            err = hipEventElapsedTime(&t, e[k], e[k + 1]);
            ms[k] += t / (double)nsteps;
        }
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (err != hipSuccess)
        return fail(c, LBM_E_DEVICE, std::string("kernel timing failed: ") + hipGetErrorString(err));
    *count = K;
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx *c, int repeats, int *widths, int *chunks, double *ms,
                        int *count)
{
    lbm_status st = enter(c);
    if (st != LBM_OK) return st;
    if (repeats <= 0) return fail(c, LBM_E_INVALID, "repeats must be positive");
    // Every candidate is timed inside whole steps, so that each pass meets
    // the caches as a real step leaves them: `repeats` times pass A, the
    // column pass and the collision pass from the current state into the
    // spare buffers, without swapping (the state stays untouched).
    hipEvent_t e0, e1;
    HIP_OR(c, hipEventCreate(&e0));
    HIP_OR(c, hipEventCreate(&e1));
    const double *fc = c->f[c->cur], *gc = c->g[c->cur];
    double *fn = c->f[1 - c->cur], *gn = c->g[1 - c->cur];
    auto steps_ms = [&](const KParams &kp, double *avg) -> hipError_t {
        hipError_t e = hipSuccess;
        for (int r = -1; r < repeats && e == hipSuccess; ++r) {  // r = -1: warm-up
            if (r == 0) e = hipEventRecord(e0, c->stream);
            if (e == hipSuccess) e = launch_rows_rho(kp, fc, gc, c->rho, c->mux, c->stream);
            if (e == hipSuccess) e = launch_cols_mu(kp, c->rho, c->mux, c->mu, c->fy, c->stream);
            if (e == hipSuccess)
                e = launch_rows_collide(kp, fc, c->mu, c->fy, fn, gn, c->rho, c->stream);
        }
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        *avg = t / repeats;
        return e;
    };
    const int cand_w[] = {1, 2, 4, 8, 16};
    const int cand_c[] = {4, 8, 16};
    // best_c < 0: tiles with windows of chunk -best_c
    int n = 0, best_w = c->kp.cols_per_block;
    int best_c = c->kp.col_stream ? LBM_COLUMN_STREAM : (c->kp.col_win ? -c->kp.col_lc : c->kp.col_lc);
    double best = INFINITY;
    hipError_t err = hipSuccess;
    for (int cw = 0; cw < 15 && err == hipSuccess; ++cw) {
        const int w = cand_w[cw / 3], ch = cand_c[cw % 3];
        KParams kp = c->kp;
        set_col_shape(&kp, w, ch);
        if (kp.cols_per_block != w) continue;  // does not fit one block
        if (!kp.use_iir_cols && kp.ny > kMaxLine) continue;
        // the general kernel ignores the chunk length: time it once
        if (!kp.use_iir_cols && ch != cand_c[0]) continue;
        double avg = 0.0;
        if ((err = steps_ms(kp, &avg)) != hipSuccess) break;
        if (widths) widths[n] = w;
        if (chunks) chunks[n] = kp.use_iir_cols ? ch : 0;
        if (ms) ms[n] = avg;
        ++n;
        if (avg < best) {
            best = avg;
            best_w = w;
            best_c = ch;
        }
    }
    // column tiles with windows (reported with the chunk negated)
    const int tile_w[] = {4, 8, 16}, tile_c[] = {8, 16};
    for (int cw = 0; cw < 6 && err == hipSuccess; ++cw) {
        const int w = tile_w[cw / 2], ch = tile_c[cw % 2];
        KParams kp = c->kp;
        if (!set_col_tiles(&kp, w, ch)) continue;
        double avg = 0.0;
        if ((err = steps_ms(kp, &avg)) != hipSuccess) break;
        if (widths) widths[n] = w;
        if (chunks) chunks[n] = -ch;
        if (ms) ms[n] = avg;
        ++n;
        if (avg < best) {
            best = avg;
            best_w = w;
            best_c = -ch;
        }
    }
    // strips streamed down the columns (reported with chunk LBM_COLUMN_STREAM)
    const int stream_w[] = {8, 16, 32};
    for (int i = 0; i < 3 && err == hipSuccess; ++i) {
        KParams kp = c->kp;
        if (!set_col_stream(&kp, stream_w[i]) || col_stream_lds(stream_w[i], kp.col_lc) > c->lds_max)
            continue;
        double avg = 0.0;
        if ((err = steps_ms(kp, &avg)) != hipSuccess) break;
        if (widths) widths[n] = stream_w[i];
        if (chunks) chunks[n] = LBM_COLUMN_STREAM;
        if (ms) ms[n] = avg;
        ++n;
        if (avg < best) {
            best = avg;
            best_w = stream_w[i];
            best_c = LBM_COLUMN_STREAM;
        }
    }
    if (err == hipSuccess) {
        if (best_c == LBM_COLUMN_STREAM)
            (void)set_col_stream(&c->kp, best_w);
        else if (best_c < 0)
            (void)set_col_tiles(&c->kp, best_w, -best_c);
        else
            set_col_shape(&c->kp, best_w, best_c);
    }
    // collision pass: populations held in registers or read twice, in one
    // pass or split for long rows
    double best_row = INFINITY;
    int best_variant = c->kp.row_split ? 2 : c->kp.row_keep;
    for (int variant = 0; variant < 3 && err == hipSuccess; ++variant) {
        KParams kp = c->kp;
        if (!collision_variant(&kp, variant)) continue;
        double avg = 0.0;
        if ((err = steps_ms(kp, &avg)) != hipSuccess) break;
        if (widths) widths[n] = 0;
        if (chunks) chunks[n] = variant;
        if (ms) ms[n] = avg;
        ++n;
        if (avg < best_row) {
            best_row = avg;
            best_variant = variant;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess)
        return fail(c, LBM_E_DEVICE, std::string("autotune failed: ") + hipGetErrorString(err));
    (void)collision_variant(&c->kp, best_variant);
    drop_graphs(c);
    if (count) *count = n;
    return LBM_OK;
}

lbm_status lbm_set_collision_variant(lbm_ctx *c, int variant)
{
    lbm_status st = enter(c);
    if (st != LBM_OK) return st;
    KParams kp = c->kp;
    if (!collision_variant(&kp, variant))
        return fail(c, LBM_E_INVALID, "collision variant not available for this mesh");
    c->kp = kp;
    drop_graphs(c);
    return LBM_OK;
}

lbm_status lbm_set_column_shape(lbm_ctx *c, int width, int chunk)
{
    lbm_status st = enter(c);
    if (st != LBM_OK) return st;
    if (chunk == LBM_COLUMN_STREAM) {
        KParams kp = c->kp;
        if (!set_col_stream(&kp, width))
            return fail(c, LBM_E_INVALID, "streamed strips of this width do not fit this mesh");
        if (col_stream_lds(width, kp.col_lc) > c->lds_max)
            return fail(c, LBM_E_INVALID, "streamed strips need more LDS than a workgroup has");
        c->kp = kp;
        drop_graphs(c);
        return LBM_OK;
    }
    if (chunk < 0) {
        KParams kp = c->kp;
        if (!set_col_tiles(&kp, width, -chunk))
            return fail(c, LBM_E_INVALID, "these column tiles do not fit this mesh");
        c->kp = kp;
        drop_graphs(c);
        return LBM_OK;
    }
    if (chunk != 0 && chunk != 4 && chunk != 8 && chunk != 16)
        return fail(c, LBM_E_INVALID,
                    "chunk must be 0, 4, 8, 16, negated for tiles, or LBM_COLUMN_STREAM");
    KParams kp = c->kp;
    set_col_shape(&kp, width, chunk == 0 ? 4 : chunk);
    if (kp.cols_per_block != width) return fail(c, LBM_E_INVALID, "width does not fit a workgroup");
    if (!kp.use_iir_cols && kp.ny > kMaxLine)
        return fail(c, LBM_E_INVALID, "columns this long need the factorised solve");
    if (chunk == 0)
        kp.use_iir_cols = 0;
    else if (!kp.use_iir_cols)
        return fail(c, LBM_E_INVALID, "this column length cannot use the factorised solve");
    c->kp = kp;
    drop_graphs(c);
    return LBM_OK;
}

lbm_status lbm_set_graph_steps(lbm_ctx *c, int64_t steps)
{
    lbm_status st = enter(c);
    if (st != LBM_OK) return st;
    if (steps < 0 || steps > 100000) return fail(c, LBM_E_INVALID, "steps must be in [0, 100000]");
    const int64_t G = steps + (steps & 1);
    if (G != c->graph_steps) drop_graphs(c);
    c->graph_steps = G;
    return LBM_OK;
}

int64_t lbm_steps_taken(const lbm_ctx *c) { return c ? c->steps : -1; }

lbm_status lbm_synchronize(lbm_ctx *c)
{
    if (!c) return LBM_E_INVALID;
    HIP_OR(c, hipSetDevice(c->device));
    HIP_OR(c, hipStreamSynchronize(c->stream));
    return c->sticky;
}

void lbm_destroy(lbm_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->owns_mem && c->mem) (void)hipFree(c->mem);
    delete c;
}

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err.c_str() : g_init_error.c_str(); }

const char *lbm_status_string(lbm_status s)
{
    switch (s) {
    case LBM_OK: return "LBM_OK";
    case LBM_NOT_CONVERGED: return "LBM_NOT_CONVERGED";
    case LBM_E_INVALID: return "LBM_E_INVALID";
    case LBM_E_DOMAIN: return "LBM_E_DOMAIN";
    case LBM_E_NOMEM: return "LBM_E_NOMEM";
    case LBM_E_DEVICE: return "LBM_E_DEVICE";
    case LBM_E_NONFINITE: return "LBM_E_NONFINITE";
    }
    return "unknown";
}

}  // extern "C"

// ---- batches of independent simulations -----------------------------------

struct lbm_batch {
    int n = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<lbm_params> prm;
    std::vector<KParams> kp;
    std::vector<SimBuffers> sb;
    std::vector<size_t> N;
    std::vector<double *> prev, partial;
    std::vector<int> red_blocks;
    KParams *d_kp = nullptr;
    SimBuffers *d_sb = nullptr;
    WorkItem *d_rows = nullptr, *d_cols = nullptr;
    int n_rows = 0, n_cols = 0;
    double *d_res = nullptr;  // per simulation: max |drho|, non-finite flag
    void *mem = nullptr;
    std::vector<int> active;
    std::vector<int> held;  // parity of the buffer a retired simulation's state is in
    std::vector<int64_t> steps;
    std::vector<lbm_status> status;
    int parity = 0;  // every active simulation holds its state in f[parity]
    int col_elems = 4096, col_lc = 8;
    int col_wmax = 1;  // widest strip (columns) of any simulation
    size_t row_lds = 0, rho_lds = 0;  // LDS of the collision pass and of pass A
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int64_t graph_len = 0;
    std::string err;
};

namespace {

thread_local std::string g_batch_error;

lbm_status bfail(lbm_batch *b, lbm_status s, const std::string &msg)
{
    if (b)
        b->err = msg;
    else
        g_batch_error = msg;
    return s;
}

#define BHIP_OR(b, call)                                                                       \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return bfail((b), LBM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

void batch_drop_graphs(lbm_batch *b)
{
    for (auto &g : b->gexec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    b->graph_len = 0;
}

// Column shape of every simulation for the batch's (col_elems, col_lc).
bool batch_apply_col_shape(lbm_batch *b, int col_elems, int lc)
{
    std::vector<KParams> kp = b->kp;
    int wmax = 1;
    for (int s = 0; s < b->n; ++s) {
        set_col_shape(&kp[s], col_elems / kp[s].ny, lc);
        if (!kp[s].use_iir_cols || kp[s].cols_per_block * kp[s].ny > col_elems) return false;
        wmax = std::max(wmax, kp[s].cols_per_block);
    }
    b->kp = kp;
    b->col_elems = col_elems;
    b->col_lc = lc;
    b->col_wmax = wmax;
    return true;
}

// Upload the parameter blocks and the work tables of the active simulations
// (largest meshes first, so the longest workgroups start first).
lbm_status batch_upload(lbm_batch *b)
{
    BHIP_OR(b, hipStreamSynchronize(b->stream));
    BHIP_OR(b, hipMemcpy(b->d_kp, b->kp.data(), sizeof(KParams) * b->n, hipMemcpyHostToDevice));
    std::vector<int> order;
    for (int s = 0; s < b->n; ++s)
        if (b->active[s]) order.push_back(s);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->N[x] > b->N[y]; });
    std::vector<WorkItem> rows, cols;
    for (int s : order) {
        const KParams &k = b->kp[s];
        for (int y0 = 0; y0 < k.ny; y0 += k.rows_per_block) rows.push_back({s, y0});
        // Workgroups go to the 8 XCDs round-robin by index.  Where a mesh's
        // strips start at a multiple of 8 and number a multiple of 8 (64 or
        // more), XCD g gets the contiguous strips [g S/8, (g+1) S/8), so that
        // neighbouring strips, which share cache lines, share an L2.
        const int S = (k.nx + k.cols_per_block - 1) / k.cols_per_block;
        if (cols.size() % 8 == 0 && S % 8 == 0 && S >= 64) {
            const int per = S / 8;
            for (int i = 0; i < S; ++i)
                cols.push_back({s, ((i % 8) * per + i / 8) * k.cols_per_block});
        } else {
            for (int x0 = 0; x0 < k.nx; x0 += k.cols_per_block) cols.push_back({s, x0});
        }
    }
    b->n_rows = (int)rows.size();
    b->n_cols = (int)cols.size();
    if (!rows.empty())
        BHIP_OR(b, hipMemcpy(b->d_rows, rows.data(), sizeof(WorkItem) * rows.size(),
                             hipMemcpyHostToDevice));
    if (!cols.empty())
        BHIP_OR(b, hipMemcpy(b->d_cols, cols.data(), sizeof(WorkItem) * cols.size(),
                             hipMemcpyHostToDevice));
    batch_drop_graphs(b);
    return LBM_OK;
}

hipError_t batch_enqueue(lbm_batch *b, int64_t nsteps)
{
    hipError_t e = hipSuccess;
    for (int64_t s = 0; s < nsteps && e == hipSuccess; ++s) {
        e = launch_batch_rows_rho(b->d_kp, b->d_sb, b->d_rows, b->n_rows, b->parity, b->rho_lds,
                                  b->stream);
        if (e == hipSuccess)
            e = launch_batch_cols_mu(b->d_kp, b->d_sb, b->d_cols, b->n_cols, b->col_elems,
                                     b->col_lc, b->col_wmax, b->stream);
        if (e == hipSuccess)
            e = launch_batch_rows_collide(b->d_kp, b->d_sb, b->d_rows, b->n_rows, b->parity,
                                          b->row_lds, b->kp[0].mrt != 0, b->stream);
        b->parity ^= 1;
    }
    return e;
}

// Enqueue nsteps as one graph launch (captured on first use for the
// current parity and work tables).
lbm_status batch_enqueue_graph(lbm_batch *b, int64_t nsteps)
{
    if (b->graph_len != nsteps) batch_drop_graphs(b);
    hipGraphExec_t &ex = b->gexec[b->parity];
    if (!ex) {
        const int parity0 = b->parity;
        hipGraph_t g = nullptr;
        BHIP_OR(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = batch_enqueue(b, nsteps);
        hipError_t e2 = hipStreamEndCapture(b->stream, &g);
        b->parity = parity0;
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return bfail(b, LBM_E_DEVICE, std::string("graph capture failed: ") +
                                              hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess)
            return bfail(b, LBM_E_DEVICE,
                         std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        b->graph_len = nsteps;
    }
    BHIP_OR(b, hipGraphLaunch(ex, b->stream));
    if (nsteps & 1) b->parity ^= 1;
    return LBM_OK;
}

int sim_parity(const lbm_batch *b, int s) { return b->active[s] ? b->parity : b->held[s]; }

lbm_status benter(lbm_batch *b)
{
    if (!b) return LBM_E_INVALID;
    BHIP_OR(b, hipSetDevice(b->device));
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_create(int32_t nsims, const lbm_params *params, const double *const *rho0,
                            const double *const *ux0, const double *const *uy0, lbm_batch **out)
{
    if (!out) return bfail(nullptr, LBM_E_INVALID, "out is NULL");
    *out = nullptr;
    g_batch_error.clear();
    if (nsims <= 0 || !params || !rho0) return bfail(nullptr, LBM_E_INVALID, "no simulations");
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return bfail(nullptr, LBM_E_NOMEM, "host allocation failed");
    auto give_up = [&](lbm_status st, const std::string &m) {
        std::string msg = m;
        lbm_batch_destroy(b);
        return bfail(nullptr, st, msg);
    };
    b->n = nsims;
    b->prm.assign(params, params + nsims);
    b->kp.resize(nsims);
    for (int s = 0; s < nsims; ++s) {
        const lbm_params *p = &params[s];
        const std::string who = "simulation " + std::to_string(s) + ": ";
        std::string why;
        lbm_status st = validate(p, &why);
        if (st != LBM_OK) return give_up(st, who + why);
        if (p->nx < 64 || p->ny < 64 || p->nx > 1024 || p->ny > 1024 || p->nx % 8 || p->ny % 8)
            return give_up(LBM_E_INVALID, who + "batch meshes need 64 <= nx, ny <= 1024, multiples of 8");
        if (!make_kparams(p, &b->kp[s], &why)) return give_up(LBM_E_INVALID, who + why);
        // each row's populations side by side, as in a context
        set_state_layout(&b->kp[s], true);
        if (!b->kp[s].use_iir_rows) return give_up(LBM_E_INVALID, who + "row pass shape");
        if (p->collision != params[0].collision)
            return give_up(LBM_E_INVALID, who + "every simulation of a batch needs the same collision");
        if (!rho0[s]) return give_up(LBM_E_INVALID, who + "rho0 is NULL");
        st = check_density(p, rho0[s], ux0 ? ux0[s] : nullptr, uy0 ? uy0[s] : nullptr,
                           (size_t)p->nx * p->ny, &why);
        if (st != LBM_OK) return give_up(st, who + why);
    }
    if (!batch_apply_col_shape(b, 4096, 8)) return give_up(LBM_E_INVALID, "column shape");
    if (hipGetDevice(&b->device) != hipSuccess) return give_up(LBM_E_DEVICE, "no HIP device");
    if (hipStreamCreate(&b->stream) != hipSuccess) return give_up(LBM_E_DEVICE, "hipStreamCreate");

    // one allocation: per simulation f A/B, g A/B, rho, mux, mu, fy, prev,
    // partials
    size_t total = 0;
    std::vector<size_t> off(nsims);
    b->N.resize(nsims);
    b->red_blocks.resize(nsims);
    for (int s = 0; s < nsims; ++s) {
        const size_t N = (size_t)params[s].nx * params[s].ny;
        b->N[s] = N;
        b->red_blocks[s] = rho_delta_blocks(b->kp[s]);
        off[s] = total;
        total += 2 * align256(9 * N * sizeof(double)) + 2 * align256(3 * N * sizeof(double)) +
                 5 * align256(N * sizeof(double)) +
                 align256(2 * (size_t)b->red_blocks[s] * sizeof(double));
    }
    if (hipMalloc(&b->mem, total) != hipSuccess) return give_up(LBM_E_NOMEM, "hipMalloc failed");
    size_t rows_cap = 0, cols_cap = 0;
    b->sb.resize(nsims);
    b->prev.resize(nsims);
    b->partial.resize(nsims);
    for (int s = 0; s < nsims; ++s) {
        char *m = (char *)b->mem + off[s];
        const size_t N = b->N[s];
        SimBuffers &q = b->sb[s];
        q.f[0] = (double *)m;
        m += align256(9 * N * sizeof(double));
        q.f[1] = (double *)m;
        m += align256(9 * N * sizeof(double));
        for (int h = 0; h < 2; ++h) {
            q.g[h] = (double *)m;
            m += align256(3 * N * sizeof(double));
        }
        double **planes[] = {&q.rho, &q.mux, &q.mu, &q.fy, &b->prev[s]};
        for (double **pl : planes) {
            *pl = (double *)m;
            m += align256(N * sizeof(double));
        }
        b->partial[s] = (double *)m;
        rows_cap += (params[s].ny + b->kp[s].rows_per_block - 1) / b->kp[s].rows_per_block;
        cols_cap += params[s].nx;  // at most one column per workgroup
        const int R = b->kp[s].rows_per_block, nx = params[s].nx;
        b->row_lds = std::max(b->row_lds, batch_row_lds(R, nx, true));
        b->rho_lds = std::max(b->rho_lds, batch_row_lds(R, nx, false));
    }
    if (hipMalloc(&b->d_kp, sizeof(KParams) * nsims) != hipSuccess ||
        hipMalloc(&b->d_sb, sizeof(SimBuffers) * nsims) != hipSuccess ||
        hipMalloc(&b->d_rows, sizeof(WorkItem) * rows_cap) != hipSuccess ||
        hipMalloc(&b->d_cols, sizeof(WorkItem) * cols_cap) != hipSuccess ||
        hipMalloc(&b->d_res, sizeof(double) * 2 * nsims) != hipSuccess)
        return give_up(LBM_E_NOMEM, "hipMalloc failed");
    if (hipMemcpy(b->d_sb, b->sb.data(), sizeof(SimBuffers) * nsims, hipMemcpyHostToDevice) !=
        hipSuccess)
        return give_up(LBM_E_DEVICE, "upload of buffers failed");
    // initial state f = feq(rho0, u0); the fields planes stage the inputs
    for (int s = 0; s < nsims; ++s) {
        const size_t N = b->N[s];
        const SimBuffers &q = b->sb[s];
        hipError_t e = hipMemcpy(q.rho, rho0[s], N * sizeof(double), hipMemcpyHostToDevice);
        const double *dux = nullptr, *duy = nullptr;
        if (e == hipSuccess && ux0 && ux0[s]) {
            e = hipMemcpy(q.mux, ux0[s], N * sizeof(double), hipMemcpyHostToDevice);
            dux = q.mux;
        }
        if (e == hipSuccess && uy0 && uy0[s]) {
            e = hipMemcpy(q.mu, uy0[s], N * sizeof(double), hipMemcpyHostToDevice);
            duy = q.mu;
        }
        if (e == hipSuccess) e = launch_init_feq(b->kp[s], q.rho, dux, duy, q.f[0], b->stream);
        if (e == hipSuccess) e = launch_density_groups(b->kp[s], q.f[0], q.g[0], b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess)
            return give_up(LBM_E_DEVICE, std::string("initialisation: ") + hipGetErrorString(e));
    }
    b->active.assign(nsims, 1);
    b->held.assign(nsims, 0);
    b->steps.assign(nsims, 0);
    b->status.assign(nsims, LBM_NOT_CONVERGED);
    lbm_status st = batch_upload(b);
    if (st != LBM_OK) return give_up(st, b->err);
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_set_column_shape(lbm_batch *b, int col_elems, int chunk)
{
    lbm_status st = benter(b);
    if (st != LBM_OK) return st;
    if ((col_elems != 2048 && col_elems != 4096) || (chunk != 4 && chunk != 8))
        return bfail(b, LBM_E_INVALID, "col_elems must be 2048 or 4096 and chunk 4 or 8");
    if (!batch_apply_col_shape(b, col_elems, chunk))
        return bfail(b, LBM_E_INVALID, "shape does not fit every simulation");
    return batch_upload(b);
}

lbm_status lbm_batch_autotune(lbm_batch *b, int repeats, int *col_elems, int *chunks, double *ms,
                              int *count)
{
    lbm_status st = benter(b);
    if (st != LBM_OK) return st;
    if (repeats <= 0) return bfail(b, LBM_E_INVALID, "repeats must be positive");
    // the column pass writes mu and F_y only: the state is untouched
    BHIP_OR(b, launch_batch_rows_rho(b->d_kp, b->d_sb, b->d_rows, b->n_rows, b->parity,
                                     b->rho_lds, b->stream));
    hipEvent_t e0, e1;
    BHIP_OR(b, hipEventCreate(&e0));
    BHIP_OR(b, hipEventCreate(&e1));
    const int cand[4][2] = {{2048, 4}, {4096, 4}, {2048, 8}, {4096, 8}};
    int n = 0, best = -1;
    double best_ms = INFINITY;
    hipError_t err = hipSuccess;
    for (int c = 0; c < 4 && err == hipSuccess; ++c) {
        if (!batch_apply_col_shape(b, cand[c][0], cand[c][1])) continue;
        if (batch_upload(b) != LBM_OK) break;
        err = launch_batch_cols_mu(b->d_kp, b->d_sb, b->d_cols, b->n_cols, b->col_elems, b->col_lc,
                                   b->col_wmax, b->stream);
        if (err == hipSuccess) err = hipEventRecord(e0, b->stream);
        for (int r = 0; r < repeats && err == hipSuccess; ++r)
            err = launch_batch_cols_mu(b->d_kp, b->d_sb, b->d_cols, b->n_cols, b->col_elems,
                                       b->col_lc, b->col_wmax, b->stream);
        if (err == hipSuccess) err = hipEventRecord(e1, b->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float t = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        if (err != hipSuccess) break;
        if (col_elems) col_elems[n] = cand[c][0];
        if (chunks) chunks[n] = cand[c][1];
        if (ms) ms[n] = t / repeats;
        ++n;
        if (t < best_ms) {
            best_ms = t;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess)
        return bfail(b, LBM_E_DEVICE, std::string("autotune failed: ") + hipGetErrorString(err));
    if (best < 0 || !batch_apply_col_shape(b, cand[best][0], cand[best][1]))
        return bfail(b, LBM_E_INVALID, "no column shape fits");
    if (count) *count = n;
    return batch_upload(b);
}

lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps)
{
    lbm_status st = benter(b);
    if (st != LBM_OK) return st;
    if (nsteps < 0) return bfail(b, LBM_E_INVALID, "nsteps must be >= 0");
    BHIP_OR(b, batch_enqueue(b, nsteps));
    for (int s = 0; s < b->n; ++s)
        if (b->active[s]) b->steps[s] += nsteps;
    return LBM_OK;
}

lbm_status lbm_batch_run_until_converged(lbm_batch *b, double tol, int64_t check_every,
                                         int64_t max_steps, int use_graph, int64_t *steps_done,
                                         double *last_delta, int32_t *status)
{
    lbm_status st = benter(b);
    if (st != LBM_OK) return st;
    if (check_every <= 0 || max_steps < 0 || !(tol >= 0))
        return bfail(b, LBM_E_INVALID, "check_every > 0, max_steps >= 0, tol >= 0 required");
    const int n = b->n;
    std::vector<double> res(2 * n), delta(n, INFINITY);
    std::vector<int64_t> taken(n, 0);
    // rho of each active simulation against its value at the previous test;
    // record: keep the differences and retire non-finite simulations, and
    // (may_converge) those below tol
    auto check_all = [&](bool record, bool may_converge) -> lbm_status {
        for (int s = 0; s < n; ++s)
            if (b->active[s])
                BHIP_OR(b, launch_rho_delta(b->kp[s], b->sb[s].f[b->parity], b->prev[s],
                                            b->partial[s], b->red_blocks[s], b->d_res + 2 * s,
                                            b->stream));
        BHIP_OR(b, hipMemcpyAsync(res.data(), b->d_res, sizeof(double) * 2 * n,
                                  hipMemcpyDeviceToHost, b->stream));
        BHIP_OR(b, hipStreamSynchronize(b->stream));
        if (!record) return LBM_OK;
        bool changed = false;
        for (int s = 0; s < n; ++s) {
            if (!b->active[s]) continue;
            delta[s] = res[2 * s];
            if (res[2 * s + 1] != 0.0) {
                b->status[s] = LBM_E_NONFINITE;
                delta[s] = NAN;
            } else if (may_converge && delta[s] < tol) {
                b->status[s] = LBM_OK;
            } else {
                continue;
            }
            b->held[s] = b->parity;
            b->active[s] = 0;
            changed = true;
        }
        return changed ? batch_upload(b) : LBM_OK;
    };
    if ((st = check_all(false, false)) != LBM_OK) return st;
    int64_t done = 0;
    bool any = true;
    while (done < max_steps && any) {
        int64_t chunk = check_every;
        if (done + chunk > max_steps) chunk = max_steps - done;
        if (use_graph && chunk == check_every)
            st = batch_enqueue_graph(b, chunk);
        else
            st = batch_enqueue(b, chunk) == hipSuccess ? LBM_OK
                                                        : bfail(b, LBM_E_DEVICE, "launch failed");
        if (st != LBM_OK) return st;
        for (int s = 0; s < n; ++s)
            if (b->active[s]) {
                b->steps[s] += chunk;
                taken[s] += chunk;
            }
        done += chunk;
        // a shorter last chunk is not a whole test interval: it cannot converge
        if ((st = check_all(true, chunk == check_every)) != LBM_OK) return st;
        any = false;
        for (int s = 0; s < n; ++s) any = any || b->active[s];
    }
    bool all_ok = true, bad = false;
    for (int s = 0; s < n; ++s) {
        if (steps_done) steps_done[s] = taken[s];
        if (last_delta) last_delta[s] = delta[s];
        if (status) status[s] = b->status[s];
        all_ok = all_ok && b->status[s] == LBM_OK;
        bad = bad || b->status[s] == LBM_E_NONFINITE;
    }
    return bad ? LBM_E_NONFINITE : (all_ok ? LBM_OK : LBM_NOT_CONVERGED);
}

lbm_status lbm_batch_moments(lbm_batch *b, int32_t sim, double *rho, double *vx, double *vy)
{
    lbm_status st = benter(b);
    if (st != LBM_OK) return st;
    if (sim < 0 || sim >= b->n) return bfail(b, LBM_E_INVALID, "no such simulation");
    const KParams &k = b->kp[sim];
    const SimBuffers &q = b->sb[sim];
    const size_t N = b->N[sim];
    double *obs = nullptr;
    BHIP_OR(b, hipMalloc(&obs, 3 * N * sizeof(double)));
    const double *fc = q.f[sim_parity(b, sim)], *gc = q.g[sim_parity(b, sim)];
    hipError_t e = launch_rows_rho(k, fc, gc, q.rho, q.mux, b->stream);
    if (e == hipSuccess) e = launch_cols_mu(k, q.rho, q.mux, q.mu, q.fy, b->stream);
    if (e == hipSuccess)
        e = launch_rows_observe(k, fc, q.mu, q.fy, q.rho, obs, obs + N, obs + 2 * N, nullptr,
                                b->stream);
    double *outs[3] = {rho, vx, vy};
    for (int i = 0; i < 3 && e == hipSuccess; ++i)
        if (outs[i])
            e = hipMemcpyAsync(outs[i], obs + i * N, N * sizeof(double), hipMemcpyDeviceToHost,
                               b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(obs);
    if (e != hipSuccess)
        return bfail(b, LBM_E_DEVICE, std::string("moments: ") + hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_batch_get_state(lbm_batch *b, int32_t sim, double *f)
{
    lbm_status st = benter(b);
    if (st != LBM_OK) return st;
    if (sim < 0 || sim >= b->n || !f) return bfail(b, LBM_E_INVALID, "no such simulation");
    // into planes f[9][ny][nx], one strided copy per population
    const KParams &k = b->kp[sim];
    const size_t nx = k.nx, N = b->N[sim], row = nx * sizeof(double);
    const double *src = b->sb[sim].f[sim_parity(b, sim)];
    for (int q = 0; q < 9; ++q)
        BHIP_OR(b, hipMemcpy2DAsync(f + q * N, row, src + q * k.fq, k.fr * sizeof(double), row,
                                    (size_t)k.ny, hipMemcpyDeviceToHost, b->stream));
    BHIP_OR(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

lbm_status lbm_batch_set_velocity(lbm_batch *b, int32_t sim, const double *vx, const double *vy)
{
    lbm_status st = benter(b);
    if (st != LBM_OK) return st;
    if (sim < 0 || sim >= b->n) return bfail(b, LBM_E_INVALID, "no such simulation");
    const KParams &k = b->kp[sim];
    const SimBuffers &q = b->sb[sim];
    const size_t N = b->N[sim];
    double *tmp = nullptr;
    BHIP_OR(b, hipStreamSynchronize(b->stream));
    BHIP_OR(b, hipMalloc(&tmp, 3 * N * sizeof(double)));
    double *fx = tmp, *ux = tmp + N, *uy = tmp + 2 * N;
    double *fc = q.f[sim_parity(b, sim)], *gc = q.g[sim_parity(b, sim)];
    hipError_t e = launch_rows_rho(k, fc, gc, q.rho, q.mux, b->stream);
    if (e == hipSuccess) e = launch_cols_mu(k, q.rho, q.mux, q.mu, q.fy, b->stream);
    if (e == hipSuccess)
        e = launch_rows_observe(k, fc, q.mu, q.fy, q.rho, nullptr, nullptr, nullptr, fx, b->stream);
    if (e == hipSuccess)
        e = vx ? hipMemcpyAsync(ux, vx, N * sizeof(double), hipMemcpyHostToDevice, b->stream)
               : hipMemsetAsync(ux, 0, N * sizeof(double), b->stream);
    if (e == hipSuccess)
        e = vy ? hipMemcpyAsync(uy, vy, N * sizeof(double), hipMemcpyHostToDevice, b->stream)
               : hipMemsetAsync(uy, 0, N * sizeof(double), b->stream);
    if (e == hipSuccess) e = launch_bare_velocity(k, q.rho, fx, q.fy, ux, uy, b->stream);
    if (e == hipSuccess) e = launch_init_feq(k, q.rho, ux, uy, fc, b->stream);
    if (e == hipSuccess) e = launch_density_groups(k, fc, gc, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess)
        return bfail(b, LBM_E_DEVICE, std::string("set_velocity: ") + hipGetErrorString(e));
    return LBM_OK;
}

int64_t lbm_batch_steps(const lbm_batch *b, int32_t sim)
{
    if (!b || sim < 0 || sim >= b->n) return -1;
    return b->steps[sim];
}

void lbm_batch_destroy(lbm_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    batch_drop_graphs(b);
    void *ptrs[] = {b->mem, b->d_kp, b->d_sb, b->d_rows, b->d_cols, b->d_res};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

const char *lbm_batch_last_error(const lbm_batch *b)
{
    return b ? b->err.c_str() : g_batch_error.c_str();
}

}  // extern "C"
