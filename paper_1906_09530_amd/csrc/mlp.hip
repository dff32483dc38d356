// Kernels of the learned warm start: a 7-128-128-3 tanh network trained in
// FP32 (forward, backpropagation, Adam) and evaluated in BF16 on the matrix
// cores, and the warm-start density and velocity fields of a static drop
// built from it.
//
// Parameters (FP32, one flat array): W1 [128][7], b1 [128], W2 [128][128],
// b2 [128], W3 [3][128], b3 [3].  Network: a1 = tanh(W1 x + b1),
// a2 = tanh(W2 a1 + b2), y = W3 a2 + b3; loss = mean over samples of
// sum_j (y_j - t_j)^2.
#include "mlp.hpp"

namespace cplbm {
namespace mlp {

namespace {

constexpr int H = kHidden, NI = kInputs, NO = kOutputs;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * NI, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + NO * H;
static_assert(OFF_B3 + NO == kParams, "parameter layout");

// ---- FP32 forward (and the first backward step) --------------------------
// A block holds 32 samples; thread t works on sample t / 8 and hidden units
// 16 (t % 8) .. +15.  W2 is staged transposed in LDS, half of its inputs k at
// a time (32 KB), so a thread reads 16 consecutive units of one input with
// four float4 loads.
constexpr int FT = 256, FS = 32, FU = 16, KH = H / 2;

template <bool TRAIN>
__global__ __launch_bounds__(FT) void k_forward_f32(const float *__restrict__ w,
                                                    const float *__restrict__ x,
                                                    const float *__restrict__ t,
                                                    const int32_t *__restrict__ idx, int n,
                                                    int nsrc, int *__restrict__ bad,
                                                    float inv_n, float *__restrict__ y_out,
                                                    float *__restrict__ xb, float *__restrict__ a1g,
                                                    float *__restrict__ a2g,
                                                    float *__restrict__ dz2g,
                                                    float *__restrict__ dyg,
                                                    float *__restrict__ loss_part)
{
    __shared__ float w2t[KH * H];  // w2t[(k - k0) * H + u] = W2[u][k]
    __shared__ float a1s[FS * H];
    __shared__ float red[FS];
    const int tid = threadIdx.x;
    const int sl = tid / 8, u0 = (tid % 8) * FU;
    const int s = blockIdx.x * FS + sl;
    const bool ok = s < n;
    int src = ok ? (idx ? idx[s] : s) : 0;
    if (src < 0 || src >= nsrc) {  // an index outside the sample set
        *bad = 1;
        src = 0;
    }
    float xv[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) xv[i] = ok ? x[(size_t)src * NI + i] : 0.f;
    if (TRAIN && ok && (tid % 8) == 0) {
#pragma unroll
        for (int i = 0; i < NI; ++i) xb[(size_t)s * NI + i] = xv[i];
    }
    // layer 1: 16 units of this sample
    float a1v[FU];
#pragma unroll
    for (int j = 0; j < FU; ++j) {
        const int u = u0 + j;
        float z = w[OFF_B1 + u];
#pragma unroll
        for (int i = 0; i < NI; ++i) z = fmaf(w[OFF_W1 + u * NI + i], xv[i], z);
        a1v[j] = tanhf(z);
        a1s[sl * H + u] = a1v[j];
    }
    if (TRAIN && ok) {
#pragma unroll
        for (int j = 0; j < FU; j += 4)
            *reinterpret_cast<float4 *>(a1g + (size_t)s * H + u0 + j) =
                make_float4(a1v[j], a1v[j + 1], a1v[j + 2], a1v[j + 3]);
    }
    // layer 2, over the two halves of the inputs
    float z2[FU];
#pragma unroll
    for (int j = 0; j < FU; ++j) z2[j] = w[OFF_B2 + u0 + j];
    for (int k0 = 0; k0 < H; k0 += KH) {
        __syncthreads();
        for (int e = tid; e < KH * H; e += FT) {
            const int u = e / KH, kk = e - u * KH;
            w2t[kk * H + u] = w[OFF_W2 + u * H + k0 + kk];
        }
        __syncthreads();
        for (int kk = 0; kk < KH; ++kk) {
            const float a = a1s[sl * H + k0 + kk];
            const float4 *wr = reinterpret_cast<const float4 *>(w2t + kk * H + u0);
#pragma unroll
            for (int q = 0; q < FU / 4; ++q) {
                const float4 v = wr[q];
                z2[4 * q + 0] = fmaf(v.x, a, z2[4 * q + 0]);
                z2[4 * q + 1] = fmaf(v.y, a, z2[4 * q + 1]);
                z2[4 * q + 2] = fmaf(v.z, a, z2[4 * q + 2]);
                z2[4 * q + 3] = fmaf(v.w, a, z2[4 * q + 3]);
            }
        }
    }
    // layer 3: partial dots over this thread's units, then over the 8 threads
    float a2v[FU], y[NO];
#pragma unroll
    for (int j = 0; j < FU; ++j) a2v[j] = tanhf(z2[j]);
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        float part = 0.f;
#pragma unroll
        for (int j = 0; j < FU; ++j) part = fmaf(w[OFF_W3 + o * H + u0 + j], a2v[j], part);
        part += __shfl_xor(part, 1);
        part += __shfl_xor(part, 2);
        part += __shfl_xor(part, 4);
        y[o] = part + w[OFF_B3 + o];
    }
    if (!TRAIN) {
        if (ok && (tid % 8) == 0) {
#pragma unroll
            for (int o = 0; o < NO; ++o) y_out[(size_t)s * NO + o] = y[o];
        }
        return;
    }
    float dy[NO], sq = 0.f;
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        const float err = ok ? y[o] - t[(size_t)src * NO + o] : 0.f;
        sq = fmaf(err, err, sq);
        dy[o] = 2.f * err * inv_n;
    }
    if (ok) {
        float d[FU];
#pragma unroll
        for (int j = 0; j < FU; ++j) {
            float back = 0.f;
#pragma unroll
            for (int o = 0; o < NO; ++o) back = fmaf(dy[o], w[OFF_W3 + o * H + u0 + j], back);
            d[j] = back * (1.f - a2v[j] * a2v[j]);
        }
#pragma unroll
        for (int j = 0; j < FU; j += 4) {
            *reinterpret_cast<float4 *>(a2g + (size_t)s * H + u0 + j) =
                make_float4(a2v[j], a2v[j + 1], a2v[j + 2], a2v[j + 3]);
            *reinterpret_cast<float4 *>(dz2g + (size_t)s * H + u0 + j) =
                make_float4(d[j], d[j + 1], d[j + 2], d[j + 3]);
        }
        if ((tid % 8) == 0) {
#pragma unroll
            for (int o = 0; o < NO; ++o) dyg[(size_t)s * NO + o] = dy[o];
        }
    }
    // block sum of squared errors (fixed order), one partial per block
    if ((tid % 8) == 0) red[sl] = sq;
    __syncthreads();
    if (tid == 0) {
        float acc = 0.f;
        for (int i = 0; i < FS; ++i) acc += red[i];
        loss_part[blockIdx.x] = acc;
    }
}

// ---- backward through W2: dz1 = (W2^T dz2) * (1 - a1^2) -------------------
// Same thread layout; W2 rows staged in LDS half at a time (32 KB).
__global__ __launch_bounds__(FT) void k_backward_dz1(const float *__restrict__ w,
                                                     const float *__restrict__ dz2g,
                                                     const float *__restrict__ a1g, int n,
                                                     float *__restrict__ dz1g)
{
    __shared__ float w2[KH * H];  // w2[(u - u0) * H + k] = W2[u][k]
    __shared__ float ds[FS * H];
    const int tid = threadIdx.x;
    const int s0 = blockIdx.x * FS;
    for (int e = tid; e < FS * H; e += FT) {
        const int s = s0 + e / H;
        ds[e] = s < n ? dz2g[(size_t)s0 * H + e] : 0.f;
    }
    const int sl = tid / 8, k0 = (tid % 8) * FU;
    const int s = s0 + sl;
    float acc[FU];
#pragma unroll
    for (int j = 0; j < FU; ++j) acc[j] = 0.f;
    for (int uh = 0; uh < H; uh += KH) {
        __syncthreads();
        for (int e = tid; e < KH * H; e += FT) w2[e] = w[OFF_W2 + uh * H + e];
        __syncthreads();
        for (int uu = 0; uu < KH; ++uu) {
            const float d = ds[sl * H + uh + uu];
            const float4 *wr = reinterpret_cast<const float4 *>(w2 + uu * H + k0);
#pragma unroll
            for (int q = 0; q < FU / 4; ++q) {
                const float4 v = wr[q];
                acc[4 * q + 0] = fmaf(v.x, d, acc[4 * q + 0]);
                acc[4 * q + 1] = fmaf(v.y, d, acc[4 * q + 1]);
                acc[4 * q + 2] = fmaf(v.z, d, acc[4 * q + 2]);
                acc[4 * q + 3] = fmaf(v.w, d, acc[4 * q + 3]);
            }
        }
    }
    if (s >= n) return;
#pragma unroll
    for (int j = 0; j < FU; j += 4) {
        const float4 a = *reinterpret_cast<const float4 *>(a1g + (size_t)s * H + k0 + j);
        *reinterpret_cast<float4 *>(dz1g + (size_t)s * H + k0 + j) =
            make_float4(acc[j] * (1.f - a.x * a.x), acc[j + 1] * (1.f - a.y * a.y),
                        acc[j + 2] * (1.f - a.z * a.z), acc[j + 3] * (1.f - a.w * a.w));
    }
}

// ---- weight gradients: C[i][j] = sum_s A[s][i] B[s][j] --------------------
// A is n x M (lda), B is n x N (ldb) or all ones when null.  One thread per
// output; a block covers 256 outputs and walks the samples in a fixed order,
// staging 32 samples of both operands in LDS.
constexpr int GT = 256, GS = 32;

__global__ __launch_bounds__(GT) void k_atb(const float *__restrict__ A, int lda, int M,
                                            const float *__restrict__ B, int ldb, int N, int n,
                                            float *__restrict__ C)
{
    __shared__ float as[GS][H + 1];
    __shared__ float bs[GS][H + 1];
    const int o = blockIdx.x * GT + threadIdx.x;
    const int i = o / N, j = o - (o / N) * N;
    const bool ok = o < M * N;
    // the block's outputs span rows i_lo..i_hi of A's columns and all of B's
    const int i_lo = (blockIdx.x * GT) / N;
    const int i_hi = min(M - 1, (blockIdx.x * GT + GT - 1) / N);
    const int mi = i_hi - i_lo + 1;
    float acc = 0.f;
    for (int s0 = 0; s0 < n; s0 += GS) {
        const int ns = min(GS, n - s0);
        __syncthreads();
        for (int e = threadIdx.x; e < GS * mi; e += GT) {
            const int r = e / mi, c = e - r * mi;
            as[r][c] = r < ns ? A[(size_t)(s0 + r) * lda + i_lo + c] : 0.f;
        }
        for (int e = threadIdx.x; e < GS * N; e += GT) {
            const int r = e / N, c = e - r * N;
            bs[r][c] = r < ns ? (B ? B[(size_t)(s0 + r) * ldb + c] : 1.f) : 0.f;
        }
        __syncthreads();
        if (ok) {
            for (int r = 0; r < ns; ++r) acc = fmaf(as[r][i - i_lo], bs[r][j], acc);
        }
    }
    if (ok) C[o] = acc;
}

// ---- Adam (Kingma and Ba 2015, Algorithm 1, bias-corrected moments) -------
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int np, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// sum of the per-block partials in a fixed order (one thread)
__global__ void k_fold(const float *__restrict__ part, int np, float scale, float *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float acc = 0.f;
    for (int i = 0; i < np; ++i) acc += part[i];
    out[0] = acc * scale;
}

// ---- BF16 inference on the matrix cores -----------------------------------
// bfloat16 = upper half of binary32 after rounding to nearest, ties to even.
__device__ __forceinline__ unsigned short to_bf16(float f)
{
    const unsigned int u = __float_as_uint(f);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// A block of 256 threads (4 waves) evaluates 64 samples.  Layer 1 in FP32
// (thread t: sample t / 4, units 32 (t % 4) .. +31), a1 rounded to bf16 in
// LDS; layer 2 with v_mfma_f32_16x16x16bf16 (wave w: samples 16w .. 16w+15,
// eight 16-unit output tiles, eight 16-deep k steps), FP32 accumulation;
// tanh, and layer 3 reduced across the 16 lanes that share a sample row.
// Operand lanes of the 16x16x16 instruction: lane l supplies A[l % 16][4 (l / 16) + 0..3]
// and B[4 (l / 16) + 0..3][l % 16]; it receives D[4 (l / 16) + 0..3][l % 16].
constexpr int IT = 256, IS = 64;

struct alignas(16) BfTile {
    unsigned short a1[IS * H];  // [sample][k]
    unsigned short w2[H * H];   // [u][k] = W2 row-major
};

__device__ __forceinline__ void bf16_tile_load_w2(const float *__restrict__ w, BfTile &t)
{
    for (int e = threadIdx.x; e < H * H; e += IT) t.w2[e] = to_bf16(w[OFF_W2 + e]);
}

// x: this thread's features (sample threadIdx.x / 4 of the tile); returns the
// outputs of sample 16 (threadIdx.x / 64) + 4 ((threadIdx.x % 64) / 16) + r in
// ys[o][r] (every lane of a 16-lane group holds them after the reduction).
__device__ __forceinline__ void bf16_tile_eval(const float *__restrict__ w, BfTile &t,
                                               const float (&xv)[NI], float (&ys)[NO][4])
{
    const int tid = threadIdx.x;
    const int sl = tid / 4, u0 = (tid % 4) * 32;
    for (int j = 0; j < 32; ++j) {
        const int u = u0 + j;
        float z = w[OFF_B1 + u];
#pragma unroll
        for (int i = 0; i < NI; ++i) z = fmaf(w[OFF_W1 + u * NI + i], xv[i], z);
        t.a1[sl * H + u] = to_bf16(tanhf(z));
    }
    __syncthreads();
    const int wave = tid / 64, lane = tid % 64;
    const int row = lane % 16, kq = 4 * (lane / 16);
    float part[NO][4] = {};
    for (int nt = 0; nt < H / 16; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < H / 16; ++kt) {
            const int k = kt * 16 + kq;
            const bf16x4 a = *reinterpret_cast<const bf16x4 *>(&t.a1[(wave * 16 + row) * H + k]);
            const bf16x4 b = *reinterpret_cast<const bf16x4 *>(&t.w2[(nt * 16 + row) * H + k]);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
        const int u = nt * 16 + row;  // output unit of this lane
        const float bu = w[OFF_B2 + u];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float a2 = tanhf(acc[r] + bu);
#pragma unroll
            for (int o = 0; o < NO; ++o) part[o][r] = fmaf(w[OFF_W3 + o * H + u], a2, part[o][r]);
        }
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float p = part[o][r];
            p += __shfl_xor(p, 1);
            p += __shfl_xor(p, 2);
            p += __shfl_xor(p, 4);
            p += __shfl_xor(p, 8);
            ys[o][r] = p + w[OFF_B3 + o];
        }
    }
}

__global__ __launch_bounds__(IT) void k_infer_bf16(const float *__restrict__ w,
                                                   const float *__restrict__ x, int n,
                                                   float *__restrict__ y)
{
    __shared__ BfTile t;
    bf16_tile_load_w2(w, t);
    const int s = blockIdx.x * IS + threadIdx.x / 4;
    float xv[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) xv[i] = s < n ? x[(size_t)s * NI + i] : 0.f;
    float ys[NO][4];
    bf16_tile_eval(w, t, xv, ys);
    const int lane = threadIdx.x % 64;
    if (lane % 16 == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int so = blockIdx.x * IS + (threadIdx.x / 64) * 16 + 4 * (lane / 16) + r;
            if (so < n) {
#pragma unroll
                for (int o = 0; o < NO; ++o) y[(size_t)so * NO + o] = ys[o][r];
            }
        }
    }
}

// ---- warm-start fields of a static drop ------------------------------------
// Node n = y * nx + x, at distance r and polar angle theta from the centre,
// has features (T/Tc, R / R_ref, kappa, k, r - R, cos 4 theta, sin 4 theta),
// normalised by (f - centre) / scale.
__device__ __forceinline__ void node_polar(const WsDrop &d, int n, double &r, double &c,
                                           double &sn)
{
    const int yy = n / d.nx, xx = n - yy * d.nx;
    const double dx = xx - d.cx, dy = yy - d.cy;
    r = sqrt(dx * dx + dy * dy);
    c = r > 0.0 ? dx / r : 1.0;  // theta = 0 at the centre itself
    sn = r > 0.0 ? dy / r : 0.0;
}

// Rows n and N + n of x: the features of node n, and those of its mirror
// image (sin 4 theta negated; every reflection of the square maps
// (cos 4 theta, sin 4 theta) to (cos 4 theta, -sin 4 theta)).
__global__ void k_ws_features(WsDrop d, float *__restrict__ x)
{
    const int N = d.nx * d.ny;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double r, c, sn;
    node_polar(d, n, r, c, sn);
    const double c2 = c * c - sn * sn, s2 = 2.0 * c * sn;
    const double f[NI] = {d.T_r, d.radius / d.radius_ref, d.kappa, d.k, r - d.radius,
                          c2 * c2 - s2 * s2, 2.0 * s2 * c2};
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const double v = (f[i] - d.center[i]) / d.scale[i];
        x[(size_t)n * NI + i] = (float)v;
        x[((size_t)N + n) * NI + i] = (float)(i == NI - 1 ? -v : v);
    }
}

// Outputs to fields, made exactly symmetric under the reflections of the
// square about the drop's centre: with y+ the outputs of node n and y- those
// of its mirror features, y0 = (y0+ + y0-)/2 and the radial velocity
// (y1+ + y1-)/2 are even, the azimuthal velocity (y2+ - y2-)/2 odd, and the
// velocity normal to a mirror line vanishes on it, so the proposed state
// carries no net momentum and the drop does not drift.  rho = exp(ln rho_g + w y0 (ln rho_l
// - ln rho_g)); velocity w times the outputs, in units of u_scale.  w = 1
// within reach of the interface (r - R <= reach - kReachBlend), 0 beyond
// reach + kReachBlend (the Maxwell gas at rest), linear in r between; an
// infinite reach keeps w = 1 everywhere.  Each block of 256 nodes also
// writes the partial sums of rho and of the mass-matching weight
// max((rho - rho_g)(rho_l - rho), 0).
constexpr int MT = 256;
constexpr double kReachBlend = 10.0;

__global__ __launch_bounds__(MT) void k_ws_map(WsDrop d, const float *__restrict__ y,
                                               double *__restrict__ rho,
                                               double *__restrict__ ux,
                                               double *__restrict__ uy,
                                               double *__restrict__ part)
{
    __shared__ double red[2][MT];
    const int N = d.nx * d.ny;
    const int n = blockIdx.x * MT + threadIdx.x;
    double rv = 0.0, wv = 0.0;
    if (n < N) {
        double r, c, sn;
        node_polar(d, n, r, c, sn);
        const double w =
            isinf(d.reach)
                ? 1.0
                : fmin(fmax((d.reach + kReachBlend - (r - d.radius)) / (2.0 * kReachBlend), 0.0),
                       1.0);
        const float *yp = y + (size_t)n * NO, *ym = y + ((size_t)N + n) * NO;
        const double y0 = w * (0.5 * ((double)yp[0] + (double)ym[0]));
        rv = exp(d.ln_rho_g + y0 * (d.ln_rho_l - d.ln_rho_g));
        rho[n] = rv;
        wv = fmax((rv - d.rho_g) * (d.rho_l - rv), 0.0);
        if (ux) {
            const double ur = w * (d.u_scale * 0.5 * ((double)yp[1] + (double)ym[1]));
            const double ut = w * (d.u_scale * 0.5 * ((double)yp[2] - (double)ym[2]));
            // a node that is its own mirror image about the line x = cx (the
            // centre column, and the edge column of a periodic mesh when cx
            // sits half a period away) has no x velocity; likewise in y
            const int yy = n / d.nx, xx = n - yy * d.nx;
            const bool self_x = fmod(2.0 * (xx - d.cx), (double)d.nx) == 0.0;
            const bool self_y = fmod(2.0 * (yy - d.cy), (double)d.ny) == 0.0;
            ux[n] = self_x ? 0.0 : ur * c - ut * sn;
            uy[n] = self_y ? 0.0 : ur * sn + ut * c;
        }
    }
    red[0][threadIdx.x] = rv;
    red[1][threadIdx.x] = wv;
    __syncthreads();
    if (threadIdx.x < 2) {
        double acc = 0.0;
        for (int i = 0; i < MT; ++i) acc += red[threadIdx.x][i];
        part[2 * blockIdx.x + threadIdx.x] = acc;
    }
}

// c = (target - sum rho) / sum w over the block partials, in block order.
__global__ void k_ws_fold(const double *__restrict__ part, int nb, double target,
                          double *__restrict__ c)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double sr = 0.0, sw = 0.0;
    for (int i = 0; i < nb; ++i) {
        sr += part[2 * i];
        sw += part[2 * i + 1];
    }
    c[0] = sw > 0.0 ? (target - sr) / sw : 0.0;
}

// rho += c w; a density that ends non-positive or non-finite sets *bad.
__global__ void k_ws_apply(double *__restrict__ rho, int N, double rho_g, double rho_l,
                           const double *__restrict__ c, int *__restrict__ bad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double r = rho[i];
    const double v = r + c[0] * fmax((r - rho_g) * (rho_l - r), 0.0);
    rho[i] = v;
    if (!(v > 0.0 && v < INFINITY)) *bad = 1;
}

}  // namespace

// Training workspace regions, each starting on a 256-byte boundary.
struct TrainWs {
    size_t xb, a1, a2, dz2, dz1, dy, lp, total;
};

static TrainWs train_ws_layout(int batch)
{
    auto up = [](size_t n) { return (n + 63) & ~size_t(63); };
    TrainWs L;
    const size_t B = batch;
    L.xb = 0;
    L.a1 = L.xb + up(B * NI);
    L.a2 = L.a1 + up(B * H);
    L.dz2 = L.a2 + up(B * H);
    L.dz1 = L.dz2 + up(B * H);
    L.dy = L.dz1 + up(B * H);
    L.lp = L.dy + up(B * NO);
    L.total = L.lp + up((B + FS - 1) / FS);
    return L;
}

size_t train_ws_floats(int batch) { return train_ws_layout(batch).total; }

hipError_t train_step(float *w, float *g, float *m, float *v, const float *x, const float *t,
                      int nsrc, const int32_t *idx, int batch, float lr, float b1, float b2,
                      float eps, float c1, float c2, float *ws, int *bad, float *loss_dev,
                      hipStream_t s)
{
    const TrainWs L = train_ws_layout(batch);
    float *xb = ws + L.xb, *a1 = ws + L.a1, *a2 = ws + L.a2, *dz2 = ws + L.dz2;
    float *dz1 = ws + L.dz1, *dy = ws + L.dy, *lp = ws + L.lp;
    const int nb = (batch + FS - 1) / FS;
    hipLaunchKernelGGL(k_forward_f32<true>, dim3(nb), dim3(FT), 0, s, w, x, t, idx, batch, nsrc,
                       bad, 1.f / batch, nullptr, xb, a1, a2, dz2, dy, lp);
    hipLaunchKernelGGL(k_backward_dz1, dim3(nb), dim3(FT), 0, s, w, dz2, a1, batch, dz1);
    auto atb = [&](const float *A, int lda, int M, const float *B, int ldb, int N, float *C) {
        const int outs = M * N;
        hipLaunchKernelGGL(k_atb, dim3((outs + GT - 1) / GT), dim3(GT), 0, s, A, lda, M, B, ldb,
                           N, batch, C);
    };
    atb(dz1, H, H, xb, NI, NI, g + OFF_W1);      // dW1[u][i] = sum dz1[s][u] x[s][i]
    atb(dz1, H, H, nullptr, 0, 1, g + OFF_B1);   // db1
    atb(dz2, H, H, a1, H, H, g + OFF_W2);        // dW2[u][k] = sum dz2[s][u] a1[s][k]
    atb(dz2, H, H, nullptr, 0, 1, g + OFF_B2);   // db2
    atb(dy, NO, NO, a2, H, H, g + OFF_W3);       // dW3[o][u] = sum dy[s][o] a2[s][u]
    atb(dy, NO, NO, nullptr, 0, 1, g + OFF_B3);  // db3
    if (loss_dev)
        hipLaunchKernelGGL(k_fold, dim3(1), dim3(64), 0, s, lp, nb, 1.f / batch, loss_dev);
    if (m)
        hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, w, g, m, v,
                           kParams, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t forward_f32(const float *w, const float *x, int n, float *y, int *bad, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_forward_f32<false>, dim3((n + FS - 1) / FS), dim3(FT), 0, s, w, x,
                       nullptr, nullptr, n, n, bad, 0.f, y, nullptr, nullptr, nullptr, nullptr,
                       nullptr, nullptr);
    return hipGetLastError();
}

hipError_t forward_bf16(const float *w, const float *x, int n, float *y, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_infer_bf16, dim3((n + IS - 1) / IS), dim3(IT), 0, s, w, x, n, y);
    return hipGetLastError();
}

int ws_field_blocks(int nodes) { return (nodes + MT - 1) / MT; }

hipError_t warm_start_field(const float *w, const WsDrop &d, bool bf16, double target_mass,
                            float *x, float *y, double *rho, double *ux, double *uy,
                            double *part, double *c, int *bad, hipStream_t s)
{
    const int N = d.nx * d.ny;
    const int nb = ws_field_blocks(N);
    hipLaunchKernelGGL(k_ws_features, dim3(nb), dim3(MT), 0, s, d, x);
    hipError_t e = bf16 ? forward_bf16(w, x, 2 * N, y, s) : forward_f32(w, x, 2 * N, y, bad, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ws_map, dim3(nb), dim3(MT), 0, s, d, y, rho, ux, uy, part);
    hipLaunchKernelGGL(k_ws_fold, dim3(1), dim3(64), 0, s, part, nb, target_mass, c);
    hipLaunchKernelGGL(k_ws_apply, dim3((N + 255) / 256), dim3(256), 0, s, rho, N, d.rho_g,
                       d.rho_l, c, bad);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace cplbm
