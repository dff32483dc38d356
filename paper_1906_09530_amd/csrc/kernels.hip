// HIP kernels of one time step of the chemical-potential multiphase LBM
// (arXiv:1906.09530) for gfx950, FP64 throughout.
//
// A step is three passes over the mesh:
//   A (rows)    rho = sum_i f_i (Eq. 3); d/dx rho and d2/dx2 rho by the
//               compact scheme (Eqs. 37-39, second derivative by applying it
//               twice, Sec. 4.3).  Writes rho and d2/dx2 rho.
//   B (columns) d/dy rho, d2/dy2 rho, the mesh chemical potential
//               mu = k^2 psi'(rho) - kappa lap(rho) (Eq. 33) with psi'
//               bounded by the upper limit of Sec. 5.6, d/dy mu and
//               F_y = -rho d/dy mu + c_s^2 d/dy rho (Eq. 12).  Writes mu, F_y.
//   C (rows)    d/dx rho, d/dx mu, F_x; BGK collision with the
//               exact-difference force term (Eqs. 1, 2, 5) and push-streaming
//               into the other distribution buffer.
//
// Line solves.  Eq. 37 on a periodic line is the circulant system
//   d_i + al (d_{i-1} + d_{i+1}) = r_i.
// Parallel cyclic reduction eliminates the neighbours at stride h = 2^s:
//   r_i <- (r_i - c (r_{i-h} + r_{i+h})) / (1 - 2 c^2),  c <- -c^2 / (1 - 2 c^2).
// Because the matrix is circulant, c is one scalar per stage (precomputed
// on the host).  |c| falls doubly exponentially (1/3, 1/7, 1/47, 1/2207, ...),
// so after a handful of stages the remaining coupling is below 1e-18 and
// d_i = r_i to FP64 round-off; indices are taken modulo the line length, which
// keeps every stage an exact linear combination of the original equations.
// The line lives in LDS; each stage is one read-neighbours/write pass.
//
// Walls (bc_y = 1): a column is treated as the even extension of length 2 ny
// about the walls.  Only the ny physical values are stored; a read of an
// extended position returns the mirrored value times the parity of the
// quantity (+1 for rho, mu, second derivatives; -1 for first derivatives
// and their right-hand sides).
#include "kernels.hpp"

namespace cplbm {

namespace {

// D2Q9 (Sec. 2)
__device__ constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
__device__ constexpr double WT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                                     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
constexpr double CS2 = 1.0 / 3.0;

// rho = sum f_i in a fixed order (every pass computes it the same way).
__device__ __forceinline__ double sum9(const double (&fi)[9])
{
    double r = fi[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) r += fi[i];
    return r;
}

__device__ __forceinline__ void load9(const double *__restrict__ f, size_t N, size_t node,
                                      double (&fi)[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) fi[i] = f[i * N + node];
}

// Equilibrium of Eq. 2 with c_s^2 = 1/3.
__device__ __forceinline__ double feq(int i, double rho, double ux, double uy, double uu)
{
    const double eu = EX[i] * ux + EY[i] * uy;
    return WT[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

// psi'(rho) of Eqs. 15, 17, 19, 21, bounded by the upper limit (Sec. 5.6):
// outside the EOS domain, or when the formula gives NaN, the limit is used.
__device__ __forceinline__ double mu0_capped(const KParams &p, double rho)
{
    const double b = p.b, RT = p.RT, A = p.A;
    const bool outside = (p.eos == 4) ? (b * rho * 0.25 >= 1.0) : (b * rho >= 1.0);
    if (outside) return p.mu_cap;
    double m;
    switch (p.eos) {
    case 0:  // van der Waals
        m = RT * (log(rho / (1.0 - b * rho)) + 1.0 / (1.0 - b * rho)) - 2.0 * p.a * rho;
        break;
    case 1:
    case 2:  // Redlich-Kwong, Soave-Redlich-Kwong
        m = RT * log(rho / (1.0 - b * rho)) + RT / (1.0 - b * rho) - A / b * log(1.0 + b * rho) -
            A * rho / (1.0 + b * rho);
        break;
    case 3: {  // Peng-Robinson
        const double s2 = 1.4142135623730950488;
        m = RT * log(rho / (1.0 - b * rho)) -
            A / (2.0 * s2 * b) * log((s2 - 1.0 + b * rho) / (s2 + 1.0 - b * rho)) +
            RT / (1.0 - b * rho) - A * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
        break;
    }
    default: {  // Carnahan-Starling
        const double eta = b * rho * 0.25, q = 1.0 - eta;
        m = RT * ((3.0 - eta) / (q * q * q) + log(rho) + 1.0) - 2.0 * p.a * rho;
        break;
    }
    }
    if (isnan(m)) return p.mu_cap;
    return m < p.mu_cap ? m : p.mu_cap;
}

// Lines held by a block in LDS.  Element e of the block is LDS slot e:
// row layout slot = l * n + j, column layout slot = j * nl + l.
struct LineMap {
    int n;       // stored length of each line
    int period;  // n (periodic) or 2 n (even extension between walls)
    int nl;      // lines in the block
    bool col;
    __device__ __forceinline__ int slot(int l, int j) const { return col ? j * nl + l : l * n + j; }
    // value at position j (any integer) of line l; par = parity of the quantity
    __device__ __forceinline__ double get(const double *buf, int l, int j, double par) const
    {
        int m = j % period;
        if (m < 0) m += period;
        if (m >= n) return par * buf[slot(l, period - 1 - m)];
        return buf[slot(l, m)];
    }
};

struct Elems {
    int l[kElemsPerThread], j[kElemsPerThread], e[kElemsPerThread];
    bool ok[kElemsPerThread];
};

__device__ __forceinline__ Elems make_elems(const LineMap &m)
{
    Elems E;
    const int total = m.n * m.nl;
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        int e = threadIdx.x + k * kBlockThreads;
        E.e[k] = e;
        E.ok[k] = e < total;
        if (m.col) {
            E.j[k] = e / m.nl;
            E.l[k] = e - E.j[k] * m.nl;
        } else {
            E.l[k] = e / m.n;
            E.j[k] = e - E.l[k] * m.n;
        }
    }
    return E;
}

// First derivative along the block's lines by the compact scheme.  `in`
// holds the input (parity par_in) for every element and is visible to the
// whole block; `tmp` is scratch.  Returns the buffer holding the result
// (parity -par_in); the calling thread's results are also left in out[].
__device__ double *cfm_solve(const KParams &p, const LineMap &m, const Elems &E, double *in,
                             double *tmp, double par_in, double (&out)[kElemsPerThread])
{
    const double par = -par_in;
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        const int l = E.l[k], j = E.j[k];
        double r = p.cfd_a2 * (m.get(in, l, j + 1, par_in) - m.get(in, l, j - 1, par_in)) +
                   p.cfd_b4 * (m.get(in, l, j + 2, par_in) - m.get(in, l, j - 2, par_in));
        tmp[E.e[k]] = r;
        out[k] = r;
    }
    __syncthreads();
    double *src = tmp, *dst = in;
    for (int s = 0; s < p.nstage; ++s) {
        const int h = 1 << s;
        const double c = p.pcr_c[s], g = p.pcr_g[s];
#pragma unroll
        for (int k = 0; k < kElemsPerThread; ++k) {
            if (!E.ok[k]) continue;
            const int l = E.l[k], j = E.j[k];
            double v = (src[E.e[k]] - c * (m.get(src, l, j - h, par) + m.get(src, l, j + h, par))) * g;
            dst[E.e[k]] = v;
            out[k] = v;
        }
        __syncthreads();
        double *t = src;
        src = dst;
        dst = t;
    }
    return src;
}

__global__ __launch_bounds__(kBlockThreads) void k_rows_rho(KParams p,
                                                            const double *__restrict__ f,
                                                            double *__restrict__ rho_out,
                                                            double *__restrict__ dxx_out)
{
    __shared__ double bA[kBlockElems], bB[kBlockElems];
    const int nx = p.nx, ny = p.ny;
    const size_t N = (size_t)nx * ny;
    const int y0 = blockIdx.x * p.rows_per_block;
    const int rows = min(p.rows_per_block, ny - y0);
    const LineMap m{nx, nx, rows, false};
    const Elems E = make_elems(m);
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        const size_t node = (size_t)(y0 + E.l[k]) * nx + E.j[k];
        double fi[9];
        load9(f, N, node, fi);
        const double r = sum9(fi);
        bA[E.e[k]] = r;
        rho_out[node] = r;
    }
    if (p.kappa_zero) return;  // uniform: the Laplacian is not used
    __syncthreads();
    double d1[kElemsPerThread], d2[kElemsPerThread];
    double *res = cfm_solve(p, m, E, bA, bB, 1.0, d1);
    cfm_solve(p, m, E, res, res == bA ? bB : bA, -1.0, d2);
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        dxx_out[(size_t)(y0 + E.l[k]) * nx + E.j[k]] = d2[k];
    }
}

__global__ __launch_bounds__(kBlockThreads) void k_cols_mu(KParams p,
                                                           const double *__restrict__ rho,
                                                           const double *__restrict__ dxx,
                                                           double *__restrict__ mu_out,
                                                           double *__restrict__ fy_out)
{
    __shared__ double bA[kBlockElems], bB[kBlockElems];
    const int nx = p.nx, ny = p.ny;
    const int x0 = blockIdx.x * p.cols_per_block;
    const int cols = min(p.cols_per_block, nx - x0);
    const LineMap m{ny, p.bc_y ? 2 * ny : ny, cols, true};
    const Elems E = make_elems(m);
    double r[kElemsPerThread];
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        r[k] = rho[(size_t)E.j[k] * nx + x0 + E.l[k]];
        bA[E.e[k]] = r[k];
    }
    __syncthreads();
    double dyr[kElemsPerThread], dyy[kElemsPerThread], dym[kElemsPerThread];
    double *res = cfm_solve(p, m, E, bA, bB, 1.0, dyr);
    if (!p.kappa_zero) cfm_solve(p, m, E, res, res == bA ? bB : bA, -1.0, dyy);
    // chemical potential, Eq. 33 (all reads of bA/bB finished at the last barrier)
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        const size_t node = (size_t)E.j[k] * nx + x0 + E.l[k];
        double mu = p.k2 * mu0_capped(p, r[k]);
        if (!p.kappa_zero) mu -= p.kappa * (dxx[node] + dyy[k]);
        mu_out[node] = mu;
        bA[E.e[k]] = mu;
    }
    __syncthreads();
    cfm_solve(p, m, E, bA, bB, 1.0, dym);
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        fy_out[(size_t)E.j[k] * nx + x0 + E.l[k]] = -r[k] * dym[k] + CS2 * dyr[k];
    }
}

template <bool OBSERVE>
__global__ __launch_bounds__(kBlockThreads) void k_rows_collide(
    KParams p, const double *__restrict__ f, const double *__restrict__ mu,
    const double *__restrict__ fy, double *__restrict__ fout, double *__restrict__ o_rho,
    double *__restrict__ o_vx, double *__restrict__ o_vy, double *__restrict__ o_fx)
{
    __shared__ double bA[kBlockElems], bB[kBlockElems];
    const int nx = p.nx, ny = p.ny;
    const size_t N = (size_t)nx * ny;
    const int y0 = blockIdx.x * p.rows_per_block;
    const int rows = min(p.rows_per_block, ny - y0);
    const LineMap m{nx, nx, rows, false};
    const Elems E = make_elems(m);
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        double fi[9];
        load9(f, N, (size_t)(y0 + E.l[k]) * nx + E.j[k], fi);
        bA[E.e[k]] = sum9(fi);
    }
    __syncthreads();
    double dxr[kElemsPerThread], dxm[kElemsPerThread];
    cfm_solve(p, m, E, bA, bB, 1.0, dxr);
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        bA[E.e[k]] = mu[(size_t)(y0 + E.l[k]) * nx + E.j[k]];
    }
    __syncthreads();
    cfm_solve(p, m, E, bA, bB, 1.0, dxm);

#pragma unroll 1
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        const int x = E.j[k], y = y0 + E.l[k];
        const size_t node = (size_t)y * nx + x;
        double fi[9];
        load9(f, N, node, fi);
        const double rho = sum9(fi);
        const double jx = (fi[1] - fi[3]) + (fi[5] - fi[6]) + (fi[8] - fi[7]);
        const double jy = (fi[2] - fi[4]) + (fi[5] - fi[8]) + (fi[6] - fi[7]);
        const double Fx = -rho * dxm[k] + CS2 * dxr[k];
        const double Fy = fy[node];
        const double ux = jx / rho, uy = jy / rho;
        if (OBSERVE) {
            if (o_rho) o_rho[node] = rho;
            if (o_vx) o_vx[node] = ux + Fx / (2.0 * rho);
            if (o_vy) o_vy[node] = uy + Fy / (2.0 * rho);
            if (o_fx) o_fx[node] = Fx;
            continue;
        }
        const double vx2 = ux + Fx / rho, vy2 = uy + Fy / rho;
        const double uu = ux * ux + uy * uy, uu2 = vx2 * vx2 + vy2 * vy2;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double eq = feq(i, rho, ux, uy, uu);
            const double eq2 = feq(i, rho, vx2, vy2, uu2);
            const double fs = fi[i] - (fi[i] - eq) * p.inv_tau + (eq2 - eq);
            int tx = x + EX[i];
            tx = tx < 0 ? tx + nx : (tx >= nx ? tx - nx : tx);
            int ty = y + EY[i];
            if (ty < 0 || ty >= ny) {
                if (p.bc_y) {
                    // half-way bounce-back; a moving wall adds -2 w rho (e.U)/c_s^2
                    const double eu = EX[i] * p.wall_ux;
                    fout[OPP[i] * N + node] = fs - 2.0 * WT[i] * rho * eu / CS2;
                    continue;
                }
                ty = ty < 0 ? ty + ny : ty - ny;
            }
            fout[i * N + (size_t)ty * nx + tx] = fs;
        }
    }
}

__global__ void k_init_feq(KParams p, const double *__restrict__ rho0,
                           const double *__restrict__ ux0, const double *__restrict__ uy0,
                           double *__restrict__ f)
{
    const size_t N = (size_t)p.nx * p.ny;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        const double rho = rho0[n], ux = ux0 ? ux0[n] : 0.0, uy = uy0 ? uy0[n] : 0.0;
        const double uu = ux * ux + uy * uy;
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i * N + n] = feq(i, rho, ux, uy, uu);
    }
}

constexpr int kRedThreads = 256;

__global__ __launch_bounds__(kRedThreads) void k_rho_delta(KParams p, const double *__restrict__ f,
                                                           double *__restrict__ prev,
                                                           double *__restrict__ partial)
{
    __shared__ double smax[kRedThreads], sbad[kRedThreads];
    const size_t N = (size_t)p.nx * p.ny;
    double dmax = 0.0, bad = 0.0;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        double fi[9];
        load9(f, N, n, fi);
        const double r = sum9(fi);
        if (!isfinite(r)) bad = 1.0;
        const double d = fabs(r - prev[n]);
        if (d > dmax) dmax = d;
        prev[n] = r;
    }
    smax[threadIdx.x] = dmax;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            sbad[threadIdx.x] = fmax(sbad[threadIdx.x], sbad[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = smax[0];
        partial[2 * blockIdx.x + 1] = sbad[0];
    }
}

__global__ __launch_bounds__(kRedThreads) void k_fold_partials(const double *__restrict__ partial,
                                                               int nblocks, double *__restrict__ out)
{
    __shared__ double smax[kRedThreads], sbad[kRedThreads];
    double dmax = 0.0, bad = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kRedThreads) {
        dmax = fmax(dmax, partial[2 * b]);
        bad = fmax(bad, partial[2 * b + 1]);
    }
    smax[threadIdx.x] = dmax;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
            sbad[threadIdx.x] = fmax(sbad[threadIdx.x], sbad[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = smax[0];
        out[1] = sbad[0];
    }
}

int row_blocks(const KParams &p) { return (p.ny + p.rows_per_block - 1) / p.rows_per_block; }
int col_blocks(const KParams &p) { return (p.nx + p.cols_per_block - 1) / p.cols_per_block; }

}  // namespace

hipError_t launch_rows_rho(const KParams &p, const double *f, double *rho, double *dxx,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_rows_rho, dim3(row_blocks(p)), dim3(kBlockThreads), 0, s, p, f, rho, dxx);
    return hipGetLastError();
}

hipError_t launch_cols_mu(const KParams &p, const double *rho, const double *dxx, double *mu,
                          double *fy, hipStream_t s)
{
    hipLaunchKernelGGL(k_cols_mu, dim3(col_blocks(p)), dim3(kBlockThreads), 0, s, p, rho, dxx, mu,
                       fy);
    return hipGetLastError();
}

hipError_t launch_rows_collide(const KParams &p, const double *f, const double *mu,
                               const double *fy, double *fout, hipStream_t s)
{
    hipLaunchKernelGGL(k_rows_collide<false>, dim3(row_blocks(p)), dim3(kBlockThreads), 0, s, p, f,
                       mu, fy, fout, nullptr, nullptr, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_rows_observe(const KParams &p, const double *f, const double *mu,
                               const double *fy, double *rho, double *vx, double *vy,
                               double *fx, hipStream_t s)
{
    hipLaunchKernelGGL(k_rows_collide<true>, dim3(row_blocks(p)), dim3(kBlockThreads), 0, s, p, f,
                       mu, fy, nullptr, rho, vx, vy, fx);
    return hipGetLastError();
}

hipError_t launch_init_feq(const KParams &p, const double *rho0, const double *ux0,
                           const double *uy0, double *f, hipStream_t s)
{
    const size_t N = (size_t)p.nx * p.ny;
    int blocks = (int)((N + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_init_feq, dim3(blocks), dim3(256), 0, s, p, rho0, ux0, uy0, f);
    return hipGetLastError();
}

int rho_delta_blocks(const KParams &p)
{
    const size_t N = (size_t)p.nx * p.ny;
    size_t b = (N + kRedThreads * 4 - 1) / (kRedThreads * 4);
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_rho_delta(const KParams &p, const double *f, double *prev, double *partial,
                            int nblocks, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_rho_delta, dim3(nblocks), dim3(kRedThreads), 0, s, p, f, prev, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fold_partials, dim3(1), dim3(kRedThreads), 0, s, partial, nblocks, out);
    return hipGetLastError();
}

}  // namespace cplbm
