// HIP kernels of one time step of the chemical-potential multiphase LBM
// (arXiv:1906.09530) for gfx950, FP64 throughout.
//
// A step is three passes over the mesh:
//   A (rows)    rho = sum_i f_i (Eq. 3); d/dx rho and d2/dx2 rho by the
//               compact scheme (Eqs. 37-39, second derivative by applying it
//               twice, Sec. 4.3); the row part of the mesh chemical potential
//               (Eq. 33), k^2 psi'(rho) - kappa d2rho/dx2, with psi' bounded
//               by the upper limit of Sec. 5.6.  Writes rho and the row part.
//               (The fast kernels of kernels_iir.hip take rho from the three
//               density groups the previous collision wrote.)
//   B (columns) d/dy rho, d2/dy2 rho, mu = row part - kappa d2rho/dy2,
//               d/dy mu and F_y = -rho d/dy mu + c_s^2 d/dy rho (Eq. 12).
//               Writes mu, F_y.
//   C (rows)    d/dx rho, d/dx mu, F_x; BGK collision with the
//               exact-difference force term (Eqs. 1, 2, 5) and push-streaming
//               into the other distribution buffer (and, fast kernels, its
//               density groups).
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
#include <cmath>

#include "kernels.hpp"
#include "physics.hpp"

namespace cplbm {

namespace {

using namespace phys;


// Lines held by a block in LDS.  Element e of the block is LDS slot e:
// row layout slot = l * n + j, column layout slot = j * nl + l.
// FAST: lines of at least kFastMinLine = 64 nodes.  Every offset the solve
// uses is at most 2^(nstage-1) <= 32 (nstage <= 6, checked on the host) or 2
// (right-hand side), so an index leaves [0, n) by less than n and folds back
// by one compare instead of a modulo.
template <bool FAST>
struct LineMap {
    int n;        // stored length of each line
    int nl;       // lines in the block
    bool col;     // column layout
    bool mirror;  // even extension of length 2n (between walls)
    __device__ __forceinline__ int slot(int l, int j) const { return col ? j * nl + l : l * n + j; }
    // value at position j (any integer) of line l; par = parity of the quantity
    __device__ __forceinline__ double get(const double *buf, int l, int j, double par) const
    {
        if (FAST) {
            if (!mirror) {
                j = j < 0 ? j + n : (j >= n ? j - n : j);
                return buf[slot(l, j)];
            }
            if (j < 0) return par * buf[slot(l, -1 - j)];
            if (j >= n) return par * buf[slot(l, 2 * n - 1 - j)];
            return buf[slot(l, j)];
        }
        const int period = mirror ? 2 * n : n;
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

template <bool FAST>
__device__ __forceinline__ Elems make_elems(const LineMap<FAST> &m)
{
    Elems E;
    const int total = m.n * m.nl;
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        int e = threadIdx.x + k * blockDim.x;
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
template <bool FAST>
__device__ __forceinline__ double *cfm_solve(const KParams &p, const LineMap<FAST> &m,
                                             const Elems &E, double *in,
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
            double v = (out[k] - c * (m.get(src, l, j - h, par) + m.get(src, l, j + h, par))) * g;
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

template <bool FAST, int MAXT>
__global__ __launch_bounds__(MAXT) void k_rows_rho(KParams p,
                                                               const double *__restrict__ f,
                                                               double *__restrict__ rho_out,
                                                               double *__restrict__ mux_out)
{
    extern __shared__ double smem[];
    const int nx = p.nx, ny = p.ny;
    const int y0 = blockIdx.x * p.rows_per_block;
    const int rows = min(p.rows_per_block, ny - y0);
    double *bA = smem, *bB = smem + p.rows_per_block * nx;
    const LineMap<FAST> m{nx, rows, false, false};
    const Elems E = make_elems(m);
    double rr[kElemsPerThread];
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        const size_t node = (size_t)(y0 + E.l[k]) * nx + E.j[k];
        double fi[9];
        load9(f, p.fq, (size_t)(y0 + E.l[k]) * p.fr + E.j[k], fi);
        const double r = sum9(fi);
        rr[k] = r;
        bA[E.e[k]] = r;
        rho_out[node] = r;
        if (p.sc)  // pseudopotential model: the plane holds psi
            mux_out[node] = sc_psi(p, r);
        else if (p.kappa_zero)
            mux_out[node] = p.k2 * mu0_capped(p, r);
    }
    if (p.kappa_zero || p.sc) return;  // uniform: the Laplacian is not used
    __syncthreads();
    double d1[kElemsPerThread], d2[kElemsPerThread];
    double *res = cfm_solve(p, m, E, bA, bB, 1.0, d1);
    cfm_solve(p, m, E, res, res == bA ? bB : bA, -1.0, d2);
    // the row part of the chemical potential, Eq. 33: k^2 psi'(rho) - kappa d2rho/dx2
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        const size_t node = (size_t)(y0 + E.l[k]) * nx + E.j[k];
        mux_out[node] = p.k2 * mu0_capped(p, rr[k]) - p.kappa * d2[k];
    }
}

// Column strip handled by this block.  With col_xcd_groups = 8 the blocks are
// renumbered so that consecutive strips (which share cache lines of every
// row) are dispatched to the same XCD and meet in its L2.
__device__ __forceinline__ int strip_of_block(const KParams &p)
{
    const int b = blockIdx.x, g = p.col_xcd_groups;
    if (g <= 1) return b;
    const int per = gridDim.x / g;
    return (b % g) * per + b / g;
}

template <bool FAST, int MAXT>
__global__ __launch_bounds__(MAXT) void k_cols_mu(KParams p,
                                                              const double *__restrict__ rho,
                                                              const double *__restrict__ mux,
                                                              double *__restrict__ mu_out,
                                                              double *__restrict__ fy_out)
{
    extern __shared__ double smem[];
    const int nx = p.nx, ny = p.ny;
    const int x0 = strip_of_block(p) * p.cols_per_block;
    const int cols = min(p.cols_per_block, nx - x0);
    double *bA = smem, *bB = smem + p.cols_per_block * ny;
    const LineMap<FAST> m{ny, cols, true, p.bc_y != 0};
    const Elems E = make_elems(m);
    if (p.sc) {
        // pseudopotential model: F_y = -G c_s^2 psi d/dy psi with G = -1;
        // psi goes on to the collision pass in the mu plane
        double ps[kElemsPerThread], dps[kElemsPerThread];
#pragma unroll
        for (int k = 0; k < kElemsPerThread; ++k) {
            if (!E.ok[k]) continue;
            const size_t node = (size_t)E.j[k] * nx + x0 + E.l[k];
            ps[k] = mux[node];
            mu_out[node] = ps[k];
            bA[E.e[k]] = ps[k];
        }
        __syncthreads();
        cfm_solve(p, m, E, bA, bB, 1.0, dps);
#pragma unroll
        for (int k = 0; k < kElemsPerThread; ++k) {
            if (!E.ok[k]) continue;
            fy_out[(size_t)E.j[k] * nx + x0 + E.l[k]] = CS2 * ps[k] * dps[k];
        }
        return;
    }
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
        double mu = mux[node];
        if (!p.kappa_zero) mu -= p.kappa * dyy[k];
        mu_out[node] = mu;
        // wetting walls hold mu at mu_wall: mu - mu_wall, extended oddly
        bA[E.e[k]] = p.wet ? mu - p.mu_wall : mu;
    }
    __syncthreads();
    cfm_solve(p, m, E, bA, bB, p.wet ? -1.0 : 1.0, dym);
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        fy_out[(size_t)E.j[k] * nx + x0 + E.l[k]] = -r[k] * dym[k] + CS2 * dyr[k];
    }
}

// KEEP: hold the nine populations of each element in registers between the
// first read and the collision (256-thread blocks); otherwise read them again.
template <bool FAST, int MAXT, bool OBSERVE>
__global__ __launch_bounds__(MAXT) void k_rows_collide(
    KParams p, const double *__restrict__ f, const double *__restrict__ mu,
    const double *__restrict__ fy, double *__restrict__ fout, double *__restrict__ o_rho,
    double *__restrict__ o_vx, double *__restrict__ o_vy, double *__restrict__ o_fx)
{
    extern __shared__ double smem[];
    const int nx = p.nx, ny = p.ny;
    const int y0 = blockIdx.x * p.rows_per_block;
    const int rows = min(p.rows_per_block, ny - y0);
    double *bA = smem, *bB = smem + p.rows_per_block * nx;
    const LineMap<FAST> m{nx, rows, false, false};
    const Elems E = make_elems(m);
    constexpr bool KEEP = MAXT <= 256;
    constexpr int NK = KEEP ? kElemsPerThread : 1;
    double fi[NK][9], rho[kElemsPerThread];
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        double (&q)[9] = fi[KEEP ? k : 0];
        load9(f, p.fq, (size_t)(y0 + E.l[k]) * p.fr + E.j[k], q);
        rho[k] = sum9(q);
        bA[E.e[k]] = rho[k];
    }
    __syncthreads();
    double dxr[kElemsPerThread], dxm[kElemsPerThread], mv[kElemsPerThread];
    if (!p.sc) {
        cfm_solve(p, m, E, bA, bB, 1.0, dxr);
    }
#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        mv[k] = mu[(size_t)(y0 + E.l[k]) * nx + E.j[k]];
        bA[E.e[k]] = mv[k];
    }
    __syncthreads();
    cfm_solve(p, m, E, bA, bB, 1.0, dxm);

#pragma unroll
    for (int k = 0; k < kElemsPerThread; ++k) {
        if (!E.ok[k]) continue;
        const int x = E.j[k], y = y0 + E.l[k];
        const size_t node = (size_t)y * nx + x;
        double (&q)[9] = fi[KEEP ? k : 0];
        if (!KEEP) load9(f, p.fq, (size_t)y * p.fr + x, q);
        const double rh = rho[k];
        const double jx = (q[1] - q[3]) + (q[5] - q[6]) + (q[8] - q[7]);
        const double jy = (q[2] - q[4]) + (q[5] - q[8]) + (q[6] - q[7]);
        // Eq. 12, or the pseudopotential force (mv holds psi)
        const double Fx = p.sc ? CS2 * mv[k] * dxm[k] : -rh * dxm[k] + CS2 * dxr[k];
        const double Fy = fy[node];
        const double ux = jx / rh, uy = jy / rh;
        if (OBSERVE) {
            if (o_rho) o_rho[node] = rh;
            if (o_vx) o_vx[node] = ux + Fx / (2.0 * rh);
            if (o_vy) o_vy[node] = uy + Fy / (2.0 * rh);
            if (o_fx) o_fx[node] = Fx;
            continue;
        }
        const double vx2 = ux + Fx / rh, vy2 = uy + Fy / rh;
        const double uu = ux * ux + uy * uy, uu2 = vx2 * vx2 + vy2 * vy2;
        double dm[6];
        if (p.mrt) mrt_departures(p, q, rh, jx, jy, ux, uy, dm);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double eq = feq(i, rh, ux, uy, uu);
            const double eq2 = feq(i, rh, vx2, vy2, uu2);
            // BGK (Eq. 1) or MRT (Eq. 4), with the exact-difference force (Eq. 5)
            const double fs = p.mrt ? mrt_relax(i, q[i], dm) + (eq2 - eq)
                                    : q[i] - (q[i] - eq) * p.inv_tau + (eq2 - eq);
            int tx = x + EX[i];
            tx = tx < 0 ? tx + nx : (tx >= nx ? tx - nx : tx);
            int ty = y + EY[i];
            if (ty < 0 || ty >= ny) {
                if (p.bc_y) {
                    // half-way bounce-back; a moving wall adds -2 w rho (e.U)/c_s^2
                    const double eu = EX[i] * p.wall_ux;
                    fout[OPP[i] * p.fq + (size_t)y * p.fr + x] = fs - 2.0 * WT[i] * rh * eu / CS2;
                    continue;
                }
                ty = ty < 0 ? ty + ny : ty - ny;
            }
            fout[i * p.fq + (size_t)ty * p.fr + tx] = fs;
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
        const size_t y = n / p.nx, o = y * p.fr + (n - y * p.nx);
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i * p.fq + o] = feq(i, rho, ux, uy, uu);
    }
}

// The three density groups of a state f, in the order the collision pass
// sums them: g0 = (f0 + f1) + f3, g1 = (f2 + f5) + f6, g2 = (f4 + f7) + f8.
__global__ void k_density_groups(KParams p, const double *__restrict__ f, double *__restrict__ g)
{
    const size_t N = (size_t)p.nx * p.ny, F = p.fq, G = p.gq;
    for (size_t n = blockIdx.x * (size_t)blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        const size_t y = n / p.nx, x = n - y * p.nx;
        const double *q = f + y * p.fr + x;
        double *h = g + y * p.gr + x;
        h[0] = (q[0] + q[F]) + q[3 * F];
        h[G] = (q[2 * F] + q[5 * F]) + q[6 * F];
        h[2 * G] = (q[4 * F] + q[7 * F]) + q[8 * F];
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
        const size_t y = n / p.nx;
        load9(f, p.fq, y * p.fr + (n - y * p.nx), fi);
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

}  // namespace

int row_blocks(const KParams &p) { return (p.ny + p.rows_per_block - 1) / p.rows_per_block; }
int col_blocks(const KParams &p) { return (p.nx + p.cols_per_block - 1) / p.cols_per_block; }

static int round_threads(int elems)
{
    int t = (elems + kElemsPerThread - 1) / kElemsPerThread;
    t = (t + 63) / 64 * 64;
    return t < 64 ? 64 : (t > kMaxBlockThreads ? kMaxBlockThreads : t);
}

// Chunks carried by the fast solve for a chunk length: the smallest M with
// |q|^(M lc) < 2^-60, and q^lc.
static void iir_carry(const KParams &p, int lc, int *M, double *qL)
{
    double ql = 1.0;
    for (int k = 0; k < lc; ++k) ql *= p.iir_q;
    int m = 1;
    double t = std::fabs(ql);
    while (t >= 0x1p-60 && m < 64) {
        t *= std::fabs(ql);
        ++m;
    }
    *M = m;
    *qL = ql;
}

void set_row_shape(KParams *p)
{
    iir_carry(*p, kIirRowChunk, &p->iir_m_row, &p->iir_qL_row);
    // one row per block for long rows, else as many whole rows as fill
    // 1024 elements (256 threads)
    const int R = p->nx >= 1024 ? 1 : 1024 / p->nx;
    p->rows_per_block = R;
    p->row_threads = round_threads(R * p->nx);
    p->use_iir_rows = iir_rows_ok(*p);
    // row segments (the segment kernels): kSegLen nodes, the last one ragged;
    // rows longer than one workgroup holds run every row pass over them
    p->seg_len = kSegLen;
    p->row_win = p->nx > kMaxWholeRow;
    p->row_split = p->row_win;
}

void set_col_shape(KParams *p, int width, int chunk)
{
    p->col_win = 0;
    p->col_tile = 0;
    p->col_stream = 0;
    p->col_lc = chunk;
    iir_carry(*p, chunk, &p->iir_m_col, &p->iir_qL_col);
    // the factorised solve holds up to kMaxColElems nodes of a strip (one
    // thread per chunk, at most kMaxBlockThreads); the general reduction
    // kernel kMaxBlockElems
    int w = width < 1 ? 1 : width;
    const bool fast = chunk == 4 || chunk == 8 || chunk == 16;
    int wmax = fast ? kMaxColElems / p->ny : 0;
    if (fast && kMaxBlockThreads * chunk / p->ny < wmax) wmax = kMaxBlockThreads * chunk / p->ny;
    if (wmax >= 1 && iir_cols_ok(*p, chunk, w < wmax ? w : wmax)) {
        w = w < wmax ? w : wmax;
        p->use_iir_cols = 1;
    } else {
        wmax = kMaxBlockElems / p->ny;
        if (wmax < 1) wmax = 1;
        w = w < wmax ? w : wmax;
        p->use_iir_cols = 0;
    }
    p->cols_per_block = w;
    p->col_threads = round_threads(w * p->ny);
    const int nb = col_blocks(*p);
    p->col_xcd_groups = (nb % 8 == 0 && nb >= 64 && p->nx % w == 0) ? 8 : 1;
}

bool set_col_tiles(KParams *p, int width, int chunk)
{
    if (!(width == 4 || width == 8 || width == 16) || !(chunk == 4 || chunk == 8 || chunk == 16))
        return false;
    const int hc = col_tile_chunks(width, chunk), E = col_window_chunks(chunk);
    int M = 0;
    double qL = 0.0;
    iir_carry(*p, chunk, &M, &qL);
    // tiles of at least 8 chunks; the window reaches past one wall only, and
    // more than one tile per column
    if (hc < 8 || p->ny % chunk != 0 || p->ny < 2 * E * chunk || p->ny <= hc * chunk ||
        M > (chunk == 4 ? 11 : (chunk == 8 ? 6 : 3)))
        return false;
    p->col_lc = chunk;
    p->iir_m_col = M;
    p->iir_qL_col = qL;
    p->use_iir_cols = 1;
    p->col_stream = 0;
    p->col_win = 1;
    p->col_tile = hc * chunk;
    p->cols_per_block = width;
    p->col_threads = (width * (hc + 2 * E) + 63) / 64 * 64;
    const int nb = ((p->nx + width - 1) / width) * ((p->ny + p->col_tile - 1) / p->col_tile);
    p->col_xcd_groups = (nb % 8 == 0 && nb >= 64) ? 8 : 1;
    return true;
}

void set_state_layout(KParams *p, bool rows_interleaved)
{
    const size_t nx = p->nx, N = nx * p->ny;
    p->fq = rows_interleaved ? nx : N;
    p->fr = rows_interleaved ? 9 * nx : nx;
    p->gq = rows_interleaved ? nx : N;
    p->gr = rows_interleaved ? 3 * nx : nx;
}

bool set_col_stream(KParams *p, int width)
{
    if (!col_stream_ok(*p, width)) return false;
    const int lc = col_stream_chunk(p->ny);
    int M = 0;
    double qL = 0.0;
    iir_carry(*p, lc, &M, &qL);
    if (M > (lc == 8 ? 6 : 11)) return false;
    p->col_lc = lc;
    p->iir_m_col = M;
    p->iir_qL_col = qL;
    p->use_iir_cols = 1;
    p->col_win = 0;
    p->col_tile = 0;
    p->col_stream = 1;
    p->cols_per_block = width;
    p->col_threads = 512;
    p->col_xcd_groups = 1;
    return true;
}

static size_t row_lds(const KParams &p) { return 2 * sizeof(double) * p.rows_per_block * p.nx; }
static size_t col_lds(const KParams &p) { return 2 * sizeof(double) * p.cols_per_block * p.ny; }
static bool row_fast(const KParams &p) { return p.nx >= kFastMinLine; }
static bool col_fast(const KParams &p) { return p.ny >= kFastMinLine; }

// Launch kernel template K<FAST, MAXT, ...> with the instantiation matching
// the line length (FAST) and block size (MAXT = 256 or 1024).
#define CPLBM_DISPATCH(K, FASTC, THREADS, ...)                                   \
    do {                                                                       \
        if ((FASTC) && (THREADS) <= 256)                                       \
            hipLaunchKernelGGL((K<true, 256 __VA_OPT__(,) __VA_ARGS__>), GRID); \
        else if (FASTC)                                                        \
            hipLaunchKernelGGL((K<true, 1024 __VA_OPT__(,) __VA_ARGS__>), GRID);\
        else if ((THREADS) <= 256)                                             \
            hipLaunchKernelGGL((K<false, 256 __VA_OPT__(,) __VA_ARGS__>), GRID);\
        else                                                                   \
            hipLaunchKernelGGL((K<false, 1024 __VA_OPT__(,) __VA_ARGS__>), GRID);\
    } while (0)

hipError_t launch_rows_rho(const KParams &p, const double *f, const double *g, double *rho,
                           double *mux, hipStream_t s)
{
    if (p.row_win) return launch_rows_rho_seg_iir(p, g, rho, mux, s);
    if (p.use_iir_rows) return launch_rows_rho_iir(p, g, rho, mux, s);
#define GRID dim3(row_blocks(p)), dim3(p.row_threads), row_lds(p), s, p, f, rho, mux
    CPLBM_DISPATCH(k_rows_rho, row_fast(p), p.row_threads);
#undef GRID
    return hipGetLastError();
}

hipError_t launch_cols_mu(const KParams &p, const double *rho, const double *mux, double *mu,
                          double *fy, hipStream_t s)
{
    if (p.use_iir_cols) return launch_cols_mu_iir(p, rho, mux, mu, fy, s);
#define GRID dim3(col_blocks(p)), dim3(p.col_threads), col_lds(p), s, p, rho, mux, mu, fy
    CPLBM_DISPATCH(k_cols_mu, col_fast(p), p.col_threads);
#undef GRID
    return hipGetLastError();
}

hipError_t launch_rows_collide(const KParams &p, const double *f, const double *mu,
                               const double *fy, double *fout, double *gout, const double *rho,
                               hipStream_t s)
{
    if (p.row_split) return launch_collide_split_iir(p, f, rho, mu, fy, fout, gout, s);
    if (p.use_iir_rows)
        return launch_rows_collide_iir(p, f, mu, fy, fout, gout, nullptr, nullptr, nullptr,
                                       nullptr, false, s);
#define GRID                                                                                 \
    dim3(row_blocks(p)), dim3(p.row_threads), row_lds(p), s, p, f, mu, fy, fout, nullptr,    \
        nullptr, nullptr, nullptr
    CPLBM_DISPATCH(k_rows_collide, row_fast(p), p.row_threads, false);
#undef GRID
    return hipGetLastError();
}

hipError_t launch_rows_observe(const KParams &p, const double *f, const double *mu,
                               const double *fy, const double *rho_in, double *rho, double *vx,
                               double *vy, double *fx, hipStream_t s)
{
    if (p.row_win) return launch_observe_seg_iir(p, f, rho_in, mu, fy, rho, vx, vy, fx, s);
    if (p.use_iir_rows)
        return launch_rows_collide_iir(p, f, mu, fy, nullptr, nullptr, rho, vx, vy, fx, true, s);
#define GRID                                                                                 \
    dim3(row_blocks(p)), dim3(p.row_threads), row_lds(p), s, p, f, mu, fy, nullptr, rho, vx, \
        vy, fx
    CPLBM_DISPATCH(k_rows_collide, row_fast(p), p.row_threads, true);
#undef GRID
    return hipGetLastError();
}

// u = v - F / (2 rho): the bare velocity whose equilibrium carries the fluid
// velocity v under the force F (Sec. 2, the half-force shift of Eq. 5).
__global__ void k_bare_velocity(size_t N, const double *__restrict__ rho,
                                const double *__restrict__ fx, const double *__restrict__ fy,
                                double *__restrict__ ux, double *__restrict__ uy)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < N;
         i += (size_t)gridDim.x * blockDim.x) {
        const double h = 0.5 / rho[i];
        ux[i] -= h * fx[i];
        uy[i] -= h * fy[i];
    }
}

hipError_t launch_bare_velocity(const KParams &p, const double *rho, const double *fx,
                                const double *fy, double *ux, double *uy, hipStream_t s)
{
    const size_t N = (size_t)p.nx * p.ny;
    int blocks = (int)((N + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_bare_velocity, dim3(blocks), dim3(256), 0, s, N, rho, fx, fy, ux, uy);
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

hipError_t launch_density_groups(const KParams &p, const double *f, double *g, hipStream_t s)
{
    const size_t N = (size_t)p.nx * p.ny;
    int blocks = (int)((N + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_density_groups, dim3(blocks), dim3(256), 0, s, p, f, g);
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
