// Time-step kernels whose compact-scheme solves use the factorised inverse of
// the circulant tridiagonal matrix (the fast path; kernels.hip holds the
// general parallel-cyclic-reduction path used for short or ragged lines).
//
// Eq. 37 on a periodic line is C d = r with C = I + al (S + S^-1).  Writing
// C = (1 + 2 al q)^-1 (I - q S)(I - q S^-1) / ... one finds, on an infinite
// line, (C^-1)_ij = K q^|i-j| with q = (-1 + sqrt(1 - 4 al^2)) / (2 al) and
// K = 1 / (1 + 2 al q); |q| = 0.382 (al = 1/3) or 0.268 (al = 1/4).  Hence
//     d_i = K (y_i + z_i),  y_i = r_i + q y_{i-1},  z_i = q (r_{i+1} + z_{i+1}),
// a causal and an anti-causal first-order recurrence.  On a periodic line of
// n >= 64 nodes the wrap-around terms of the exact periodic inverse carry a
// factor q^n < 1e-26 and are absorbed in the same recurrences run cyclically.
//
// Each thread owns LC consecutive nodes of one line (a chunk).  It runs both
// recurrences over its chunk from zero, publishes the two partial sums
//     P_c = sum_{m<LC} q^m r_{last-m},   B_c = sum_{m<LC} q^(m+1) r_{first+m},
// and then adds the contributions of the M chunks before and after it,
//     y_k += q^(k+1) sum_{m=1..M} q^((m-1)LC) P_{c-m},
//     z_k += q^(LC-1-k) sum_{m=1..M} q^((m-1)LC) B_{c+m},
// with M = kCarry(LC) chunks, enough that |q|^(M LC) < 2^-60 for either
// scheme.  Two barriers per solve.  Between walls the column is the even
// extension of length 2 ny: a chunk beyond a wall is the mirror image of a
// physical chunk, whose P and B swap roles (P of the image of chunk i is
// par B_i / q, B of the image is par q P_i, par being the parity of the
// right-hand side).  Ghost slots in LDS hold these images (and the periodic
// ones), so the solve reads neighbours without tests (see Chunk).
#include "kernels.hpp"
#include "physics.hpp"

namespace cplbm {

namespace {

using namespace phys;

// Chunks carried on each side by the solve for chunk length lc: the weight
// of the next chunk, |q|^(M lc), is below 2^-60 for both compact schemes
// (alpha = 1/3 has the larger pole, |q| = 0.382, and sets M).
constexpr int kCarry(int lc) { return lc == 4 ? 11 : (lc == 8 ? 6 : 3); }

// The thread's chunk within the block's lines, and the LDS layout of a
// block's line solves:
//   edges   4 (nc + 2) per line: each chunk's first two and last two values
//           (all the right-hand side needs of a neighbour), with a ghost
//           chunk before the first and after the last;
//   cP, cB  nc + kCarry(LC) per line: one carry per chunk, with kCarry ghost
//           chunks before the first (cP) or after the last (cB).
// The ghosts hold the periodic images, or at walls the reflected values, so
// the solve reads its neighbours without wrapping or testing indices.
// Column layout (col): slot (index + offset) * nl + l; row layout: line l
// contiguous.
template <int LC>
struct Chunk {
    static constexpr int MC = kCarry(LC);
    int n;      // line length
    int nc;     // chunks per line (n / LC)
    int nl;     // lines held by the block (row or column count of the layout)
    bool col;
    bool mirror;
    int l, c;   // this thread's line and chunk
    bool ok;    // the line exists (ragged last block)
    // edge value e of chunk ci in [-1, nc]: e = 0, 1 its first two nodes,
    // e = 2, 3 its last two
    __device__ __forceinline__ int eslot(int ci, int e) const
    {
        return col ? ((ci + 1) * 4 + e) * nl + l : l * 4 * (nc + 2) + (ci + 1) * 4 + e;
    }
    // cP of chunk ci in [-MC, nc), cB of chunk ci in [0, nc + MC)
    __device__ __forceinline__ int pslot(int ci) const
    {
        return col ? (ci + MC) * nl + l : l * (nc + MC) + ci + MC;
    }
    __device__ __forceinline__ int bslot(int ci) const
    {
        return col ? ci * nl + l : l * (nc + MC) + ci;
    }
};

// The block's LDS carved for the line solves (and the collision pass's edge
// exchange: six planes of one slot per chunk, after the carries).
struct LineLds {
    double *vbuf, *cP, *cB, *edge;
};
template <int LC>
__device__ __forceinline__ LineLds carve_lds(double *smem, const Chunk<LC> &m)
{
    LineLds L;
    L.vbuf = smem;
    L.cP = smem + (size_t)m.nl * 4 * (m.nc + 2);
    L.cB = L.cP + (size_t)m.nl * (m.nc + Chunk<LC>::MC);
    L.edge = L.cB + (size_t)m.nl * (m.nc + Chunk<LC>::MC);
    return L;
}

// A chunk's part of a solve: the right-hand side of Eq. 37 from its values u
// and the two values on each side, both recurrences from zero over the
// chunk, and the two carries it publishes.
template <int LC>
__device__ __forceinline__ void iir_chunk(const KParams &p, const double (&u)[LC], double um2,
                                          double um1, double up0, double up1, double (&y)[LC],
                                          double (&z)[LC], double &Pc, double &Bc)
{
    const double q = p.iir_q;
    double r[LC];
    auto U = [&](int i) -> double {
        return i == -2 ? um2 : i == -1 ? um1 : i == LC ? up0 : i == LC + 1 ? up1 : u[i];
    };
#pragma unroll
    for (int k = 0; k < LC; ++k)
        r[k] = p.cfd_a2 * (U(k + 1) - U(k - 1)) + p.cfd_b4 * (U(k + 2) - U(k - 2));
    y[0] = r[0];
#pragma unroll
    for (int k = 1; k < LC; ++k) y[k] = r[k] + q * y[k - 1];
    z[LC - 1] = 0.0;
#pragma unroll
    for (int k = LC - 2; k >= 0; --k) z[k] = q * (r[k + 1] + z[k + 1]);
    Pc = y[LC - 1];
    Bc = q * (r[0] + z[0]);
}

// The derivative on a chunk: its own recurrences plus the sums Yc and Zc
// carried in from the chunks before and after it.
template <int LC>
__device__ __forceinline__ void iir_combine(const KParams &p, double Yc, double Zc,
                                            const double (&y)[LC], const double (&z)[LC],
                                            double (&d)[LC])
{
#pragma unroll
    for (int k = 0; k < LC; ++k)
        d[k] = p.iir_K * ((y[k] + p.iir_qp[k + 1] * Yc) + (z[k] + p.iir_qp[LC - 1 - k] * Zc));
}

// First derivative of u (parity par_u) along the thread's line; the whole
// block calls it together.
template <int LC>
__device__ __forceinline__ void iir_solve(const KParams &p, const Chunk<LC> &m, double qL,
                                          const double (&u)[LC], double par_u, const LineLds &L,
                                          double (&d)[LC])
{
    constexpr int MC = Chunk<LC>::MC;
    double *vbuf = L.vbuf, *cP = L.cP, *cB = L.cB;
    const int c = m.c, nc = m.nc;
    if (m.ok) {
        vbuf[m.eslot(c, 0)] = u[0];
        vbuf[m.eslot(c, 1)] = u[1];
        vbuf[m.eslot(c, 2)] = u[LC - 2];
        vbuf[m.eslot(c, 3)] = u[LC - 1];
        // ghost chunks: periodic images, or the even (par_u = 1) or odd
        // (par_u = -1) reflection about the wall half a node past the end
        if (c == 0) {
            if (m.mirror) {
                vbuf[m.eslot(-1, 2)] = par_u * u[1];
                vbuf[m.eslot(-1, 3)] = par_u * u[0];
            } else {
                vbuf[m.eslot(nc, 0)] = u[0];
                vbuf[m.eslot(nc, 1)] = u[1];
            }
        }
        if (c == nc - 1) {
            if (m.mirror) {
                vbuf[m.eslot(nc, 0)] = par_u * u[LC - 1];
                vbuf[m.eslot(nc, 1)] = par_u * u[LC - 2];
            } else {
                vbuf[m.eslot(-1, 2)] = u[LC - 2];
                vbuf[m.eslot(-1, 3)] = u[LC - 1];
            }
        }
    }
    __syncthreads();
    const double q = p.iir_q;
    double y[LC], z[LC];
    if (m.ok) {
        // u at j0-2, j0-1 (end of the previous chunk), j0+LC, j0+LC+1 (start
        // of the next)
        double Pc, Bc;
        iir_chunk<LC>(p, u, vbuf[m.eslot(c - 1, 2)], vbuf[m.eslot(c - 1, 3)],
                      vbuf[m.eslot(c + 1, 0)], vbuf[m.eslot(c + 1, 1)], y, z, Pc, Bc);
        cP[m.pslot(m.c)] = Pc;
        cB[m.bslot(m.c)] = Bc;
        // ghost chunks: periodic images, or at walls the carries of the
        // reflected line (parity -par_u), which run the other way
        if (m.mirror) {
            const double par_r = -par_u;
            if (m.c < MC) cP[m.pslot(-1 - m.c)] = par_r * p.iir_inv_q * Bc;
            if (m.c >= nc - MC) cB[m.bslot(2 * nc - 1 - m.c)] = par_r * q * Pc;
        } else {
            if (m.c >= nc - MC) cP[m.pslot(m.c - nc)] = Pc;
            if (m.c < MC) cB[m.bslot(m.c + nc)] = Bc;
        }
    }
    __syncthreads();
    if (!m.ok) return;
    // the MC chunks on each side, nearest last (Horner in q^LC)
    double Yc = 0.0, Zc = 0.0;
#pragma unroll
    for (int mm = MC; mm >= 1; --mm) {
        Yc = Yc * qL + cP[m.pslot(m.c - mm)];
        Zc = Zc * qL + cB[m.bslot(m.c + mm)];
    }
    iir_combine<LC>(p, Yc, Zc, y, z, d);
}

// The same solve on a window of nw consecutive chunks w = 0 .. nw - 1 of a
// line, which the caller loads (x periodic; a column periodic or mirrored
// about its walls): every chunk publishes its edge values and (w in
// [1, nw - 1)) its carries, and the chunks w in [MC + 1, nw - MC - 1) receive
// the derivative.  Those chunks sum the carries of exactly the MC chunks on
// each side that the whole-line solve sums, computed from the same values,
// so their derivative is the whole-line one (bitwise for rows).  The block
// holds nl such windows side by side (line l of them, interleaved in LDS so
// that neighbouring lines sit in neighbouring banks); the whole block calls
// it together.
template <int LC>
__device__ __forceinline__ void iir_solve_window(const KParams &p, int w, int nw, double qL,
                                                 const double (&u)[LC], double *vbuf, double *cP,
                                                 double *cB, double (&d)[LC], int l = 0,
                                                 int nl = 1)
{
    constexpr int MC = kCarry(LC);
    auto E = [&](int ci, int e) { return (4 * ci + e) * nl + l; };
    if (w < nw) {
        vbuf[E(w, 0)] = u[0];
        vbuf[E(w, 1)] = u[1];
        vbuf[E(w, 2)] = u[LC - 2];
        vbuf[E(w, 3)] = u[LC - 1];
    }
    __syncthreads();
    double y[LC], z[LC];
    if (w >= 1 && w < nw - 1) {
        double Pc, Bc;
        iir_chunk<LC>(p, u, vbuf[E(w - 1, 2)], vbuf[E(w - 1, 3)], vbuf[E(w + 1, 0)],
                      vbuf[E(w + 1, 1)], y, z, Pc, Bc);
        cP[w * nl + l] = Pc;
        cB[w * nl + l] = Bc;
    }
    __syncthreads();
    if (w < MC + 1 || w >= nw - MC - 1) return;
    double Yc = 0.0, Zc = 0.0;
#pragma unroll
    for (int mm = MC; mm >= 1; --mm) {
        Yc = Yc * qL + cP[(w - mm) * nl + l];
        Zc = Zc * qL + cB[(w + mm) * nl + l];
    }
    iir_combine<LC>(p, Yc, Zc, y, z, d);
}

// 16-byte vector access to LC consecutive doubles (32-byte aligned).
template <int LC>
__device__ __forceinline__ void vload(const double *__restrict__ src, double (&v)[LC])
{
#pragma unroll
    for (int k = 0; k < LC; k += 2) {
        const double2 t = *reinterpret_cast<const double2 *>(src + k);
        v[k] = t.x;
        v[k + 1] = t.y;
    }
}

template <int LC>
__device__ __forceinline__ void vstore(double *__restrict__ dst, const double (&v)[LC])
{
#pragma unroll
    for (int k = 0; k < LC; k += 2) *reinterpret_cast<double2 *>(dst + k) = make_double2(v[k], v[k + 1]);
}

// Row chunk of this thread: rows_per_block lines of nx, nc = nx / LC chunks each.
template <int LC>
__device__ __forceinline__ Chunk<LC> row_chunk(const KParams &p, int rows)
{
    Chunk<LC> m;
    m.n = p.nx;
    m.nc = p.nx / LC;
    m.nl = p.rows_per_block;
    m.col = false;
    m.mirror = false;
    m.l = threadIdx.x / m.nc;
    m.c = threadIdx.x - m.l * m.nc;
    m.ok = m.l < rows;
    return m;
}

constexpr int kRowLC = 4;

// A row segment's window reaches kSegWin chunks past each end of the
// segment in the collision pass: the chunk beyond each end, whose collision
// gives the populations the end nodes receive; the MC chunks whose carries
// that chunk's derivative sums; and one more, whose edge values the
// outermost carry needs.  Pass A chains two derivatives, so its window
// reaches kRhoWin chunks.
constexpr int kSegWin = kCarry(kRowLC) + 2;
constexpr int kRhoWin = 2 * (kCarry(kRowLC) + 1);
// pass A's segments: 208 chunks, which with its window's 48 fill a
// 256-thread workgroup
constexpr int kRhoSegLen = 832;
// threads of a segment workgroup: the window's chunks, in whole waves
constexpr int kSegThreads = ((kSegLen / kRowLC + 2 * kSegWin) + 63) / 64 * 64;
constexpr int kRhoThreads = ((kRhoSegLen / kRowLC + 2 * kRhoWin) + 63) / 64 * 64;

// Segments of len nodes in a row: ceil(nx / len), the last one ragged (a
// whole number of chunks, as nx is).
__device__ __forceinline__ int row_segments(const KParams &p, int len)
{
    return (p.nx + len - 1) / len;
}

// Segment chunk of this thread: thread t holds chunk t - kSegWin of a
// segment of seg_n nodes of one row; ok marks the chunks that collide, the
// segment's own and the one beyond each end.
template <int LC>
__device__ __forceinline__ Chunk<LC> seg_chunk(const KParams &p, int seg_n)
{
    Chunk<LC> m;
    m.n = seg_n;
    m.nc = seg_n / LC;
    m.nl = 1;
    m.col = false;
    m.mirror = false;
    m.l = 0;
    m.c = (int)threadIdx.x - kSegWin;
    m.ok = m.c >= -1 && m.c <= m.nc;
    return m;
}

// Pass A on rows [y0, y0 + rows_per_block) of one mesh: rho, and the row part
// of the chemical potential of Eq. 33, k^2 psi'(rho) - kappa d2rho/dx2.
// rho comes from the state's three density groups g (written by the previous
// collision pass): rho = (g0 + g1) + g2.  SC: the pseudopotential model,
// whose plane holds psi instead (a template argument, so that the
// chemical-potential kernel carries none of its arithmetic).
template <bool SC = false>
__device__ __forceinline__ void rows_rho_body(const KParams &p, int y0, const double *__restrict__ g,
                                              double *__restrict__ rho_out,
                                              double *__restrict__ mux_out)
{
    constexpr int LC = kRowLC;
    extern __shared__ double smem[];
    const int nx = p.nx, ny = p.ny;
    const int rows = min(p.rows_per_block, ny - y0);
    const Chunk<LC> m = row_chunk<LC>(p, rows);
    const LineLds L = carve_lds(smem, m);
    const size_t base = (size_t)(y0 + m.l) * nx + m.c * LC;
    const size_t gb = (size_t)(y0 + m.l) * p.gr + m.c * LC;
    double rho[LC];
    if (m.ok) {
        double g0[LC], g1[LC], g2[LC];
        vload<LC>(g + gb, g0);
        vload<LC>(g + p.gq + gb, g1);
        vload<LC>(g + 2 * p.gq + gb, g2);
#pragma unroll
        for (int k = 0; k < LC; ++k) rho[k] = (g0[k] + g1[k]) + g2[k];
        vstore<LC>(rho_out + base, rho);
    }
    // bulk part first: its transcendental work overlaps the solves' barriers
    double mx[LC];
    if (m.ok) {
#pragma unroll
        for (int k = 0; k < LC; ++k)
            mx[k] = SC ? sc_psi(p, rho[k]) : p.k2 * mu0_capped(p, rho[k]);
    }
    // uniform: the Laplacian is not used (kappa = 0), or the pseudopotential
    // model, whose plane holds psi
    if (p.kappa_zero || SC) {
        if (m.ok) vstore<LC>(mux_out + base, mx);
        return;
    }
    double d1[LC], d2[LC];
    iir_solve<LC>(p, m, p.iir_qL_row, rho, 1.0, L, d1);
    iir_solve<LC>(p, m, p.iir_qL_row, d1, -1.0, L, d2);
    if (m.ok) {
#pragma unroll
        for (int k = 0; k < LC; ++k) mx[k] -= p.kappa * d2[k];
        vstore<LC>(mux_out + base, mx);
    }
}

template <int MAXT, bool SC>
__global__ __launch_bounds__(MAXT) void k_rows_rho_iir(KParams p, const double *__restrict__ g,
                                                       double *__restrict__ rho_out,
                                                       double *__restrict__ mux_out)
{
    rows_rho_body<SC>(p, blockIdx.x * p.rows_per_block, g, rho_out, mux_out);
}

__device__ __forceinline__ int strip_of_block(const KParams &p)
{
    const int b = blockIdx.x, g = p.col_xcd_groups;
    if (g <= 1) return b;
    const int per = gridDim.x / g;
    return (b % g) * per + b / g;
}

// Pass B on columns [x0, x0 + cols_per_block) of one mesh.  Threads beyond
// the strip's chunks (a batch launch sized for the largest strip) only take
// part in the barriers.
template <int LC>
__device__ __forceinline__ void cols_mu_body(const KParams &p, int x0,
                                             const double *__restrict__ rho,
                                             const double *__restrict__ mux,
                                             double *__restrict__ mu_out,
                                             double *__restrict__ fy_out)
{
    extern __shared__ double smem[];
    const int nx = p.nx, ny = p.ny, W = p.cols_per_block;
    const int cols = min(W, nx - x0);
    Chunk<LC> m;
    m.n = ny;
    m.nc = ny / LC;
    m.nl = W;
    m.col = true;
    m.mirror = p.bc_y != 0;
    m.c = threadIdx.x / W;
    m.l = threadIdx.x - m.c * W;
    m.ok = m.l < cols && m.c < m.nc;
    const LineLds L = carve_lds(smem, m);
    const size_t col = x0 + m.l;
    const int j0 = m.c * LC;
    if (p.sc) {
        // pseudopotential model: F_y = -G c_s^2 psi d/dy psi with G = -1; psi
        // is passed on to the collision pass in the mu plane
        double ps[LC], dps[LC];
        if (m.ok) {
#pragma unroll
            for (int k = 0; k < LC; ++k) {
                const size_t node = (size_t)(j0 + k) * nx + col;
                ps[k] = mux[node];
                mu_out[node] = ps[k];
            }
        }
        iir_solve<LC>(p, m, p.iir_qL_col, ps, 1.0, L, dps);
        if (m.ok) {
#pragma unroll
            for (int k = 0; k < LC; ++k)
                fy_out[(size_t)(j0 + k) * nx + col] = CS2 * ps[k] * dps[k];
        }
        return;
    }
    // With chunks of 8 or more nodes (one 1024-thread workgroup per CU at
    // most) both inputs are loaded up front, so that their latencies
    // overlap; 4-node chunks keep the registers for two workgroups per CU
    // and load the row part of mu after the solves.
    constexpr bool kEarly = LC >= 8;
    double r[LC], mx[LC];
    if (m.ok) {
#pragma unroll
        for (int k = 0; k < LC; ++k) r[k] = rho[(size_t)(j0 + k) * nx + col];
        if (kEarly) {
#pragma unroll
            for (int k = 0; k < LC; ++k) mx[k] = mux[(size_t)(j0 + k) * nx + col];
        }
    }
    double dyr[LC], dyy[LC], mu[LC], dym[LC];
    iir_solve<LC>(p, m, p.iir_qL_col, r, 1.0, L, dyr);
    if (!p.kappa_zero) iir_solve<LC>(p, m, p.iir_qL_col, dyr, -1.0, L, dyy);
    if (m.ok) {
#pragma unroll
        for (int k = 0; k < LC; ++k) {
            const size_t node = (size_t)(j0 + k) * nx + col;
            double v = kEarly ? mx[k] : mux[node];
            if (!p.kappa_zero) v -= p.kappa * dyy[k];
            mu[k] = v;
            mu_out[node] = v;
        }
    }
    if (p.wet) {
        // wetting walls hold mu at mu_wall: differentiate mu - mu_wall on its
        // odd extension about the walls
        double mw[LC];
#pragma unroll
        for (int k = 0; k < LC; ++k) mw[k] = mu[k] - p.mu_wall;
        iir_solve<LC>(p, m, p.iir_qL_col, mw, -1.0, L, dym);
    } else {
        iir_solve<LC>(p, m, p.iir_qL_col, mu, 1.0, L, dym);
    }
    if (m.ok) {
#pragma unroll
        for (int k = 0; k < LC; ++k)
            fy_out[(size_t)(j0 + k) * nx + col] = -r[k] * dym[k] + CS2 * dyr[k];
    }
}

template <int LC, int MAXT>
__global__ __launch_bounds__(MAXT) void k_cols_mu_iir(KParams p, const double *__restrict__ rho,
                                                      const double *__restrict__ mux,
                                                      double *__restrict__ mu_out,
                                                      double *__restrict__ fy_out)
{
    cols_mu_body<LC>(p, strip_of_block(p) * p.cols_per_block, rho, mux, mu_out, fy_out);
}

// Pass B over a tile of col_tile rows of columns [x0, x0 + cols_per_block),
// with a window of kColWin chunks above and below it: each of the three
// chained derivatives needs MC + 1 chunks of the previous one's values past
// the chunks it serves, so the window holds three times that, and the tile's
// derivatives are the whole-column values to round-off.  Beyond a wall the
// window holds the column's mirror image: rho and the row part of mu are
// even about the wall, so their derivatives come out odd and even as the
// whole-column solve's ghost chunks make them, and for wetting walls
// mu - mu_wall is odd (its sign flips beyond the wall).  Columns of any
// length run in tiles of one width.
template <int LC>
constexpr int kColWin = 3 * (kCarry(LC) + 1);

template <int LC>
__device__ __forceinline__ void cols_mu_win_body(const KParams &p, int x0, int ty,
                                                 const double *__restrict__ rho,
                                                 const double *__restrict__ mux,
                                                 double *__restrict__ mu_out,
                                                 double *__restrict__ fy_out)
{
    constexpr int E = kColWin<LC>;
    extern __shared__ double smem[];
    const int nx = p.nx, ny = p.ny, W = p.cols_per_block;
    const int y0 = ty * p.col_tile, hc = min(p.col_tile, ny - y0) / LC, nw = hc + 2 * E;
    const int w = threadIdx.x / W, l = threadIdx.x - w * W, c = w - E;
    const int col = x0 + l;
    const bool in = w < nw && col < nx;
    const bool core = in && c >= 0 && c < hc;
    // the chunk's rows; chunks never straddle a wall (ny and the tiles are
    // whole chunks)
    const int yc = y0 + c * LC;
    const bool beyond = p.bc_y && (yc < 0 || yc >= ny);
    auto row_of = [&](int y) -> size_t {
        if (p.bc_y) y = y < 0 ? -1 - y : (y >= ny ? 2 * ny - 1 - y : y);
        else y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
        return (size_t)y * nx + col;
    };
    double *vbuf = smem, *cP = smem + 4 * nw * W, *cB = cP + nw * W;
    double r[LC], mx[LC];
    if (in) {
#pragma unroll
        for (int k = 0; k < LC; ++k) {
            const size_t node = row_of(yc + k);
            r[k] = rho[node];
            mx[k] = mux[node];
        }
    }
    const double qL = p.iir_qL_col;
    if (p.sc) {
        // pseudopotential model: F_y = c_s^2 psi d/dy psi; psi (even about
        // a wall) is passed on in the mu plane
        double dps[LC];
        iir_solve_window<LC>(p, w, nw, qL, mx, vbuf, cP, cB, dps, l, W);
        if (core) {
#pragma unroll
            for (int k = 0; k < LC; ++k) {
                const size_t node = (size_t)(yc + k) * nx + col;
                mu_out[node] = mx[k];
                fy_out[node] = CS2 * mx[k] * dps[k];
            }
        }
        return;
    }
    double dyr[LC], dyy[LC], mu[LC], dym[LC];
#pragma unroll
    for (int k = 0; k < LC; ++k) dyr[k] = dyy[k] = 0.0;
    iir_solve_window<LC>(p, w, nw, qL, r, vbuf, cP, cB, dyr, l, W);
    if (!p.kappa_zero) iir_solve_window<LC>(p, w, nw, qL, dyr, vbuf, cP, cB, dyy, l, W);
#pragma unroll
    for (int k = 0; k < LC; ++k) {
        double v = mx[k];
        if (!p.kappa_zero) v -= p.kappa * dyy[k];
        mu[k] = v;
    }
    if (p.wet) {
        double mw[LC];
        const double sg = beyond ? -1.0 : 1.0;
#pragma unroll
        for (int k = 0; k < LC; ++k) mw[k] = sg * (mu[k] - p.mu_wall);
        iir_solve_window<LC>(p, w, nw, qL, mw, vbuf, cP, cB, dym, l, W);
    } else {
        iir_solve_window<LC>(p, w, nw, qL, mu, vbuf, cP, cB, dym, l, W);
    }
    if (core) {
#pragma unroll
        for (int k = 0; k < LC; ++k) {
            const size_t node = (size_t)(yc + k) * nx + col;
            mu_out[node] = mu[k];
            fy_out[node] = -r[k] * dym[k] + CS2 * dyr[k];
        }
    }
}

// One workgroup per (strip, tile); the permuted block index keeps the tiles
// of one strip, and neighbouring strips, on one XCD.
template <int LC>
__global__ __launch_bounds__(1024) void k_cols_mu_win(KParams p, const double *__restrict__ rho,
                                                      const double *__restrict__ mux,
                                                      double *__restrict__ mu_out,
                                                      double *__restrict__ fy_out)
{
    const int nt = (p.ny + p.col_tile - 1) / p.col_tile;
    const int idx = strip_of_block(p), strip = idx / nt;
    cols_mu_win_body<LC>(p, strip * p.cols_per_block, idx - strip * nt, rho, mux, mu_out,
                         fy_out);
}

// ---- pass B streamed down strips of whole cache lines ------------------
// A workgroup takes a strip of SW columns (SW = 16: one 128-byte line of each
// row of a plane) and walks down it in tiles of ST chunks of LC rows, each of
// its SW * ST threads holding one chunk of one column.  The three chained
// solves of the pass (d/dy rho; d2/dy2 rho and so mu; d/dy mu and so F_y) run
// as a pipeline one tile apart: step s loads the densities of tile s + 1 and
// finishes the first solve on tile s - 1, the second on tile s - 2 and the
// third on tile s - 3.  A solve on a tile sums the causal carries of the MC
// chunks before it, which a ring in LDS keeps from the step before, and the
// anti-causal carries of the MC chunks after it, which the threads compute
// from the next tile's values (the previous solve's output of the same
// step).  Between walls each solve closes at the walls as the whole-column
// solve does, with the mirror image's edge values and carries; a periodic
// column is one window from kColWin chunks above its first row to kColWin
// chunks below its last, wrapped, as for the tiles above, so each solve is
// the window solve of iir_solve_window on that window.  Either way the stored
// values are the whole-column ones to round-off.  Every value of a plane is
// read once (besides a periodic column's two windows), in whole lines, where
// strips of whole columns read a quarter of a line per row.  512 threads: the
// carried tiles take ~240 registers with 8-node chunks, and a 1024-thread
// workgroup would spill.
template <int SW, int ST, int LC>
struct StreamLds {
    static constexpr int MC = kCarry(LC);
    static constexpr int R = 2 * ST;        // causal carries kept per solve (chunks)
    static constexpr int NE = ST + MC + 2;  // edge slots: see stream_solve
    static_assert(ST > MC, "the next tile must hold the chunks whose carries a tile sums");
    static_assert((R & (R - 1)) == 0, "the carry ring is indexed with a mask");
    // edges, three carry rings, anti-causal carries, the left buffers of the
    // three solves, and the look-ahead chunks' causal carries
    static constexpr int doubles =
        NE * 4 * SW + 3 * R * SW + (ST + MC) * SW + 3 * 4 * SW + MC * SW;
};

// Solve k (0, 1, 2) of step s: the derivative d of the thread's chunk of the
// solve's current tile (s - 1 - k) from its values u, with un the thread's
// chunk of the next tile.  Edge slots: 0 the previous tile's last chunk (kept
// in `left` from the step before), 1 + c the current tile's chunk c, ST + 1 + c
// the next tile's chunk c (c <= MC).  Between walls (wall) the chunks are the
// column's own nc chunks, and the chunks next to a wall take the edge values
// and the carries of the chunks beyond it from the mirror image of u (parity
// par), as the whole-column solve's ghost chunks do: the carry of the image
// of chunk i is -par B_i / q before the first wall and -par q P_i after the
// last (lookP holds the next tile's P for images that fall there).  The whole
// block calls it together.
template <int SW, int ST, int LC>
__device__ __forceinline__ void stream_solve(const KParams &p, int k, int s, int c, int l, int nc,
                                             bool wall, double par, const double (&u)[LC],
                                             const double (&un)[LC], double *edge,
                                             double *cPr, double *cB, double *left,
                                             double *lookP, double (&d)[LC])
{
    constexpr int MC = StreamLds<SW, ST, LC>::MC, R = StreamLds<SW, ST, LC>::R;
    auto ES = [&](int slot, int e) { return (slot * 4 + e) * SW + l; };
    auto EI = [](int e) { return e < 2 ? e : LC - 4 + e; };
#pragma unroll
    for (int e = 0; e < 4; ++e) edge[ES(1 + c, e)] = u[EI(e)];
    if (c <= MC) {
#pragma unroll
        for (int e = 0; e < 4; ++e) edge[ES(ST + 1 + c, e)] = un[EI(e)];
    }
    double *lk = left + k * 4 * SW;  // two buffers of the last two values
    if (c == 0) {
        edge[ES(0, 2)] = lk[((s & 1) * 2) * SW + l];
        edge[ES(0, 3)] = lk[((s & 1) * 2 + 1) * SW + l];
    }
    if (c == ST - 1) {
        lk[(((s + 1) & 1) * 2) * SW + l] = u[LC - 2];
        lk[(((s + 1) & 1) * 2 + 1) * SW + l] = u[LC - 1];
    }
    __syncthreads();
    const int t = s - 1 - k;
    const int g = t * ST + c;  // the chunk's index along the column (or window)
    double *cPk = cPr + k * R * SW;
    // the chunk's own recurrences enter the derivative only as y + z
    double w[LC], Pc, Bc;
    {
        double um2 = edge[ES(c, 2)], um1 = edge[ES(c, 3)], up0 = edge[ES(c + 2, 0)],
               up1 = edge[ES(c + 2, 1)];
        if (wall && g == 0) {
            um2 = par * u[1];
            um1 = par * u[0];
        }
        if (wall && g == nc - 1) {
            up0 = par * u[LC - 1];
            up1 = par * u[LC - 2];
        }
        double y[LC], z[LC];
        iir_chunk<LC>(p, u, um2, um1, up0, up1, y, z, Pc, Bc);
#pragma unroll
        for (int j = 0; j < LC; ++j) w[j] = y[j] + z[j];
    }
    // ring slot of chunk i: (i + 4 R) & (R - 1), positive in the first steps
    // (whose tiles lie before the column)
    cPk[((g + 4 * R) & (R - 1)) * SW + l] = Pc;
    cB[c * SW + l] = Bc;
    if (c < MC) {
        // the carries of the next tile's chunk c
        double vp0 = edge[ES(ST + 2 + c, 0)], vp1 = edge[ES(ST + 2 + c, 1)];
        if (wall && g + ST == nc - 1) {
            vp0 = par * un[LC - 1];
            vp1 = par * un[LC - 2];
        }
        double y2[LC], z2[LC], P2, B2;
        iir_chunk<LC>(p, un, edge[ES(ST + c, 2)], edge[ES(ST + c, 3)], vp0, vp1, y2, z2, P2, B2);
        cB[(ST + c) * SW + l] = B2;
        lookP[c * SW + l] = P2;
    }
    __syncthreads();
    const double qL = p.iir_qL_col;
    double Yc = 0.0, Zc = 0.0;
    // only the first tile and the tiles within MC chunks of the last wall
    // meet images (the same for the whole block)
    if (!wall || (t > 0 && (t + 1) * ST + MC <= nc)) {
#pragma unroll
        for (int mm = MC; mm >= 1; --mm) {
            Yc = Yc * qL + cPk[((g - mm + 4 * R) & (R - 1)) * SW + l];
            Zc = Zc * qL + cB[(c + mm) * SW + l];
        }
#pragma unroll
        for (int j = 0; j < LC; ++j)
            d[j] = p.iir_K * (w[j] + (p.iir_qp[j + 1] * Yc + p.iir_qp[LC - 1 - j] * Zc));
        return;
    }
#pragma unroll
    for (int mm = MC; mm >= 1; --mm) {
        const int gp = g - mm, gq = g + mm;
        double cp, cb;
        if (wall && gp < 0) {
            // image of chunk -1 - gp, in the first tile
            cp = -par * p.iir_inv_q * cB[(-1 - gp) * SW + l];
        } else {
            cp = cPk[((gp + 4 * R) & (R - 1)) * SW + l];
        }
        if (wall && gq >= nc) {
            // image of chunk h, in this tile, the one before or the next
            const int h = 2 * nc - 1 - gq;
            const double ph = h >= (t + 1) * ST ? lookP[(h - (t + 1) * ST) * SW + l]
                                                : cPk[((h + 4 * R) & (R - 1)) * SW + l];
            cb = -par * p.iir_q * ph;
        } else {
            cb = cB[(c + mm) * SW + l];
        }
        Yc = Yc * qL + cp;
        Zc = Zc * qL + cb;
    }
#pragma unroll
    for (int j = 0; j < LC; ++j)
        d[j] = p.iir_K * (w[j] + (p.iir_qp[j + 1] * Yc + p.iir_qp[LC - 1 - j] * Zc));
}

template <int SW, int ST, int LC>
__global__ __launch_bounds__(SW * ST) void k_cols_mu_stream(KParams p,
                                                            const double *__restrict__ rho,
                                                            const double *__restrict__ mux,
                                                            double *__restrict__ mu_out,
                                                            double *__restrict__ fy_out)
{
    using S = StreamLds<SW, ST, LC>;
    extern __shared__ double smem[];
    double *edge = smem, *cPr = edge + S::NE * 4 * SW, *cB = cPr + 3 * S::R * SW,
           *left = cB + (ST + S::MC) * SW, *lookP = left + 3 * 4 * SW;
    // the carries and edges of chunks before the window start from zero
    for (int i = threadIdx.x; i < S::doubles; i += SW * ST) smem[i] = 0.0;
    const int nx = p.nx, ny = p.ny;
    const int c = threadIdx.x / SW, l = threadIdx.x - c * SW;
    const int col = blockIdx.x * SW + l;  // nx is a multiple of SW
    // between walls the solves close at the walls with mirror images and
    // take the column alone; periodic columns take the window of kColWin
    // chunks past each end
    const bool wall = p.bc_y != 0;
    const int E = wall ? 0 : kColWin<LC>;
    const int nc = ny / LC, NV = nc + 2 * E, ntile = (NV + ST - 1) / ST;
    // parities of the solves' inputs about a wall: rho even, d/dy rho odd, mu
    // even (mu - mu_wall odd for wetting walls)
    const double par2 = p.wet ? -1.0 : 1.0;
    // the LC values of window chunk v (zero outside the window): its rows
    // run down from the first one, or up beyond a wall (the mirror image)
    auto load = [&](const double *__restrict__ src, int v, double (&o)[LC]) {
        if (v >= 0 && v < NV) {
            const int y = (v - E) * LC;
            int r0 = y, dr = 1;
            if (y < 0) {
                r0 = p.bc_y ? -1 - y : y + ny;
                dr = p.bc_y ? -1 : 1;
            } else if (y >= ny) {
                r0 = p.bc_y ? 2 * ny - 1 - y : y - ny;
                dr = p.bc_y ? -1 : 1;
            }
            const double *q = src + (ptrdiff_t)r0 * nx + col;
            const ptrdiff_t st = (ptrdiff_t)dr * nx;
#pragma unroll
            for (int k = 0; k < LC; ++k) o[k] = q[k * st];
        } else {
#pragma unroll
            for (int k = 0; k < LC; ++k) o[k] = 0.0;
        }
    };
    // rn: rho of tile s; r1, r2, r3: of tiles s - 1, s - 2, s - 3; a1, a2:
    // d/dy rho of tiles s - 2, s - 3; m3: the third solve's input on tile s - 3
    double rn[LC], r1[LC], r2[LC], r3[LC], a1[LC], a2[LC], m3[LC];
#pragma unroll
    for (int k = 0; k < LC; ++k) r1[k] = r2[k] = r3[k] = a1[k] = a2[k] = m3[k] = 0.0;
    load(rho, c, rn);
    __syncthreads();
    for (int s = 0; s < ntile + 3; ++s) {
        // solve k runs on tile s - 1 - k when that tile is in the window (a
        // tile before it would only meet zeros; after it, nothing is stored)
        const bool run0 = s >= 1 && s <= ntile, run1 = s >= 2 && s <= ntile + 1 && !p.kappa_zero,
                   run2 = s >= 3;
        double rp[LC], mx[LC];
        load(rho, (s + 1) * ST + c, rp);
        load(mux, (s - 2) * ST + c, mx);
        double d1[LC];
        if (run0) {
            stream_solve<SW, ST, LC>(p, 0, s, c, l, nc, wall, 1.0, r1, rn, edge, cPr, cB, left,
                                     lookP, d1);
        } else {
#pragma unroll
            for (int k = 0; k < LC; ++k) d1[k] = 0.0;
        }
        // mu on tile s - 2, and the third solve's input there
        double mw[LC];
        {
            double d2[LC];
            if (run1) {
                stream_solve<SW, ST, LC>(p, 1, s, c, l, nc, wall, -1.0, a1, d1, edge, cPr, cB,
                                         left, lookP, d2);
            } else {
#pragma unroll
                for (int k = 0; k < LC; ++k) d2[k] = 0.0;
            }
            // (wetting walls: the solve differentiates mu - mu_wall, odd
            // about the walls; no chunk lies beyond a wall here)
            const int v2 = (s - 2) * ST + c, y2 = (v2 - E) * LC;
            double m[LC];
#pragma unroll
            for (int k = 0; k < LC; ++k) {
                m[k] = mx[k];
                if (!p.kappa_zero) m[k] -= p.kappa * d2[k];
                mw[k] = p.wet ? m[k] - p.mu_wall : m[k];
            }
            if (v2 >= E && v2 < E + nc) {
                double *q = mu_out + (ptrdiff_t)y2 * nx + col;
#pragma unroll
                for (int k = 0; k < LC; ++k) q[(ptrdiff_t)k * nx] = m[k];
            }
        }
        double d3[LC];
        if (run2) {
            stream_solve<SW, ST, LC>(p, 2, s, c, l, nc, wall, par2, m3, mw, edge, cPr, cB, left,
                                     lookP, d3);
        } else {
#pragma unroll
            for (int k = 0; k < LC; ++k) d3[k] = 0.0;
        }
        const int v3 = (s - 3) * ST + c;
        if (v3 >= E && v3 < E + nc) {
            double *q = fy_out + (ptrdiff_t)(v3 - E) * LC * nx + col;
#pragma unroll
            for (int k = 0; k < LC; ++k) q[(ptrdiff_t)k * nx] = -r3[k] * d3[k] + CS2 * a2[k];
        }
#pragma unroll
        for (int k = 0; k < LC; ++k) {
            r3[k] = r2[k];
            r2[k] = r1[k];
            r1[k] = rn[k];
            rn[k] = rp[k];
            a2[k] = a1[k];
            a1[k] = d1[k];
            m3[k] = mw[k];
        }
    }
}

// Pass C on rows [y0, y0 + rows_per_block) of one mesh.
// KEEP: the nine populations stay in registers from the first read to the
// collision; otherwise each is read again when needed (fewer registers, so
// more waves per SIMD; the second read is served by the caches).
//
// Besides the new state fout, the pass writes its three density groups gout
// (in the layout KParams gives): with f the streamed populations at a node,
//   g0 = (f0 + f1) + f3,   g1 = (f2 + f5) + f6,   g2 = (f4 + f7) + f8,
// the populations that arrive from the same row, from the row below and from
// the row above.  The next pass A forms rho = (g0 + g1) + g2 from them and so
// reads 3 planes instead of 9.  Each group is summed in this order whatever
// the source of its members (shifted along the row, or bounced back at a
// wall), so the groups are a function of fout alone.
//
// SEG: the split variant for long rows.  The block holds one segment
// [xs, xs + seg_len) of row y0 and a window of kSegWin chunks on each side
// (x periodic).  F_x comes from the row derivatives of the rho plane of pass A
// (rho_in) and of mu over the window; the chunk beyond each end of the segment
// also collides, without storing anything, so that the segment's end nodes
// receive the populations that cross its ends and every density group is
// written.  Each population is stored by the segment that owns its source
// node.
template <bool OBSERVE, bool KEEP, bool SEG = false, bool MRT = false>
__device__ __forceinline__ void rows_collide_body(
    const KParams &p, int y0, const double *__restrict__ f, const double *__restrict__ mu,
    const double *__restrict__ fy, double *__restrict__ fout, double *__restrict__ gout,
    double *__restrict__ o_rho, double *__restrict__ o_vx, double *__restrict__ o_vy,
    double *__restrict__ o_fx, int xs = 0, const double *__restrict__ rho_in = nullptr,
    int seg_n = 0)
{
    constexpr int LC = kRowLC;
    extern __shared__ double smem[];
    const int nx = p.nx, ny = p.ny;
    const int rows = SEG ? 1 : min(p.rows_per_block, ny - y0);
    const Chunk<LC> m = SEG ? seg_chunk<LC>(p, seg_n) : row_chunk<LC>(p, rows);
    // SEG: the window's chunks; LDS holds the window solve (edges, carries)
    // and then the edge exchange of the density groups
    const int nw = m.nc + 2 * kSegWin;
    const int nlc = SEG ? nw : p.rows_per_block * m.nc;
    LineLds L;
    if (SEG) {
        L.vbuf = smem;
        L.cP = smem + 4 * nw;
        L.cB = L.cP + nw;
        L.edge = L.cB + nw;
    } else {
        L = carve_lds(smem, m);
    }
    const int xc = xs + m.c * LC;
    const int y = y0 + m.l, x0 = !SEG ? xc : (xc < 0 ? xc + nx : (xc >= nx ? xc - nx : xc));
    // node (x0, y) in the scalar planes, in f and in g
    const size_t base = (size_t)y * nx + x0, fb = (size_t)y * p.fr + x0,
                 gb = (size_t)y * p.gr + x0;
    constexpr int NI = KEEP ? 9 : 1;
    double fi[NI][LC], rho[LC], mv[LC], jx[LC], jy[LC];
    // a segment's loads that do not depend on f (the rho and mu planes over
    // its window, F_y) go out first, so that their latency hides behind the
    // populations' (they are used after the moment sums and the solves'
    // barriers); over whole rows, where the rows' data are cache-resident on
    // the meshes that use them, they follow the populations
    double Fy[LC], wr[LC], wu[LC];
    if (SEG) {
        if ((int)threadIdx.x < nw) {
            vload<LC>(rho_in + base, wr);
            vload<LC>(mu + base, wu);
        }
        if (m.ok) vload<LC>(fy + base, Fy);
    }
    if (m.ok) {
        // rho = f0 + f1 + ... + f8 in index order; momentum in opposite pairs,
        // jx = (f1 - f3) + (f5 - f6) + (f8 - f7), jy = (f2 - f4) + (f5 - f8) +
        // (f6 - f7), formed as the planes arrive
        double t1[LC], t2[LC], t5[LC], t6[LC], t7[LC], dx1[LC], dx2[LC], dy1[LC];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            double t[LC];
            vload<LC>(f + i * p.fq + fb, t);
#pragma unroll
            for (int k = 0; k < LC; ++k) {
                if (KEEP) fi[i][k] = t[k];
                rho[k] = i == 0 ? t[k] : rho[k] + t[k];
                switch (i) {
                case 1: t1[k] = t[k]; break;
                case 2: t2[k] = t[k]; break;
                case 3: dx1[k] = t1[k] - t[k]; break;
                case 4: dy1[k] = t2[k] - t[k]; break;
                case 5: t5[k] = t[k]; break;
                case 6: dx2[k] = t5[k] - t[k]; t6[k] = t[k]; break;
                case 7: t7[k] = t[k]; break;
                case 8:
                    jx[k] = (dx1[k] + dx2[k]) + (t[k] - t7[k]);
                    jy[k] = (dy1[k] + (t5[k] - t[k])) + (t6[k] - t7[k]);
                    break;
                default: break;
                }
            }
        }
        if (!SEG) vload<LC>(mu + base, mv);
    }
    double Fx[LC];
    if (SEG) {
        // F_x of Eq. 12 (or of the pseudopotential model) from the planes,
        // bitwise as a whole-row derivative pass over them would give it
        const int w = threadIdx.x;
        double dxr[LC], dxm[LC];
        if (!p.sc) iir_solve_window<LC>(p, w, nw, p.iir_qL_row, wr, L.vbuf, L.cP, L.cB, dxr);
        iir_solve_window<LC>(p, w, nw, p.iir_qL_row, wu, L.vbuf, L.cP, L.cB, dxm);
        if (m.ok) {
#pragma unroll
            for (int k = 0; k < LC; ++k)
                Fx[k] = p.sc ? CS2 * wu[k] * dxm[k] : -wr[k] * dxm[k] + CS2 * dxr[k];
        }
    } else {
        // F_x of Eq. 12, or of the pseudopotential model (mv holds psi)
        double dxr[LC], dxm[LC];
        if (!p.sc) iir_solve<LC>(p, m, p.iir_qL_row, rho, 1.0, L, dxr);
        iir_solve<LC>(p, m, p.iir_qL_row, mv, 1.0, L, dxm);
        if (m.ok) {
            vload<LC>(fy + base, Fy);
#pragma unroll
            for (int k = 0; k < LC; ++k)
                Fx[k] = p.sc ? CS2 * mv[k] * dxm[k] : -rho[k] * dxm[k] + CS2 * dxr[k];
        }
    }
    if (OBSERVE) {
        if (!m.ok || (SEG && (m.c < 0 || m.c >= m.nc))) return;
#pragma unroll
        for (int k = 0; k < LC; ++k) {
            const double rh = rho[k], ir = 1.0 / rh;
            const double ux = jx[k] * ir, uy = jy[k] * ir;
            const size_t node = base + k;
            if (o_rho) o_rho[node] = rh;
            if (o_vx) o_vx[node] = ux + 0.5 * Fx[k] * ir;
            if (o_vy) o_vy[node] = uy + 0.5 * Fy[k] * ir;
            if (o_fx) o_fx[node] = Fx[k];
        }
        return;
    }
    // Edge exchange of the density groups: the value a chunk's first node
    // receives from the left neighbour (populations 1, 5, 8) and its last
    // node from the right neighbour (3, 6, 7), six slots per chunk.
    double *edge = L.edge;
    const int slot = SEG ? (int)threadIdx.x : m.l * m.nc + m.c;
    // SEG: the chunks beyond the segment's ends only supply edge values
    const bool store = !SEG || (m.c >= 0 && m.c < m.nc);
    // the row's down-going groups bounce back at a bottom wall, the
    // up-going ones at a top wall
    const bool refl_d = p.bc_y && y == 0, refl_u = p.bc_y && y == ny - 1;
    double gm[LC], gu[LC], gd[LC], hm = 0.0, hu = 0.0, hd = 0.0;
    if (m.ok) {
        double ux[LC], uy[LC], vx2[LC], vy2[LC], uu[LC], uu2[LC];
#pragma unroll
        for (int k = 0; k < LC; ++k) {
            const double ir = 1.0 / rho[k];
            ux[k] = jx[k] * ir;
            uy[k] = jy[k] * ir;
            vx2[k] = ux[k] + Fx[k] * ir;
            vy2[k] = uy[k] + Fy[k] * ir;
            uu[k] = ux[k] * ux[k] + uy[k] * uy[k];
            uu2[k] = vx2[k] * vx2[k] + vy2[k] * vy2[k];
        }
        // MRT (Eq. 4): the relaxed moments' departures from equilibrium need
        // all nine populations of a node before the first is collided
        double dm[MRT ? LC : 1][6];
        if (MRT) {
            double qa[9][LC];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if (KEEP) {
#pragma unroll
                    for (int k = 0; k < LC; ++k) qa[i][k] = fi[KEEP ? i : 0][k];
                } else {
                    vload<LC>(f + i * p.fq + fb, qa[i]);
                }
            }
#pragma unroll
            for (int k = 0; k < LC; ++k) {
                double qk[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) qk[i] = qa[i][k];
                mrt_departures(p, qk, rho[k], jx[k], jy[k], ux[k], uy[k], dm[MRT ? k : 0]);
            }
        }
        // collision and push streaming, one population at a time: population
        // i of node (x, y) goes to (x + e_x, y + e_y)
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            double q[LC], v[LC];
            if (KEEP) {
#pragma unroll
                for (int k = 0; k < LC; ++k) q[k] = fi[KEEP ? i : 0][k];
            } else {
                vload<LC>(f + i * p.fq + fb, q);
            }
#pragma unroll
            for (int k = 0; k < LC; ++k) {
                const double eq = feq(i, rho[k], ux[k], uy[k], uu[k]);
                const double eq2 = feq(i, rho[k], vx2[k], vy2[k], uu2[k]);
                if (MRT)
                    v[k] = mrt_relax(i, q[k], dm[MRT ? k : 0]) + (eq2 - eq);
                else
                    v[k] = q[k] - (q[k] - eq) * p.inv_tau + (eq2 - eq);
            }
            const bool refl = (EY[i] < 0 && refl_d) || (EY[i] > 0 && refl_u);
            if (refl) {
                // half-way bounce-back into the opposite population of the
                // same node; a moving wall adds -2 w rho (e.U)/c_s^2
#pragma unroll
                for (int k = 0; k < LC; ++k)
                    v[k] = v[k] - 2.0 * WT[i] * rho[k] * (EX[i] * p.wall_ux) / CS2;
            }
            // density groups at the arrival nodes; a value that arrives
            // from a neighbouring chunk is added after the exchange, and a
            // later member that must follow it waits in hm, hu or hd
            switch (i) {
            case 0:
#pragma unroll
                for (int k = 0; k < LC; ++k) gm[k] = v[k];
                break;
            case 1:
#pragma unroll
                for (int k = 1; k < LC; ++k) gm[k] += v[k - 1];
                edge[0 * nlc + slot] = v[LC - 1];
                break;
            case 3:
#pragma unroll
                for (int k = 1; k < LC - 1; ++k) gm[k] += v[k + 1];
                hm = v[1];
                edge[1 * nlc + slot] = v[0];
                break;
            case 2:
#pragma unroll
                for (int k = 0; k < LC; ++k) gu[k] = v[k];
                break;
            case 5:
                if (refl_u) {
#pragma unroll
                    for (int k = 0; k < LC; ++k) gu[k] += v[k];
                } else {
#pragma unroll
                    for (int k = 1; k < LC; ++k) gu[k] += v[k - 1];
                    edge[2 * nlc + slot] = v[LC - 1];
                }
                break;
            case 6:
                if (refl_u) {
#pragma unroll
                    for (int k = 0; k < LC; ++k) gu[k] += v[k];
                } else {
#pragma unroll
                    for (int k = 1; k < LC - 1; ++k) gu[k] += v[k + 1];
                    hu = v[1];
                    edge[3 * nlc + slot] = v[0];
                }
                break;
            case 4:
#pragma unroll
                for (int k = 0; k < LC; ++k) gd[k] = v[k];
                break;
            case 7:
                if (refl_d) {
#pragma unroll
                    for (int k = 0; k < LC; ++k) gd[k] += v[k];
                } else {
#pragma unroll
                    for (int k = 0; k < LC - 1; ++k) gd[k] += v[k + 1];
                    edge[4 * nlc + slot] = v[0];
                }
                break;
            case 8:
                if (refl_d) {
#pragma unroll
                    for (int k = 0; k < LC; ++k) gd[k] += v[k];
                } else {
#pragma unroll
                    for (int k = 1; k < LC - 1; ++k) gd[k] += v[k - 1];
                    hd = v[LC - 2];
                    edge[5 * nlc + slot] = v[LC - 1];
                }
                break;
            default: break;
            }
            if (!store) continue;
            if (refl) {
                vstore<LC>(fout + OPP[i] * p.fq + fb, v);
                continue;
            }
            int ty = y + EY[i];
            ty = ty < 0 ? ty + ny : (ty >= ny ? ty - ny : ty);
            double *dst = fout + i * p.fq + (size_t)ty * p.fr;
            if (EX[i] == 0) {
                vstore<LC>(dst + x0, v);
                continue;
            }
            // Shifted populations: the aligned chunk [x0, x0 + LC) of the
            // target row receives LC - 1 of this thread's values and one
            // value of the neighbouring chunk, taken from the adjacent lane.
            // Where that chunk is not on the adjacent lane (first/last lane
            // of the wave, first/last chunk of the row), the boundary value
            // goes out as a single store from its owner instead.
            const int lane = threadIdx.x & 63;
            if (EX[i] > 0) {
                const double from_left = __shfl_up(v[LC - 1], 1);
                const bool left_here = lane > 0 && m.c > 0;
                double w[LC];
                w[0] = from_left;
#pragma unroll
                for (int k = 1; k < LC; ++k) w[k] = v[k - 1];
                if (left_here) {
                    vstore<LC>(dst + x0, w);
                } else {
#pragma unroll
                    for (int k = 1; k < LC; ++k) dst[x0 + k] = w[k];
                }
                const bool right_here = lane < 63 && m.c < m.nc - 1;
                if (!right_here) {
                    const int tx = x0 + LC == nx ? 0 : x0 + LC;
                    dst[tx] = v[LC - 1];
                }
            } else {
                const double from_right = __shfl_down(v[0], 1);
                const bool right_here = lane < 63 && m.c < m.nc - 1;
                double w[LC];
#pragma unroll
                for (int k = 0; k < LC - 1; ++k) w[k] = v[k + 1];
                w[LC - 1] = from_right;
                if (right_here) {
                    vstore<LC>(dst + x0, w);
                } else {
#pragma unroll
                    for (int k = 0; k < LC - 1; ++k) dst[x0 + k] = w[k];
                }
                const bool left_here = lane > 0 && m.c > 0;
                if (!left_here) {
                    const int tx = x0 == 0 ? nx - 1 : x0 - 1;
                    dst[tx] = v[0];
                }
            }
        }
    }
    __syncthreads();
    if (!m.ok || !store) return;
    // x is periodic: the neighbours of the first and last chunk wrap (in a
    // segment they are the window's chunks beyond its ends)
    const int row0 = m.l * m.nc;
    const int left = SEG ? slot - 1 : row0 + (m.c > 0 ? m.c - 1 : m.nc - 1);
    const int right = SEG ? slot + 1 : row0 + (m.c < m.nc - 1 ? m.c + 1 : 0);
    gm[0] = (gm[0] + edge[0 * nlc + left]) + hm;
    gm[LC - 1] += edge[1 * nlc + right];
    if (!refl_u) {
        gu[0] = (gu[0] + edge[2 * nlc + left]) + hu;
        gu[LC - 1] += edge[3 * nlc + right];
    }
    if (!refl_d) {
        gd[0] += edge[5 * nlc + left];
        gd[LC - 1] = (gd[LC - 1] + edge[4 * nlc + right]) + hd;
    }
    // g0 of this row; g1 of the row above (of this row at a top wall, as
    // g2); g2 of the row below (of this row at a bottom wall, as g1)
    const size_t up =
        refl_u ? 2 * p.gq + gb : p.gq + (size_t)(y + 1 < ny ? y + 1 : 0) * p.gr + x0;
    const size_t dn =
        refl_d ? p.gq + gb : 2 * p.gq + (size_t)(y > 0 ? y - 1 : ny - 1) * p.gr + x0;
    vstore<LC>(gout + gb, gm);
    vstore<LC>(gout + up, gu);
    vstore<LC>(gout + dn, gd);
}

template <int MAXT, bool OBSERVE, bool KEEP, bool MRT = false>
__global__ __launch_bounds__(MAXT) void k_rows_collide_iir(
    KParams p, const double *__restrict__ f, const double *__restrict__ mu,
    const double *__restrict__ fy, double *__restrict__ fout, double *__restrict__ gout,
    double *__restrict__ o_rho, double *__restrict__ o_vx, double *__restrict__ o_vy,
    double *__restrict__ o_fx)
{
    rows_collide_body<OBSERVE, KEEP, false, MRT>(p, blockIdx.x * p.rows_per_block, f, mu, fy,
                                                 fout, gout, o_rho, o_vx, o_vy, o_fx);
}

// ---- row segments: the split collision pass, and long rows -------------
// Rows longer than one 256-thread workgroup holds with the populations in
// registers may run pass C over row segments of kSegLen nodes (the last one
// ragged), one workgroup per segment that holds f in registers.  Each
// workgroup takes the row derivatives over its segment's window (the
// segment and kSegWin chunks on each side, x periodic), so the pass stays
// one kernel and every density group is written.  Rows longer than one
// workgroup holds at all (more than 4096 nodes) also run pass A and the
// observation pass over windowed segments.

template <bool KEEP, bool MRT>
__global__ __launch_bounds__(kSegThreads) void k_collide_seg_iir(
    KParams p, const double *__restrict__ f, const double *__restrict__ rho,
    const double *__restrict__ mu, const double *__restrict__ fy, double *__restrict__ fout,
    double *__restrict__ gout)
{
    const int nseg = row_segments(p, p.seg_len);
    const int y = blockIdx.x / nseg, sg = blockIdx.x - y * nseg;
    const int xs = sg * p.seg_len;
    rows_collide_body<false, KEEP, true, MRT>(p, y, f, mu, fy, fout, gout, nullptr, nullptr,
                                              nullptr, nullptr, xs, rho,
                                              min(p.seg_len, p.nx - xs));
}

// Observation (rho, v, F_x of the current state) over row segments.
__global__ __launch_bounds__(kSegThreads) void k_observe_seg_iir(
    KParams p, const double *__restrict__ f, const double *__restrict__ rho,
    const double *__restrict__ mu, const double *__restrict__ fy, double *__restrict__ o_rho,
    double *__restrict__ o_vx, double *__restrict__ o_vy, double *__restrict__ o_fx)
{
    const int nseg = row_segments(p, p.seg_len);
    const int y = blockIdx.x / nseg, sg = blockIdx.x - y * nseg;
    const int xs = sg * p.seg_len;
    rows_collide_body<true, false, true, false>(p, y, f, mu, fy, nullptr, nullptr, o_rho, o_vx,
                                                o_vy, o_fx, xs, rho, min(p.seg_len, p.nx - xs));
}

// Pass A over a row segment of kRhoSegLen nodes (the last one ragged) and a
// window of kRhoWin chunks on each side (rows longer than one workgroup holds): the same values as the
// whole-row pass, since each derivative sums the carries of exactly MC chunks
// on each side, computed from the same values.
template <bool SC>
__global__ __launch_bounds__(kRhoThreads) void k_rows_rho_seg_iir(KParams p,
                                                                  const double *__restrict__ g,
                                                                  double *__restrict__ rho_out,
                                                                  double *__restrict__ mux_out)
{
    constexpr int LC = kRowLC;
    extern __shared__ double smem[];
    const int nseg = row_segments(p, kRhoSegLen);
    const int y = blockIdx.x / nseg, sg = blockIdx.x - y * nseg;
    const int xs = sg * kRhoSegLen, nc = min(kRhoSegLen, p.nx - xs) / LC;
    const int nx = p.nx, w = threadIdx.x, nw = nc + 2 * kRhoWin, c = w - kRhoWin;
    const int xc = xs + c * LC;
    const int x0 = xc < 0 ? xc + nx : (xc >= nx ? xc - nx : xc);
    const size_t base = (size_t)y * nx + x0, gb = (size_t)y * p.gr + x0;
    const bool core = c >= 0 && c < nc;
    double *vbuf = smem, *cP = smem + 4 * nw, *cB = cP + nw;
    double rho[LC], mx[LC];
    if (w < nw) {
        double g0[LC], g1[LC], g2[LC];
        vload<LC>(g + gb, g0);
        vload<LC>(g + p.gq + gb, g1);
        vload<LC>(g + 2 * p.gq + gb, g2);
#pragma unroll
        for (int k = 0; k < LC; ++k) rho[k] = (g0[k] + g1[k]) + g2[k];
        if (core) {
            vstore<LC>(rho_out + base, rho);
#pragma unroll
            for (int k = 0; k < LC; ++k)
                mx[k] = SC ? sc_psi(p, rho[k]) : p.k2 * mu0_capped(p, rho[k]);
        }
    }
    if (p.kappa_zero || SC) {
        if (core) vstore<LC>(mux_out + base, mx);
        return;
    }
    double d1[LC], d2[LC];
#pragma unroll
    for (int k = 0; k < LC; ++k) d1[k] = 0.0;
    iir_solve_window<LC>(p, w, nw, p.iir_qL_row, rho, vbuf, cP, cB, d1);
    iir_solve_window<LC>(p, w, nw, p.iir_qL_row, d1, vbuf, cP, cB, d2);
    if (core) {
#pragma unroll
        for (int k = 0; k < LC; ++k) mx[k] -= p.kappa * d2[k];
        vstore<LC>(mux_out + base, mx);
    }
}

// ---- batched passes: one launch covers the blocks of every active mesh ----
// Work item b names the mesh and its first row (row passes) or column
// (column pass); each mesh has its own parameter block and buffers.  parity
// selects which of the mesh's two state buffers (distribution and density
// groups) holds the state.

__global__ __launch_bounds__(256) void kb_rows_rho(const KParams *__restrict__ kps,
                                                   const SimBuffers *__restrict__ sb,
                                                   const WorkItem *__restrict__ work, int parity)
{
    const WorkItem w = work[blockIdx.x];
    const SimBuffers &b = sb[w.sim];
    if (kps[w.sim].sc)  // uniform over the workgroup
        rows_rho_body<true>(kps[w.sim], w.start, b.g[parity], b.rho, b.mux);
    else
        rows_rho_body<false>(kps[w.sim], w.start, b.g[parity], b.rho, b.mux);
}

template <int LC, int MAXT>
__global__ __launch_bounds__(MAXT) void kb_cols_mu(const KParams *__restrict__ kps,
                                                   const SimBuffers *__restrict__ sb,
                                                   const WorkItem *__restrict__ work)
{
    const WorkItem w = work[blockIdx.x];
    const SimBuffers &b = sb[w.sim];
    cols_mu_body<LC>(kps[w.sim], w.start, b.rho, b.mux, b.mu, b.fy);
}

template <bool MRT>
__global__ __launch_bounds__(256) void kb_rows_collide(const KParams *__restrict__ kps,
                                                       const SimBuffers *__restrict__ sb,
                                                       const WorkItem *__restrict__ work,
                                                       int parity)
{
    const WorkItem w = work[blockIdx.x];
    const SimBuffers &b = sb[w.sim];
    rows_collide_body<false, true, false, MRT>(kps[w.sim], w.start, b.f[parity], b.mu, b.fy,
                                               b.f[1 - parity], b.g[1 - parity], nullptr,
                                               nullptr, nullptr, nullptr);
}

}  // namespace

// LDS of a block of nl lines of n nodes in chunks of lc: the values with
// their ghosts, the two carry planes with theirs and (collision pass) the six
// edge planes of one slot per chunk (the layout of Chunk and carve_lds).
static size_t line_lds(int n, int nl, int lc, bool edges)
{
    const size_t nc = n / lc, L = nl;
    return sizeof(double) * (L * 4 * (nc + 2) + 2 * L * (nc + kCarry(lc)) + (edges ? 6 * L * nc : 0));
}

size_t batch_row_lds(int rows, int nx, bool collide) { return line_lds(nx, rows, kRowLC, collide); }

// every mesh's strip (w <= wmax columns of ny, w ny <= col_elems) fits
size_t batch_col_lds(int col_elems, int lc, int wmax)
{
    const size_t W = wmax;
    return sizeof(double) * (4 * ((size_t)col_elems / lc + 2 * W) +
                             2 * ((size_t)col_elems / lc + W * kCarry(lc)));
}

hipError_t launch_batch_rows_rho(const KParams *kps, const SimBuffers *sb, const WorkItem *work,
                                 int nwork, int parity, size_t lds, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    hipLaunchKernelGGL(kb_rows_rho, dim3(nwork), dim3(256), lds, s, kps, sb, work, parity);
    return hipGetLastError();
}

hipError_t launch_batch_cols_mu(const KParams *kps, const SimBuffers *sb, const WorkItem *work,
                                int nwork, int col_elems, int lc, int wmax, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    const int T = col_elems / lc;
    const size_t lds = batch_col_lds(col_elems, lc, wmax);
    if (lc == 4 && T <= 256)
        hipLaunchKernelGGL((kb_cols_mu<4, 256>), dim3(nwork), dim3(T), lds, s, kps, sb, work);
    else if (lc == 4)
        hipLaunchKernelGGL((kb_cols_mu<4, 1024>), dim3(nwork), dim3(T), lds, s, kps, sb, work);
    else if (T <= 256)
        hipLaunchKernelGGL((kb_cols_mu<8, 256>), dim3(nwork), dim3(T), lds, s, kps, sb, work);
    else
        hipLaunchKernelGGL((kb_cols_mu<8, 1024>), dim3(nwork), dim3(T), lds, s, kps, sb, work);
    return hipGetLastError();
}

hipError_t launch_batch_rows_collide(const KParams *kps, const SimBuffers *sb,
                                     const WorkItem *work, int nwork, int parity, size_t lds,
                                     bool mrt, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    if (mrt)
        hipLaunchKernelGGL(kb_rows_collide<true>, dim3(nwork), dim3(256), lds, s, kps, sb, work,
                           parity);
    else
        hipLaunchKernelGGL(kb_rows_collide<false>, dim3(nwork), dim3(256), lds, s, kps, sb, work,
                           parity);
    return hipGetLastError();
}

bool iir_rows_ok(const KParams &p)
{
    return p.nx >= kFastMinLine && p.nx % kRowLC == 0 && p.nx / kRowLC > kCarry(kRowLC) &&
           p.iir_m_row <= kCarry(kRowLC) &&
           p.rows_per_block * (p.nx / kRowLC) <= kMaxBlockThreads;
}

bool iir_cols_ok(const KParams &p, int lc, int width)
{
    return p.ny >= kFastMinLine && p.ny % lc == 0 && p.ny / lc > kCarry(lc) &&
           p.iir_m_col <= kCarry(lc) && width * (p.ny / lc) <= kMaxBlockThreads &&
           width * p.ny <= kMaxColElems;
}

static size_t row_lds_iir(const KParams &p, bool collide)
{
    return line_lds(p.nx, p.rows_per_block, kRowLC, collide);
}

static size_t col_lds_iir(const KParams &p)
{
    return line_lds(p.ny, p.cols_per_block, p.col_lc, false);
}

static int row_threads_iir(const KParams &p) { return p.rows_per_block * (p.nx / kRowLC); }
static int col_threads_iir(const KParams &p) { return p.cols_per_block * (p.ny / p.col_lc); }

#define CPLBM_IIR_THREADS(T, K256, K1024, GRIDARGS)                                       \
    do {                                                                                   \
        if ((T) <= 256)                                                                    \
            hipLaunchKernelGGL(K256, GRIDARGS);                                            \
        else                                                                               \
            hipLaunchKernelGGL(K1024, GRIDARGS);                                           \
    } while (0)

hipError_t launch_rows_rho_iir(const KParams &p, const double *g, double *rho, double *mux,
                               hipStream_t s)
{
    const int T = row_threads_iir(p);
#define ARGS dim3(row_blocks(p)), dim3(T), row_lds_iir(p, false), s, p, g, rho, mux
    if (p.sc)
        CPLBM_IIR_THREADS(T, (k_rows_rho_iir<256, true>), (k_rows_rho_iir<1024, true>), ARGS);
    else
        CPLBM_IIR_THREADS(T, (k_rows_rho_iir<256, false>), (k_rows_rho_iir<1024, false>), ARGS);
#undef ARGS
    return hipGetLastError();
}

int col_tile_chunks(int width, int lc)
{
    const int E = lc == 4 ? kColWin<4> : (lc == 8 ? kColWin<8> : kColWin<16>);
    return kMaxBlockThreads / width - 2 * E;
}

int col_window_chunks(int lc)
{
    return lc == 4 ? kColWin<4> : (lc == 8 ? kColWin<8> : kColWin<16>);
}

template <int SW, int ST, int LC>
static hipError_t launch_stream(const KParams &p, const double *rho, const double *mux,
                                double *mu, double *fy, hipStream_t s)
{
    const size_t lds = sizeof(double) * StreamLds<SW, ST, LC>::doubles;
    hipLaunchKernelGGL((k_cols_mu_stream<SW, ST, LC>), dim3(p.nx / SW), dim3(SW * ST), lds, s, p,
                       rho, mux, mu, fy);
    return hipGetLastError();
}

// Chunk length of the streamed column pass: 8 nodes where the columns are
// whole 8-node chunks, else 4.
int col_stream_chunk(int ny) { return ny % 8 == 0 ? 8 : 4; }

size_t col_stream_lds(int width, int lc)
{
    int d = 0;
    if (lc == 8) {
        d = width == 8    ? StreamLds<8, 64, 8>::doubles
            : width == 32 ? StreamLds<32, 16, 8>::doubles
                          : StreamLds<16, 32, 8>::doubles;
    } else {
        d = width == 8    ? StreamLds<8, 64, 4>::doubles
            : width == 32 ? StreamLds<32, 16, 4>::doubles
                          : StreamLds<16, 32, 4>::doubles;
    }
    return sizeof(double) * (size_t)d;
}

bool col_stream_ok(const KParams &p, int width)
{
    const int lc = col_stream_chunk(p.ny);
    const int win = lc == 8 ? kColWin<8> * 8 : kColWin<4> * 4;
    // between walls the solves close with mirror images; periodic columns
    // need the window, which must not wrap more than once
    return !p.sc && (width == 8 || width == 16 || width == 32) && p.nx % width == 0 &&
           p.ny % 4 == 0 && p.ny >= kFastMinLine && (p.bc_y || p.ny >= win);
}

hipError_t launch_cols_mu_iir(const KParams &p, const double *rho, const double *mux, double *mu,
                              double *fy, hipStream_t s)
{
    if (p.col_stream) {
        if (!col_stream_ok(p, p.cols_per_block)) return hipErrorInvalidValue;
        if (p.col_lc != col_stream_chunk(p.ny)) return hipErrorInvalidValue;
        if (p.col_lc == 8) {
            switch (p.cols_per_block) {
            case 8: return launch_stream<8, 64, 8>(p, rho, mux, mu, fy, s);
            case 32: return launch_stream<32, 16, 8>(p, rho, mux, mu, fy, s);
            default: return launch_stream<16, 32, 8>(p, rho, mux, mu, fy, s);
            }
        }
        switch (p.cols_per_block) {
        case 8: return launch_stream<8, 64, 4>(p, rho, mux, mu, fy, s);
        case 32: return launch_stream<32, 16, 4>(p, rho, mux, mu, fy, s);
        default: return launch_stream<16, 32, 4>(p, rho, mux, mu, fy, s);
        }
    }
    if (p.col_win) {
        const int W = p.cols_per_block, nw = p.col_tile / p.col_lc + 2 * col_window_chunks(p.col_lc);
        const int nb = ((p.nx + W - 1) / W) * ((p.ny + p.col_tile - 1) / p.col_tile);
        const size_t lds = sizeof(double) * 6 * (size_t)nw * W;
        const int T = (W * nw + 63) / 64 * 64;
#define ARGS dim3(nb), dim3(T), lds, s, p, rho, mux, mu, fy
        switch (p.col_lc) {
        case 4: hipLaunchKernelGGL(k_cols_mu_win<4>, ARGS); break;
        case 8: hipLaunchKernelGGL(k_cols_mu_win<8>, ARGS); break;
        default: hipLaunchKernelGGL(k_cols_mu_win<16>, ARGS); break;
        }
#undef ARGS
        return hipGetLastError();
    }
    const int T = col_threads_iir(p);
#define ARGS dim3(col_blocks(p)), dim3(T), col_lds_iir(p), s, p, rho, mux, mu, fy
    switch (p.col_lc) {
    case 4: CPLBM_IIR_THREADS(T, (k_cols_mu_iir<4, 256>), (k_cols_mu_iir<4, 1024>), ARGS); break;
    case 8: CPLBM_IIR_THREADS(T, (k_cols_mu_iir<8, 256>), (k_cols_mu_iir<8, 1024>), ARGS); break;
    default: CPLBM_IIR_THREADS(T, (k_cols_mu_iir<16, 256>), (k_cols_mu_iir<16, 1024>), ARGS); break;
    }
#undef ARGS
    return hipGetLastError();
}

bool iir_split_ok(const KParams &p)
{
    return p.nx > kSegLen && p.nx % kRowLC == 0 && p.seg_len == kSegLen &&
           p.iir_m_row <= kCarry(kRowLC);
}

// Workgroups of a segment kernel (segments of len nodes): one per segment
// of every row, threads for the widest window.
static int seg_blocks(const KParams &p, int len) { return p.ny * ((p.nx + len - 1) / len); }
static int seg_threads(int len, int win) { return ((len / kRowLC + 2 * win) + 63) / 64 * 64; }

hipError_t launch_rows_rho_seg_iir(const KParams &p, const double *g, double *rho, double *mux,
                                   hipStream_t s)
{
    if (!iir_split_ok(p)) return hipErrorInvalidValue;
    const int nw = kRhoSegLen / kRowLC + 2 * kRhoWin;
    const size_t lds = sizeof(double) * 6 * (size_t)nw;
#define ARGS                                                                                   \
    dim3(seg_blocks(p, kRhoSegLen)), dim3(seg_threads(kRhoSegLen, kRhoWin)), lds, s, p, g, rho, \
        mux
    if (p.sc)
        hipLaunchKernelGGL((k_rows_rho_seg_iir<true>), ARGS);
    else
        hipLaunchKernelGGL((k_rows_rho_seg_iir<false>), ARGS);
#undef ARGS
    return hipGetLastError();
}

hipError_t launch_observe_seg_iir(const KParams &p, const double *f, const double *rho,
                                  const double *mu, const double *fy, double *o_rho, double *o_vx,
                                  double *o_vy, double *o_fx, hipStream_t s)
{
    if (!iir_split_ok(p)) return hipErrorInvalidValue;
    const int nw = p.seg_len / kRowLC + 2 * kSegWin;
    const size_t lds = sizeof(double) * 12 * (size_t)nw;
    hipLaunchKernelGGL(k_observe_seg_iir, dim3(seg_blocks(p, p.seg_len)),
                       dim3(seg_threads(p.seg_len, kSegWin)), lds, s, p, f, rho, mu, fy, o_rho,
                       o_vx, o_vy, o_fx);
    return hipGetLastError();
}

hipError_t launch_collide_split_iir(const KParams &p, const double *f, const double *rho,
                                    const double *mu, const double *fy, double *fout,
                                    double *gout, hipStream_t s)
{
    if (!iir_split_ok(p)) return hipErrorInvalidValue;
    const int S = p.seg_len, blocks = seg_blocks(p, S);
    const int nw = S / kRowLC + 2 * kSegWin;
    const int T = seg_threads(S, kSegWin);
    // the window solve's edges and carries (4 + 2 per chunk), then the six
    // edge planes of the density groups
    const size_t lds = sizeof(double) * 12 * (size_t)nw;
#define ARGS dim3(blocks), dim3(T), lds, s, p, f, rho, mu, fy, fout, gout
    if (p.row_keep && p.mrt)
        hipLaunchKernelGGL((k_collide_seg_iir<true, true>), ARGS);
    else if (p.row_keep)
        hipLaunchKernelGGL((k_collide_seg_iir<true, false>), ARGS);
    else if (p.mrt)
        hipLaunchKernelGGL((k_collide_seg_iir<false, true>), ARGS);
    else
        hipLaunchKernelGGL((k_collide_seg_iir<false, false>), ARGS);
#undef ARGS
    return hipGetLastError();
}

hipError_t launch_rows_collide_iir(const KParams &p, const double *f, const double *mu,
                                   const double *fy, double *fout, double *gout, double *o_rho,
                                   double *o_vx, double *o_vy, double *o_fx, bool observe,
                                   hipStream_t s)
{
    const int T = row_threads_iir(p);
#define ARGS                                                                                   \
    dim3(row_blocks(p)), dim3(T), row_lds_iir(p, true), s, p, f, mu, fy, fout, gout, o_rho,     \
        o_vx, o_vy, o_fx
    // holding f in registers only pays with 256-thread blocks (no spills)
    const bool keep = p.row_keep && T <= 256;
    if (observe)
        CPLBM_IIR_THREADS(T, (k_rows_collide_iir<256, true, false>),
                          (k_rows_collide_iir<1024, true, false>), ARGS);
    else if (keep && p.mrt)
        hipLaunchKernelGGL((k_rows_collide_iir<256, false, true, true>), ARGS);
    else if (keep)
        hipLaunchKernelGGL((k_rows_collide_iir<256, false, true>), ARGS);
    else if (p.mrt)
        CPLBM_IIR_THREADS(T, (k_rows_collide_iir<256, false, false, true>),
                          (k_rows_collide_iir<1024, false, false, true>), ARGS);
    else
        CPLBM_IIR_THREADS(T, (k_rows_collide_iir<256, false, false>),
                          (k_rows_collide_iir<1024, false, false>), ARGS);
#undef ARGS
    return hipGetLastError();
}

}  // namespace cplbm
