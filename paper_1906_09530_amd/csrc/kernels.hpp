// Device-side parameter block and kernel launchers of the solver.
#pragma once

#include <hip/hip_runtime.h>

namespace cplbm {

constexpr int kMaxStages = 8;        // parallel cyclic reduction stages
constexpr int kElemsPerThread = 4;   // line elements held by one thread
constexpr int kMaxBlockThreads = 1024;
constexpr int kMaxBlockElems = kMaxBlockThreads * kElemsPerThread;  // 4096 doubles per LDS buffer
// nodes of a column strip the factorised solve holds (one thread per chunk,
// at most 1024 chunks; its LDS, four edge values and two carries per chunk,
// stays under ~50 KB)
constexpr int kMaxColElems = 16384;
constexpr int kFastMinLine = 64;     // lines this long skip the general modulo indexing

// Everything a kernel needs, passed by value.
struct KParams {
    int nx, ny, bc_y, eos;
    // row passes: whole rows per block, threads per block
    int rows_per_block, row_threads;
    // column pass: whole columns per block, threads per block, and the
    // block -> strip permutation that keeps neighbouring strips on one XCD
    int cols_per_block, col_threads, col_xcd_groups;
    int nstage;      // reduction stages of the line solve
    int kappa_zero;  // kappa == 0: the Laplacian is not needed
    double a, b, RT, A;  // EOS constants; A = a alpha(T)
    double eos_c1;       // A / b (RK, RKS) or A / (2 sqrt(2) b) (PR)
    double k2, kappa, inv_tau, mu_cap, wall_ux;
    // collision: 0 BGK (Eq. 1), 1 MRT (Eq. 4) with mrt_w = s_k / |M_k|^2 of
    // (e, eps, q_x, q_y, p_xx, p_xy); force: 0 chemical potential (Eq. 12),
    // 1 pseudopotential comparison model (Sec. 5.1)
    int mrt, sc;
    double mrt_w[6];
    // wetting walls: mu is held at mu_wall (mesh units) on the walls
    int wet;
    double mu_wall;
    double cfd_a2, cfd_b4;  // a/2 and b/4 of Eq. 37 (h = 1)
    double pcr_c[kMaxStages], pcr_g[kMaxStages];
    // factorised inverse of the circulant compact-scheme matrix (fast path):
    // pole q, 1/q, K = 1/(1 + 2 al q), powers q^0..q^16, and per pass the
    // chunk length, its power q^LC and the number of carried chunks M
    int use_iir_rows, use_iir_cols, col_lc;
    // column pass over tiles of col_tile rows with windows (col_win; tall
    // columns), streamed down strips in tiles (col_stream), else over whole
    // columns
    int col_win, col_tile, col_stream;
    int row_keep;   // collision pass holds f in registers (tuned)
    int row_split;  // collision pass over row segments (tuned; see below)
    int row_win;    // rows beyond one workgroup: every row pass over segments
    int seg_len;    // row segment of the segment kernels (0: none)
    int iir_m_row, iir_m_col;
    double iir_q, iir_inv_q, iir_K, iir_qL_row, iir_qL_col;
    double iir_qp[17];
    // layout of the distribution f and of its density groups g: population
    // (group) i of node (x, y) at f[i fq + y fr + x] (g[i gq + y gr + x]);
    // planes (fq = nx ny, fr = nx) or each row's populations side by side
    // (fq = nx, fr = 9 nx; gq = nx, gr = 3 nx)
    size_t fq, fr, gq, gr;
};

// Plane-major (f[9][ny][nx], g[3][ny][nx]) or row-interleaved
// (f[ny][9][nx], g[ny][3][nx]) layout of the state.
void set_state_layout(KParams *p, bool rows_interleaved);

constexpr int kIirRowChunk = 4;
// row segment of the segment kernels: 224 chunks, which with the collision
// window's 26 fill a 256-thread workgroup
constexpr int kSegLen = 896;
constexpr int kMaxWholeRow = 4096;    // longest row one workgroup holds

int row_blocks(const KParams &p);
int col_blocks(const KParams &p);

// The state is f together with its three density groups g (layout: KParams fq..gr):
// at each node g0 = (f0 + f1) + f3, g1 = (f2 + f5) + f6, g2 = (f4 + f7) + f8,
// so that rho = (g0 + g1) + g2.  The collision pass writes g with the new f;
// wherever f is set otherwise, launch_density_groups forms them.
//
// Pass A over rows: rho and the row part of the chemical potential (Eq. 33),
// mux = k^2 psi'(rho) - kappa d2rho/dx2 (k^2 psi'(rho) when kappa = 0).  The
// fast kernels read rho from g, the general ones sum f.
hipError_t launch_rows_rho(const KParams &p, const double *f, const double *g, double *rho,
                           double *mux, hipStream_t s);
// Pass B over columns: d/dy rho, d2/dy2 rho, mu = mux - kappa d2rho/dy2 (Eq. 33),
// d/dy mu, F_y (Eq. 12).
hipError_t launch_cols_mu(const KParams &p, const double *rho, const double *mux, double *mu,
                          double *fy, hipStream_t s);
// Pass C over rows: d/dx rho, d/dx mu, F_x, collision and streaming f -> fout,
// and (fast kernels) the density groups gout of fout.  rho: pass A's density
// plane, read by the segment variant (row_split) only.
hipError_t launch_rows_collide(const KParams &p, const double *f, const double *mu,
                               const double *fy, double *fout, double *gout, const double *rho,
                               hipStream_t s);
// Pass C in observation mode: rho, v = u + F/(2 rho), F_x (any output may be
// null).  rho_in: pass A's density plane, read over segments (row_win) only.
hipError_t launch_rows_observe(const KParams &p, const double *f, const double *mu,
                               const double *fy, const double *rho_in, double *rho, double *vx,
                               double *vy, double *fx, hipStream_t s);
// g = the density groups of f.
hipError_t launch_density_groups(const KParams &p, const double *f, double *g, hipStream_t s);
// f = feq(rho0, u0) (u0 pointers may be null: rest).
hipError_t launch_init_feq(const KParams &p, const double *rho0, const double *ux0,
                           const double *uy0, double *f, hipStream_t s);
// In place: (ux, uy) <- (ux, uy) - (fx, fy) / (2 rho).
hipError_t launch_bare_velocity(const KParams &p, const double *rho, const double *fx,
                                const double *fy, double *ux, double *uy, hipStream_t s);
// rho of f compared with prev: per-block max |rho - prev| and a non-finite
// flag into partial[2*block]; prev <- rho.  Then one block folds the partials
// into out[0] (max) and out[1] (flag).
hipError_t launch_rho_delta(const KParams &p, const double *f, double *prev, double *partial,
                            int nblocks, double *out, hipStream_t s);
int rho_delta_blocks(const KParams &p);

// Block shapes for a mesh: rows per block, and columns per block for a
// requested strip width (clamped to what one block's LDS holds) and chunk
// length of the fast column solve (4, 8 or 16 nodes per thread).  Both pick
// the factorised-inverse kernels whenever the line allows it.
void set_row_shape(KParams *p);
void set_col_shape(KParams *p, int width, int chunk);
// The column pass over tiles: strips of `width` columns (4, 8 or 16) cut into
// tiles of rows, chunk 4, 8 or 16, each tile with a window above and below.
// False (p unchanged) if the columns are too short for a tile's windows or
// not a whole number of chunks.
bool set_col_tiles(KParams *p, int width, int chunk);
// Rows of one tile (in chunks) for a strip width and chunk length, and the
// window's chunks on each side.
int col_tile_chunks(int width, int lc);
int col_window_chunks(int lc);
// The column pass streamed down strips of `width` columns (8, 16 or 32; 16
// reads whole 128-byte lines of each row), one workgroup per strip walking
// down it in tiles of chunks (8 nodes where ny is a multiple of 8, else 4)
// with the three chained solves pipelined one tile apart.  False (p
// unchanged) where the mesh does not allow it: the pseudopotential model, nx
// not a multiple of the width, ny not a multiple of 4 or shorter than the
// window (168 rows with 8-node chunks, 144 with 4).
bool set_col_stream(KParams *p, int width);
bool col_stream_ok(const KParams &p, int width);
int col_stream_chunk(int ny);
// LDS of one streaming workgroup (bytes) for chunk length lc.
size_t col_stream_lds(int width, int lc);

// ---- batches of independent meshes ------------------------------------
// Device-side buffers of one mesh of a batch.
struct SimBuffers {
    double *f[2], *g[2];  // state A/B: distribution and its density groups
    double *rho, *mux, *mu, *fy;
};
// One workgroup of a batched pass: the mesh and its first row or column.
struct WorkItem {
    int sim, start;
};
// LDS of a batched row block holding rows rows of nx nodes (pass A, or the
// collision pass), and of a batched column block of col_elems nodes in
// chunks of lc for strips of at most wmax columns.
size_t batch_row_lds(int rows, int nx, bool collide);
size_t batch_col_lds(int col_elems, int lc, int wmax);
// Batched passes: rows use 256-thread workgroups (each mesh's rows_per_block
// rows of nx <= 1024 nodes); the column pass uses col_elems / lc threads
// (each mesh's cols_per_block = col_elems / ny columns), lc = 4 or 8.
hipError_t launch_batch_rows_rho(const KParams *kps, const SimBuffers *sb, const WorkItem *work,
                                 int nwork, int parity, size_t lds, hipStream_t s);
hipError_t launch_batch_cols_mu(const KParams *kps, const SimBuffers *sb, const WorkItem *work,
                                int nwork, int col_elems, int lc, int wmax, hipStream_t s);
// (mrt: every simulation of the batch uses the MRT collision of Eq. 4)
hipError_t launch_batch_rows_collide(const KParams *kps, const SimBuffers *sb,
                                     const WorkItem *work, int nwork, int parity, size_t lds,
                                     bool mrt, hipStream_t s);

// Fast-path kernels (kernels_iir.hip) and their eligibility.
bool iir_rows_ok(const KParams &p);
bool iir_cols_ok(const KParams &p, int chunk, int width);
hipError_t launch_rows_rho_iir(const KParams &p, const double *g, double *rho, double *mux,
                               hipStream_t s);
hipError_t launch_cols_mu_iir(const KParams &p, const double *rho, const double *mux, double *mu,
                              double *fy, hipStream_t s);
hipError_t launch_rows_collide_iir(const KParams &p, const double *f, const double *mu,
                                   const double *fy, double *fout, double *gout, double *o_rho,
                                   double *o_vx, double *o_vy, double *o_fx, bool observe,
                                   hipStream_t s);
// Row segments of kSegLen nodes (the last one ragged) for rows longer than
// kSegLen whose length is a whole number of 4-node chunks: one workgroup per
// segment, with the row derivatives taken over a window around it.  The
// collision pass (f in registers into fout, gout; F_x from the rho plane of
// pass A and the mu plane), pass A, and the observation pass.
bool iir_split_ok(const KParams &p);
hipError_t launch_collide_split_iir(const KParams &p, const double *f, const double *rho,
                                    const double *mu, const double *fy, double *fout,
                                    double *gout, hipStream_t s);
hipError_t launch_rows_rho_seg_iir(const KParams &p, const double *g, double *rho, double *mux,
                                   hipStream_t s);
hipError_t launch_observe_seg_iir(const KParams &p, const double *f, const double *rho,
                                  const double *mu, const double *fy, double *o_rho, double *o_vx,
                                  double *o_vy, double *o_fx, hipStream_t s);

}  // namespace cplbm
