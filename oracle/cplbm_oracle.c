/*
 * cplbm_oracle.c -- CPU oracle of the chemical-potential multiphase lattice
 * Boltzmann scheme of Wen, Zhao, Qiu, Ye and Shan, "Chemical-Potential
 * Multiphase Lattice Boltzmann Method with Superlarge Density Ratios"
 * (arXiv:1906.09530).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or helper with the GPU library.
 *
 * Everything is IEEE double precision, naive loops, no blocking or fusion.
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -o liboracle.so cplbm_oracle.c -lm
 * The same source built with -fopenmp runs the independent loops (lines of
 * the compact scheme, nodes of the pointwise steps, rows of the streaming)
 * on several threads.  Every line and node is computed by one thread in the
 * same order as in the serial build, so the results are bitwise identical. 
 *
 * Conventions (lattice units of the mesh space, Sec. 4.1):
 *   node index  y*nx + x, x in [0,nx), y in [0,ny);
 *   distribution field f[i][y][x], i = 0..8 (D2Q9, Sec. 2);
 *   the state stored is the pre-collision f_i(x,t).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the OpenMP build (n > 0 sets them); 1 for the serial build. */
int orc_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ---- D2Q9 lattice (Sec. 2, text after Eq. 2) ---------------------------- */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
#define CS2 (1.0 / 3.0)

/* ---- equations of state (Sec. 3.2) -------------------------------------- */
enum { EOS_VDW = 0, EOS_RK = 1, EOS_RKS = 2, EOS_PR = 3, EOS_CS = 4 };

typedef struct {
    int32_t nx, ny;
    int32_t bc_y;      /* 0: periodic in y; 1: half-way bounce-back walls */
    int32_t eos;       /* EOS_* */
    double wall_ux;    /* tangential velocity of both walls (moving frame) */
    double a, b, R;    /* EOS constants, momentum space */
    double T;          /* absolute temperature (momentum space) */
    double alpha_T;    /* alpha(T) of RK/RKS/PR; ignored by VdW and CS */
    double kappa;      /* surface-tension coefficient on the mesh (Eq. 33) */
    double tau;        /* BGK relaxation time (Eq. 1) */
    double k;          /* proportional coefficient (Eq. 25) */
    double mu_cap;     /* upper limit of the bulk chemical potential (Sec. 5.6) */
    double cfd_alpha;  /* alpha of the compact scheme (Eqs. 37-39) */
    int32_t collision; /* 0: BGK (Eq. 1); 1: MRT (Eq. 4) */
    int32_t force;     /* 0: chemical potential (Eq. 12); 1: pseudopotential (Sec. 5.1) */
    double s_e, s_eps, s_q;  /* MRT relaxation rates (Eq. 4); s_v = 1/tau */
    int32_t wetting;   /* walls: 0 neighbour-node chemical potential; 1 prescribed */
    double mu_wall;    /* prescribed wall chemical potential, momentum units */
} orc_params;

/* Temperature functions of the RK, RKS and PR EOS (Eqs. 16 and 18). */
double orc_alpha_T(int eos, double T, double Tc, double omega)
{
    if (eos == EOS_RK) return 1.0 / sqrt(T);
    if (eos == EOS_RKS) {
        double m = 0.480 + 1.574 * omega - 0.176 * omega * omega;
        double s = 1.0 + m * (1.0 - sqrt(T / Tc));
        return s * s;
    }
    if (eos == EOS_PR) {
        double m = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
        double s = 1.0 + m * (1.0 - sqrt(T / Tc));
        return s * s;
    }
    return 1.0;
}

/* Bulk pressure p0(rho): Eqs. 14, 16, 18, 20. */
double orc_p0(int eos, double a, double b, double R, double T, double al, double rho)
{
    switch (eos) {
    case EOS_VDW:
        return rho * R * T / (1.0 - b * rho) - a * rho * rho;
    case EOS_RK:
    case EOS_RKS:
        return rho * R * T / (1.0 - b * rho) - a * al * rho * rho / (1.0 + b * rho);
    case EOS_PR:
        return rho * R * T / (1.0 - b * rho) -
               a * al * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
    case EOS_CS: {
        double eta = b * rho / 4.0;
        return rho * R * T * (1.0 + eta + eta * eta - eta * eta * eta) /
                   ((1.0 - eta) * (1.0 - eta) * (1.0 - eta)) -
               a * rho * rho;
    }
    }
    return NAN;
}

/* Bulk chemical potential psi'(rho), i.e. the printed chemical potentials
 * without their -kappa*lap(rho) term: Eqs. 15, 17, 19, 21. */
double orc_mu0(int eos, double a, double b, double R, double T, double al, double rho)
{
    switch (eos) {
    case EOS_VDW:
        return R * T * (log(rho / (1.0 - b * rho)) + 1.0 / (1.0 - b * rho)) - 2.0 * a * rho;
    case EOS_RK:
    case EOS_RKS:
        return R * T * log(rho / (1.0 - b * rho)) + R * T / (1.0 - b * rho) -
               a * al / b * log(1.0 + b * rho) - a * al * rho / (1.0 + b * rho);
    case EOS_PR: {
        double s2 = sqrt(2.0);
        return R * T * log(rho / (1.0 - b * rho)) -
               a * al / (2.0 * s2 * b) * log((s2 - 1.0 + b * rho) / (s2 + 1.0 - b * rho)) +
               R * T / (1.0 - b * rho) - a * al * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
    }
    case EOS_CS: {
        double eta = b * rho / 4.0;
        return R * T * ((3.0 - eta) / ((1.0 - eta) * (1.0 - eta) * (1.0 - eta)) + log(rho) + 1.0) -
               2.0 * a * rho;
    }
    }
    return NAN;
}

/* The bounded bulk chemical potential.  Sec. 5.6: mu overflows once rho
 * reaches 1/b (or the packing limit of CS) and an upper limit keeps it
 * finite; the limit applies to psi'(rho) in momentum units, before the k^2
 * scaling of Eq. 33.  Outside the EOS domain, or when the formula is not a
 * finite number below the limit, the limit itself is used. */
double orc_mu0_capped(const orc_params *p, double rho)
{
    int outside = (p->eos == EOS_CS) ? (p->b * rho / 4.0 >= 1.0) : (p->b * rho >= 1.0);
    if (outside) return p->mu_cap;
    double m = orc_mu0(p->eos, p->a, p->b, p->R, p->T, p->alpha_T, rho);
    if (isnan(m)) return p->mu_cap;
    return m < p->mu_cap ? m : p->mu_cap;
}

/* ---- compact finite differences (Sec. 4.3, Eqs. 37-38) ------------------ */

/* Tridiagonal solve (Thomas algorithm) of sub[i] x[i-1] + dia[i] x[i] +
 * sup[i] x[i+1] = r[i], i = 0..n-1, without wrap-around. */
static void thomas(int n, const double *sub, const double *dia, const double *sup,
                   const double *r, double *x, double *cp, double *dp)
{
    cp[0] = sup[0] / dia[0];
    dp[0] = r[0] / dia[0];
    for (int i = 1; i < n; i++) {
        double m = dia[i] - sub[i] * cp[i - 1];
        cp[i] = sup[i] / m;
        dp[i] = (r[i] - sub[i] * dp[i - 1]) / m;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; i--) x[i] = dp[i] - cp[i] * x[i + 1];
}

/* First derivative of the periodic samples u[0..n-1] (spacing h = 1) by the
 * alpha-family compact scheme, Eq. 37 with the coefficients of Eq. 38:
 *   al d[i-1] + d[i] + al d[i+1] = a (u[i+1]-u[i-1])/2 + b (u[i+2]-u[i-2])/4,
 * indices modulo n.  The cyclic system is solved by the Thomas algorithm
 * plus a Sherman-Morrison correction for the two corner entries. n >= 3. */
void orc_cfm_line(int n, double al, const double *u, double *d)
{
    double ca = 2.0 * (al + 2.0) / 3.0, cb = (4.0 * al - 1.0) / 3.0;
    double *buf = (double *)malloc(sizeof(double) * 9 * (size_t)n);
    double *sub = buf, *dia = buf + n, *sup = buf + 2 * n, *r = buf + 3 * n;
    double *y = buf + 4 * n, *z = buf + 5 * n, *uu = buf + 6 * n;
    double *cp = buf + 7 * n, *dp = buf + 8 * n;
    for (int i = 0; i < n; i++) {
        int ip1 = (i + 1) % n, im1 = (i - 1 + n) % n;
        int ip2 = (i + 2) % n, im2 = (i - 2 + 2 * n) % n;
        r[i] = ca * (u[ip1] - u[im1]) / 2.0 + cb * (u[ip2] - u[im2]) / 4.0;
        sub[i] = al;
        dia[i] = 1.0;
        sup[i] = al;
        uu[i] = 0.0;
    }
    /* A = B + w v^T with the corners A[0][n-1] = A[n-1][0] = al moved into
     * w = (g, 0, .., 0, al), v = (1, 0, .., 0, al/g); g = -1. */
    double g = -1.0;
    dia[0] = 1.0 - g;
    dia[n - 1] = 1.0 - al * al / g;
    uu[0] = g;
    uu[n - 1] = al;
    thomas(n, sub, dia, sup, r, y, cp, dp);
    thomas(n, sub, dia, sup, uu, z, cp, dp);
    double vy = y[0] + al / g * y[n - 1];
    double vz = z[0] + al / g * z[n - 1];
    double fac = vy / (1.0 + vz);
    for (int i = 0; i < n; i++) d[i] = y[i] - fac * z[i];
    free(buf);
}

/* d/dx of a field along every row (x is always periodic). */
static void cfm_rows(const orc_params *p, const double *u, double *d)
{
    int nx = p->nx, ny = p->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++) orc_cfm_line(nx, p->cfd_alpha, u + (size_t)y * nx, d + (size_t)y * nx);
}

/* d/dy of a field along every column.  Periodic in y, or, between walls, on
 * the even extension of the column about the two wall planes (length 2 ny):
 * the ghost values mirror the fluid nodes, which gives the neighbour-node
 * value of the chemical-potential boundary condition of Sec. 5.5. */
static void cfm_cols(const orc_params *p, const double *u, double *d)
{
    int nx = p->nx, ny = p->ny;
    int n = p->bc_y ? 2 * ny : ny;
#pragma omp parallel for schedule(static)
    for (int x = 0; x < nx; x++) {
        double *line = (double *)malloc(sizeof(double) * 2 * n);
        double *dl = line + n;
        for (int y = 0; y < ny; y++) line[y] = u[(size_t)y * nx + x];
        if (p->bc_y)
            for (int y = 0; y < ny; y++) line[ny + y] = u[(size_t)(ny - 1 - y) * nx + x];
        orc_cfm_line(n, p->cfd_alpha, line, dl);
        for (int y = 0; y < ny; y++) d[(size_t)y * nx + x] = dl[y];
        free(line);
    }
}

/* d/dy of the chemical potential between walls that hold it at a prescribed
 * value u_w (the chemical-potential boundary condition of a wetting wall,
 * Sec. 5.5 and its ref. [45]): the column of u - u_w is extended oddly about
 * the two wall planes (length 2 ny), so that u takes the value u_w on the
 * walls, and differentiated as one periodic line. */
static void cfm_cols_wall_value(const orc_params *p, const double *u, double u_w, double *d)
{
    int nx = p->nx, ny = p->ny, n = 2 * ny;
#pragma omp parallel for schedule(static)
    for (int x = 0; x < nx; x++) {
        double *line = (double *)malloc(sizeof(double) * 2 * n);
        double *dl = line + n;
        for (int y = 0; y < ny; y++) line[y] = u[(size_t)y * nx + x] - u_w;
        for (int y = 0; y < ny; y++) line[ny + y] = -(u[(size_t)(ny - 1 - y) * nx + x] - u_w);
        orc_cfm_line(n, p->cfd_alpha, line, dl);
        for (int y = 0; y < ny; y++) d[(size_t)y * nx + x] = dl[y];
        free(line);
    }
}

/* Second derivative along columns: the first-derivative scheme applied twice
 * (Sec. 4.3).  Between walls both applications act on the extended line. */
static void cfm_cols2(const orc_params *p, const double *u, double *d2)
{
    int nx = p->nx, ny = p->ny;
    int n = p->bc_y ? 2 * ny : ny;
#pragma omp parallel for schedule(static)
    for (int x = 0; x < nx; x++) {
        double *line = (double *)malloc(sizeof(double) * 3 * n);
        double *d1 = line + n, *dd = line + 2 * n;
        for (int y = 0; y < ny; y++) line[y] = u[(size_t)y * nx + x];
        if (p->bc_y)
            for (int y = 0; y < ny; y++) line[ny + y] = u[(size_t)(ny - 1 - y) * nx + x];
        orc_cfm_line(n, p->cfd_alpha, line, d1);
        orc_cfm_line(n, p->cfd_alpha, d1, dd);
        for (int y = 0; y < ny; y++) d2[(size_t)y * nx + x] = dd[y];
        free(line);
    }
}

/* Column derivative of a field as the step computes it: the first
 * derivative (second = 0) or the scheme applied twice (second = 1), periodic
 * in y or on the even extension between walls. */
void orc_cfm_columns(const orc_params *p, const double *u, double *d, int second)
{
    if (second)
        cfm_cols2(p, u, d);
    else
        cfm_cols(p, u, d);
}

/* The same for a field held at u_w on the walls (odd extension of u - u_w). */
void orc_cfm_columns_wall_value(const orc_params *p, const double *u, double u_w, double *d)
{
    cfm_cols_wall_value(p, u, u_w, d);
}

/* ---- lattice Boltzmann pieces (Sec. 2) ---------------------------------- */

/* Equilibrium of Eq. 2 with c_s^2 = 1/3. */
double orc_feq(int i, double rho, double ux, double uy)
{
    double eu = EX[i] * ux + EY[i] * uy;
    double uu = ux * ux + uy * uy;
    return W[i] * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

/* Density and momentum of Eq. 3 at one node.  The x and y momentum sums are
 * grouped in opposite pairs so that mirror-symmetric populations give an
 * exact zero. */
void orc_node_moments(const double *fi, double *rho, double *jx, double *jy)
{
    double r = 0.0;
    for (int i = 0; i < 9; i++) r += fi[i];
    *rho = r;
    *jx = (fi[1] - fi[3]) + (fi[5] - fi[6]) + (fi[8] - fi[7]);
    *jy = (fi[2] - fi[4]) + (fi[5] - fi[8]) + (fi[6] - fi[7]);
}

/* Forced BGK collision at one node: Eq. 1 with the exact-difference force
 * term of Eq. 5, F_i = feq(rho, u + F/rho) - feq(rho, u). */
void orc_collide_node(const double *fi, double rho, double ux, double uy, double Fx, double Fy,
                      double tau, double *fout)
{
    double dux = Fx / rho, duy = Fy / rho;
    for (int i = 0; i < 9; i++) {
        double eq = orc_feq(i, rho, ux, uy);
        double eq2 = orc_feq(i, rho, ux + dux, uy + duy);
        fout[i] = fi[i] - (fi[i] - eq) / tau + (eq2 - eq);
    }
}

/* ---- multiple-relaxation-time collision (Eq. 4) -------------------------
 * m = M f are the velocity moments of D2Q9 in the order the relaxation
 * matrix S = diag(0, s_e, s_eps, 0, s_q, 0, s_q, s_v, s_v) refers to:
 * density rho, energy e, energy square eps, momentum j_x, energy flux q_x,
 * j_y, q_y, and the stresses p_xx, p_xy.  Each row is a polynomial in the
 * lattice velocity (e, eps and q from the orthogonalised powers of |e|^2):
 *   1, 3|e|^2 - 4, (9|e|^4 - 21|e|^2 + 8)/2, e_x, (3|e|^2 - 5) e_x, e_y,
 *   (3|e|^2 - 5) e_y, e_x^2 - e_y^2, e_x e_y. */
void orc_mrt_matrix(double *M)
{
    for (int i = 0; i < 9; i++) {
        double ex = EX[i], ey = EY[i], e2 = ex * ex + ey * ey;
        double row[9] = {1.0,
                         3.0 * e2 - 4.0,
                         (9.0 * e2 * e2 - 21.0 * e2 + 8.0) / 2.0,
                         ex,
                         (3.0 * e2 - 5.0) * ex,
                         ey,
                         (3.0 * e2 - 5.0) * ey,
                         ex * ex - ey * ey,
                         ex * ey};
        for (int k = 0; k < 9; k++) M[k * 9 + i] = row[k];
    }
}

/* The rows of M are mutually orthogonal, so M^-1 = M^T diag(1 / |M_k|^2). */
void orc_mrt_inverse(double *Minv)
{
    double M[81];
    orc_mrt_matrix(M);
    for (int k = 0; k < 9; k++) {
        double n2 = 0.0;
        for (int i = 0; i < 9; i++) n2 += M[k * 9 + i] * M[k * 9 + i];
        for (int i = 0; i < 9; i++) Minv[i * 9 + k] = M[k * 9 + i] / n2;
    }
}

/* Forced MRT collision at one node, Eq. 4 with the exact-difference force
 * term of Eq. 5: f* = f - M^-1 S (m - m_eq) + feq(rho, u + F/rho) - feq(rho, u),
 * with m_eq = M feq(rho, u) and S = diag(0, s_e, s_eps, 0, s_q, 0, s_q, 1/tau,
 * 1/tau). */
void orc_collide_node_mrt(const double *fi, double rho, double ux, double uy, double Fx,
                          double Fy, double tau, double s_e, double s_eps, double s_q,
                          double *fout)
{
    double M[81], Minv[81], eq[9], m[9], meq[9], dm[9];
    double S[9] = {0.0, s_e, s_eps, 0.0, s_q, 0.0, s_q, 1.0 / tau, 1.0 / tau};
    orc_mrt_matrix(M);
    orc_mrt_inverse(Minv);
    for (int i = 0; i < 9; i++) eq[i] = orc_feq(i, rho, ux, uy);
    for (int k = 0; k < 9; k++) {
        m[k] = 0.0;
        meq[k] = 0.0;
        for (int i = 0; i < 9; i++) {
            m[k] += M[k * 9 + i] * fi[i];
            meq[k] += M[k * 9 + i] * eq[i];
        }
        dm[k] = S[k] * (m[k] - meq[k]);
    }
    double dux = Fx / rho, duy = Fy / rho;
    for (int i = 0; i < 9; i++) {
        double back = 0.0;
        for (int k = 0; k < 9; k++) back += Minv[i * 9 + k] * dm[k];
        fout[i] = fi[i] - back + (orc_feq(i, rho, ux + dux, uy + duy) - eq[i]);
    }
}

/* ---- pseudopotential comparison model (Sec. 5.1) -------------------------
 * The Shan-Chen interaction force F = -G c_s^2 psi grad psi with G = -1 and
 * the effective mass taken from the EOS, here the mesh pressure k^2 p0
 * (Eq. 29): the force then carries the non-ideal part of that pressure,
 * k^2 p0 = rho c_s^2 + G c_s^2 psi^2 / 2, so
 * psi = sqrt(2 (rho c_s^2 - k^2 p0) / c_s^2) (0 where the argument is
 * negative).  The gradient of psi comes from the same compact scheme. */
double orc_sc_psi(const orc_params *p, double rho)
{
    double pr = p->k * p->k * orc_p0(p->eos, p->a, p->b, p->R, p->T, p->alpha_T, rho);
    double arg = 2.0 * (rho * CS2 - pr) / CS2;
    return arg > 0.0 ? sqrt(arg) : 0.0;
}

/* Scalar fields of one step, computed from the current f (Secs. 3-4):
 * rho, u, grad rho, the mesh chemical potential of Eq. 33 and the force of
 * Eq. 12.  Any output pointer may be NULL. */
typedef struct {
    double *rho, *jx, *jy, *dxr, *dyr, *mu, *fx, *fy;
} fields;

static void compute_fields(const orc_params *p, const double *f, fields *o)
{
    int nx = p->nx, ny = p->ny;
    size_t N = (size_t)nx * ny;
    double *dxxr = (double *)malloc(sizeof(double) * N);
    double *dyyr = (double *)malloc(sizeof(double) * N);
    double *dxm = (double *)malloc(sizeof(double) * N);
    double *dym = (double *)malloc(sizeof(double) * N);

    /* 1. moments (Eq. 3) */
#pragma omp parallel for schedule(static)
    for (size_t n = 0; n < N; n++) {
        double fi[9];
        for (int i = 0; i < 9; i++) fi[i] = f[(size_t)i * N + n];
        orc_node_moments(fi, &o->rho[n], &o->jx[n], &o->jy[n]);
    }
    if (p->force == 1) {
        /* pseudopotential model: F = c_s^2 psi grad psi (G = -1); the mu
         * output holds psi */
#pragma omp parallel for schedule(static)
        for (size_t n = 0; n < N; n++) o->mu[n] = orc_sc_psi(p, o->rho[n]);
        cfm_rows(p, o->mu, dxm);
        cfm_cols(p, o->mu, dym);
        cfm_rows(p, o->rho, o->dxr);
        cfm_cols(p, o->rho, o->dyr);
#pragma omp parallel for schedule(static)
        for (size_t n = 0; n < N; n++) {
            o->fx[n] = CS2 * o->mu[n] * dxm[n];
            o->fy[n] = CS2 * o->mu[n] * dym[n];
        }
        free(dxxr);
        free(dyyr);
        free(dxm);
        free(dym);
        return;
    }
    /* 2. density gradient and Laplacian by the compact scheme; the
     *    Laplacian is d/dx(d/dx rho) + d/dy(d/dy rho) (Sec. 4.3). */
    cfm_rows(p, o->rho, o->dxr);
    cfm_rows(p, o->dxr, dxxr);
    cfm_cols(p, o->rho, o->dyr);
    cfm_cols2(p, o->rho, dyyr);
    /* 3-4. mesh chemical potential, Eq. 33: k^2 psi'(rho) - kappa lap rho */
#pragma omp parallel for schedule(static)
    for (size_t n = 0; n < N; n++) {
        double m0 = orc_mu0_capped(p, o->rho[n]);
        o->mu[n] = p->k * p->k * m0 - p->kappa * (dxxr[n] + dyyr[n]);
    }
    /* 5. gradient of the chemical potential (between wetting walls the wall
     *    holds the prescribed value, k^2 mu_wall on the mesh) */
    cfm_rows(p, o->mu, dxm);
    if (p->bc_y && p->wetting)
        cfm_cols_wall_value(p, o->mu, p->k * p->k * p->mu_wall, dym);
    else
        cfm_cols(p, o->mu, dym);
    /* 6. nonideal force, Eq. 12: F = -rho grad mu + c_s^2 grad rho */
#pragma omp parallel for schedule(static)
    for (size_t n = 0; n < N; n++) {
        o->fx[n] = -o->rho[n] * dxm[n] + CS2 * o->dxr[n];
        o->fy[n] = -o->rho[n] * dym[n] + CS2 * o->dyr[n];
    }
    free(dxxr);
    free(dyyr);
    free(dxm);
    free(dym);
}

static void alloc_fields(fields *o, size_t N)
{
    double *m = (double *)malloc(sizeof(double) * 8 * N);
    o->rho = m;
    o->jx = m + N;
    o->jy = m + 2 * N;
    o->dxr = m + 3 * N;
    o->dyr = m + 4 * N;
    o->mu = m + 5 * N;
    o->fx = m + 6 * N;
    o->fy = m + 7 * N;
}

/* Streaming, the left side of Eq. 1: f_i(x + e_i) <- f*_i(x).  x is
 * periodic.  Between walls, a population whose target lies outside
 * [0, ny) returns to its own node in the opposite direction (half-way
 * bounce-back, walls at y = -1/2 and y = ny - 1/2); a wall moving with
 * velocity (U, 0) adds -2 w_i rho (e_i . U) / c_s^2 (Ladd's rule). */
void orc_stream(const orc_params *p, const double *fstar, const double *rho, double *fout)
{
    int nx = p->nx, ny = p->ny;
    size_t N = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            size_t n = (size_t)y * nx + x;
            for (int i = 0; i < 9; i++) {
                int tx = ((x + EX[i]) % nx + nx) % nx;
                int ty = y + EY[i];
                double v = fstar[(size_t)i * N + n];
                if (ty < 0 || ty >= ny) {
                    if (p->bc_y) {
                        double eu = EX[i] * p->wall_ux;
                        fout[(size_t)OPP[i] * N + n] = v - 2.0 * W[i] * rho[n] * eu / CS2;
                        continue;
                    }
                    ty = (ty + ny) % ny;
                }
                fout[(size_t)i * N + (size_t)ty * nx + tx] = v;
            }
        }
}

/* f = feq(rho0, u0) (initial state). */
void orc_init(const orc_params *p, const double *rho0, const double *ux0, const double *uy0,
              double *f)
{
    size_t N = (size_t)p->nx * p->ny;
    for (size_t n = 0; n < N; n++)
        for (int i = 0; i < 9; i++) f[(size_t)i * N + n] = orc_feq(i, rho0[n], ux0[n], uy0[n]);
}

/* One time step, Eq. 1 (or Eq. 4): moments, chemical potential, force,
 * collision, streaming.  f is replaced by f(t+1). */
void orc_step(const orc_params *p, double *f)
{
    size_t N = (size_t)p->nx * p->ny;
    fields o;
    alloc_fields(&o, N);
    compute_fields(p, f, &o);
    double *fs = (double *)malloc(sizeof(double) * 9 * N);
#pragma omp parallel for schedule(static)
    for (size_t n = 0; n < N; n++) {
        double fi[9], fo[9];
        for (int i = 0; i < 9; i++) fi[i] = f[(size_t)i * N + n];
        if (p->collision == 1)
            orc_collide_node_mrt(fi, o.rho[n], o.jx[n] / o.rho[n], o.jy[n] / o.rho[n], o.fx[n],
                                 o.fy[n], p->tau, p->s_e, p->s_eps, p->s_q, fo);
        else
            orc_collide_node(fi, o.rho[n], o.jx[n] / o.rho[n], o.jy[n] / o.rho[n], o.fx[n],
                             o.fy[n], p->tau, fo);
        for (int i = 0; i < 9; i++) fs[(size_t)i * N + n] = fo[i];
    }
    orc_stream(p, fs, o.rho, f);
    free(fs);
    free(o.rho);
}

void orc_run(const orc_params *p, double *f, int64_t nsteps)
{
    for (int64_t s = 0; s < nsteps; s++) orc_step(p, f);
}

/* Observables of the current state: rho, the physical velocity
 * v = u + F/(2 rho) (Sec. 2, after Eq. 5), and optionally the mesh chemical
 * potential and the force.  Output pointers may be NULL. */
void orc_moments(const orc_params *p, const double *f, double *rho, double *vx, double *vy,
                 double *mu, double *fx, double *fy)
{
    size_t N = (size_t)p->nx * p->ny;
    fields o;
    alloc_fields(&o, N);
    compute_fields(p, f, &o);
    for (size_t n = 0; n < N; n++) {
        if (rho) rho[n] = o.rho[n];
        if (vx) vx[n] = o.jx[n] / o.rho[n] + o.fx[n] / (2.0 * o.rho[n]);
        if (vy) vy[n] = o.jy[n] / o.rho[n] + o.fy[n] / (2.0 * o.rho[n]);
        if (mu) mu[n] = o.mu[n];
        if (fx) fx[n] = o.fx[n];
        if (fy) fy[n] = o.fy[n];
    }
    free(o.rho);
}

/* Run until max|rho(t) - rho(t - every)| < tol, checked every `every` steps.
 * Returns 0 when converged, 1 when max_steps is reached, -5 on a non-finite
 * density.  *steps receives the steps taken, *delta the last difference. */
int orc_run_until_converged(const orc_params *p, double *f, double tol, int64_t every,
                            int64_t max_steps, int64_t *steps, double *delta)
{
    size_t N = (size_t)p->nx * p->ny;
    double *prev = (double *)malloc(sizeof(double) * N);
    double *cur = (double *)malloc(sizeof(double) * N);
    int64_t done = 0;
    int status = 1;
    double d = INFINITY;
    orc_moments(p, f, prev, NULL, NULL, NULL, NULL, NULL);
    while (done < max_steps) {
        int64_t n = every;
        if (done + n > max_steps) n = max_steps - done;
        orc_run(p, f, n);
        done += n;
        orc_moments(p, f, cur, NULL, NULL, NULL, NULL, NULL);
        d = 0.0;
        int bad = 0;
        for (size_t q = 0; q < N; q++) {
            if (!isfinite(cur[q])) bad = 1;
            double e = fabs(cur[q] - prev[q]);
            if (e > d) d = e;
        }
        if (bad) {
            status = -5;
            d = NAN;
            break;
        }
        if (n == every && d < tol) {
            status = 0;
            break;
        }
        memcpy(prev, cur, sizeof(double) * N);
    }
    *steps = done;
    *delta = d;
    free(prev);
    free(cur);
    return status;
}
