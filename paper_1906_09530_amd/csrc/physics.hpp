// Pointwise physics shared by the kernels: D2Q9 lattice, moments, the
// equilibrium and the bounded bulk chemical potential (arXiv:1906.09530).
#pragma once

#include "kernels.hpp"
#include "lnx.hpp"

namespace cplbm {
namespace phys {

// D2Q9 (Sec. 2)
constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr double WT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
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

// The nine populations at offset `node` of a state whose planes lie `stride`
// apart.
__device__ __forceinline__ void load9(const double *__restrict__ f, size_t stride, size_t node,
                                      double (&fi)[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) fi[i] = f[i * stride + node];
}

// Equilibrium of Eq. 2 with c_s^2 = 1/3.
__device__ __forceinline__ double feq(int i, double rho, double ux, double uy, double uu)
{
    const double eu = EX[i] * ux + EY[i] * uy;
    return WT[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

// Multiple-relaxation-time collision (Eq. 4) in the moment basis whose
// relaxation matrix the paper gives as S = diag(0, s_e, s_eps, 0, s_q, 0,
// s_q, s_v, s_v): moments (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy) of
// D2Q9.  The rows are mutually orthogonal, so M^-1 = M^T diag(1/|M_k|^2).
// mrt_row(k, i) is M_{k i} of the six relaxed moments, k = 0..5 for
// (e, eps, q_x, q_y, p_xx, p_xy); |M_k|^2 = 36, 36, 12, 12, 4, 4.
constexpr double mrt_row(int k, int i)
{
    const int ex = EX[i], ey = EY[i], e2 = ex * ex + ey * ey;
    return k == 0   ? -4.0 + 3.0 * e2
           : k == 1 ? 4.0 - 10.5 * e2 + 4.5 * e2 * e2
           : k == 2 ? ex * (3.0 * e2 - 5.0)
           : k == 3 ? ey * (3.0 * e2 - 5.0)
           : k == 4 ? double(ex * ex - ey * ey)
                    : double(ex * ey);
}

// The relaxed moments' departures from equilibrium, weighted for the
// inverse transform: d_k = s_k (m_k - m_k^eq) / |M_k|^2 (p.mrt_w = s_k /
// |M_k|^2).  m^eq are the moments of the equilibrium of Eq. 2:
// e = rho(-2 + 3u^2), eps = rho(1 - 3u^2), q = -rho u, p_xx = rho(ux^2 - uy^2),
// p_xy = rho ux uy.
__device__ __forceinline__ void mrt_departures(const KParams &p, const double (&q)[9], double rho,
                                               double jx, double jy, double ux, double uy,
                                               double (&d)[6])
{
    double m[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            if (mrt_row(k, i) != 0.0) s += mrt_row(k, i) * q[i];
        m[k] = s;
    }
    const double uu = ux * ux + uy * uy;
    const double meq[6] = {rho * (-2.0 + 3.0 * uu), rho * (1.0 - 3.0 * uu), -jx, -jy,
                           rho * (ux * ux - uy * uy), rho * (ux * uy)};
#pragma unroll
    for (int k = 0; k < 6; ++k) d[k] = p.mrt_w[k] * (m[k] - meq[k]);
}

// Post-collision population i without the force term: f_i - (M^-1 S (m - m^eq))_i.
__device__ __forceinline__ double mrt_relax(int i, double fi, const double (&d)[6])
{
    double r = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        if (mrt_row(k, i) != 0.0) r += mrt_row(k, i) * d[k];
    return fi - r;
}

// Bulk pressure p0(rho) of Eqs. 14, 16, 18, 20 (momentum units).
__device__ __forceinline__ double p0_eos(const KParams &p, double rho)
{
    const double br = p.b * rho, RT = p.RT, A = p.A;
    switch (p.eos) {
    case 0: return rho * RT / (1.0 - br) - p.a * rho * rho;
    case 1:
    case 2: return rho * RT / (1.0 - br) - A * rho * rho / (1.0 + br);
    case 3: return rho * RT / (1.0 - br) - A * rho * rho / (1.0 + 2.0 * br - br * br);
    default: {
        const double eta = 0.25 * br, q = 1.0 - eta;
        return rho * RT * (1.0 + eta + eta * eta - eta * eta * eta) / (q * q * q) -
               p.a * rho * rho;
    }
    }
}

// Effective mass of the pseudopotential comparison model (Sec. 5.1), from
// the mesh pressure k^2 p0 (Eq. 29) with G = -1: the interaction force
// -G c_s^2 psi grad psi then carries the pressure k^2 p0 - rho c_s^2, so
// psi = sqrt(2 (rho c_s^2 - k^2 p0) / c_s^2), taken as 0 where the root's
// argument is negative.
__device__ __forceinline__ double sc_psi(const KParams &p, double rho)
{
    const double a = 2.0 * rho - 6.0 * (p.k2 * p0_eos(p, rho));
    return a > 0.0 ? sqrt(a) : 0.0;
}

// psi'(rho) of Eqs. 15, 17, 19, 21, bounded by the upper limit (Sec. 5.6):
// outside the EOS domain, or when the formula gives NaN, the limit is used.
__device__ __forceinline__ double mu0_capped(const KParams &p, double rho)
{
    const double b = p.b, RT = p.RT, A = p.A;
    const bool outside = (p.eos == 4) ? (b * rho * 0.25 >= 1.0) : (b * rho >= 1.0);
    if (outside) return p.mu_cap;
    double m;
    const double br = b * rho;
    switch (p.eos) {
    case 0: {  // van der Waals
        const double iv = 1.0 / (1.0 - br);
        m = RT * (lnx(rho * iv) + iv) - 2.0 * p.a * rho;
        break;
    }
    case 1:
    case 2: {  // Redlich-Kwong, Soave-Redlich-Kwong; eos_c1 = A / b
        // one reciprocal for both denominators, 1 - b rho and 1 + b rho
        const double d1 = 1.0 - br, d2 = 1.0 + br;
        const double inv = 1.0 / (d1 * d2);
        const double iv = d2 * inv;
        m = RT * lnx(rho * iv) + RT * iv - p.eos_c1 * lnx(d2) - A * rho * (d1 * inv);
        break;
    }
    case 3: {  // Peng-Robinson; eos_c1 = A / (2 sqrt(2) b)
        // one reciprocal for the three denominators 1 - b rho, sqrt2 + 1 - b rho
        // and 1 + 2 b rho - (b rho)^2 (all positive inside the domain)
        const double s2 = 1.4142135623730950488;
        const double d1 = 1.0 - br, d2 = s2 + 1.0 - br, d3 = 1.0 + 2.0 * br - br * br;
        const double inv = 1.0 / (d1 * d2 * d3);
        const double iv = d2 * d3 * inv;
        m = RT * lnx(rho * iv) - p.eos_c1 * lnx((s2 - 1.0 + br) * (d1 * d3 * inv)) + RT * iv -
            A * rho * (d1 * d2 * inv);
        break;
    }
    default: {  // Carnahan-Starling
        const double eta = br * 0.25, q = 1.0 - eta;
        m = RT * ((3.0 - eta) / (q * q * q) + lnx(rho) + 1.0) - 2.0 * p.a * rho;
        break;
    }
    }
    if (isnan(m)) return p.mu_cap;
    return m < p.mu_cap ? m : p.mu_cap;
}

}  // namespace phys
}  // namespace cplbm
