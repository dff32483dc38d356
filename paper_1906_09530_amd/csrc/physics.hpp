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
