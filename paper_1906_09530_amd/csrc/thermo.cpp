// Host-side thermodynamics; see thermo.hpp.
#include "thermo.hpp"

#include <cmath>

namespace cplbm {

// Each EOS of Sec. 3.2 splits as p0 = R T g(rho) - A h(rho).  The functions
// below give g, h and their first two rho-derivatives in closed form.
static void repulsive(const Eos &e, long double r, long double *g, long double *g1,
                      long double *g2)
{
    const long double b = e.b;
    if (e.kind == EOS_CS) {
        // g = (4/b) G(eta), G = (eta + eta^2 + eta^3 - eta^4)/(1 - eta)^3,
        // G' = (1 + 4 eta + 4 eta^2 - 4 eta^3 + eta^4)/(1 - eta)^4,
        // G'' = (8 + 20 eta - 4 eta^2)/(1 - eta)^5, eta = b rho / 4.
        long double eta = b * r / 4.0L, q = 1.0L - eta;
        long double q3 = q * q * q;
        *g = r * (1.0L + eta + eta * eta - eta * eta * eta) / q3;
        *g1 = (1.0L + 4.0L * eta + 4.0L * eta * eta - 4.0L * eta * eta * eta + eta * eta * eta * eta) /
              (q3 * q);
        *g2 = b / 4.0L * (8.0L + 20.0L * eta - 4.0L * eta * eta) / (q3 * q * q);
        return;
    }
    long double q = 1.0L - b * r;
    *g = r / q;
    *g1 = 1.0L / (q * q);
    *g2 = 2.0L * b / (q * q * q);
}

static void attractive(const Eos &e, long double r, long double *h, long double *h1,
                       long double *h2)
{
    const long double b = e.b;
    switch (e.kind) {
    case EOS_RK:
    case EOS_RKS: {  // h = rho^2 / (1 + b rho)
        long double s = 1.0L + b * r;
        *h = r * r / s;
        *h1 = r * (2.0L + b * r) / (s * s);
        *h2 = 2.0L / (s * s * s);
        return;
    }
    case EOS_PR: {  // h = rho^2 / D, D = 1 + 2 b rho - b^2 rho^2
        long double D = 1.0L + 2.0L * b * r - b * b * r * r;
        long double D1 = 2.0L * b * (1.0L - b * r);
        *h = r * r / D;
        *h1 = 2.0L * r * (1.0L + b * r) / (D * D);
        *h2 = 2.0L * ((1.0L + 2.0L * b * r) * D - 2.0L * r * (1.0L + b * r) * D1) / (D * D * D);
        return;
    }
    default:  // VdW, CS: h = rho^2
        *h = r * r;
        *h1 = 2.0L * r;
        *h2 = 2.0L;
        return;
    }
}

long double eos_p0(const Eos &e, long double T, long double A, long double rho)
{
    long double g, g1, g2, h, h1, h2;
    repulsive(e, rho, &g, &g1, &g2);
    attractive(e, rho, &h, &h1, &h2);
    return e.R * T * g - A * h;
}

long double eos_dp0(const Eos &e, long double T, long double A, long double rho)
{
    long double g, g1, g2, h, h1, h2;
    repulsive(e, rho, &g, &g1, &g2);
    attractive(e, rho, &h, &h1, &h2);
    return e.R * T * g1 - A * h1;
}

long double eos_mu0(const Eos &e, long double T, long double A, long double rho)
{
    const long double b = e.b, RT = e.R * T;
    switch (e.kind) {
    case EOS_VDW:
        return RT * (logl(rho / (1.0L - b * rho)) + 1.0L / (1.0L - b * rho)) - 2.0L * e.a * rho;
    case EOS_RK:
    case EOS_RKS:
        return RT * logl(rho / (1.0L - b * rho)) + RT / (1.0L - b * rho) -
               A / b * logl(1.0L + b * rho) - A * rho / (1.0L + b * rho);
    case EOS_PR: {
        const long double s2 = sqrtl(2.0L);
        return RT * logl(rho / (1.0L - b * rho)) -
               A / (2.0L * s2 * b) * logl((s2 - 1.0L + b * rho) / (s2 + 1.0L - b * rho)) +
               RT / (1.0L - b * rho) - A * rho / (1.0L + 2.0L * b * rho - b * b * rho * rho);
    }
    default: {  // CS
        long double eta = b * rho / 4.0L, q = 1.0L - eta;
        return RT * ((3.0L - eta) / (q * q * q) + logl(rho) + 1.0L) - 2.0L * e.a * rho;
    }
    }
}

long double eos_rho_max(const Eos &e) { return e.kind == EOS_CS ? 4.0L / e.b : 1.0L / e.b; }

long double eos_alpha(const Eos &e, long double T, long double Tc)
{
    if (e.kind == EOS_RK) return 1.0L / sqrtl(T);
    if (e.kind == EOS_RKS || e.kind == EOS_PR) {
        const long double w = e.omega;
        long double m = e.kind == EOS_RKS ? 0.480L + 1.574L * w - 0.176L * w * w
                                          : 0.37464L + 1.54226L * w - 0.26992L * w * w;
        long double s = 1.0L + m * (1.0L - sqrtl(T / Tc));
        return s * s;
    }
    return 1.0L;
}

// Root of f on [lo, hi] by bisection (f(lo), f(hi) of opposite sign).
template <class F>
static bool bisect(F f, long double lo, long double hi, long double *root, int iters = 200)
{
    long double flo = f(lo), fhi = f(hi);
    if (!(flo < 0) == !(fhi < 0)) return false;
    for (int it = 0; it < iters; ++it) {
        long double mid = 0.5L * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        long double fm = f(mid);
        if (!(fm < 0) == !(flo < 0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
    }
    *root = 0.5L * (lo + hi);
    return true;
}

bool eos_critical(const Eos &e, long double *Tc, long double *rhoc, long double *pc)
{
    // At fixed A the critical conditions R T g1 = A h1 and R T g2 = A h2
    // leave h1 g2 - h2 g1 = 0, a single equation in rho.
    auto phi = [&](long double r) {
        long double g, g1, g2, h, h1, h2;
        repulsive(e, r, &g, &g1, &g2);
        attractive(e, r, &h, &h1, &h2);
        return h1 * g2 - h2 * g1;
    };
    long double rmax = eos_rho_max(e), rc;
    if (!bisect(phi, rmax * 1e-9L, rmax * (1.0L - 1e-9L), &rc, 400)) return false;
    long double g, g1, g2, h, h1, h2;
    repulsive(e, rc, &g, &g1, &g2);
    attractive(e, rc, &h, &h1, &h2);
    long double q = e.a * h1 / (e.R * g1);  // = T_c alpha(T_c)^-1
    long double T = e.kind == EOS_RK ? powl(q, 2.0L / 3.0L) : q;
    long double A = e.kind == EOS_RK ? e.a / sqrtl(T) : e.a;
    *Tc = T;
    *rhoc = rc;
    *pc = eos_p0(e, T, A, rc);
    return true;
}

bool eos_maxwell(const Eos &e, long double T_r, long double *rho_g, long double *rho_l)
{
    if (!(T_r > 0.0L && T_r < 1.0L)) return false;
    long double Tc, rc, pc;
    if (!eos_critical(e, &Tc, &rc, &pc)) return false;
    const long double T = T_r * Tc;
    const long double A = e.a * eos_alpha(e, T, Tc);
    const long double rmax = eos_rho_max(e);
    auto p = [&](long double r) { return eos_p0(e, T, A, r); };
    auto dp = [&](long double r) { return eos_dp0(e, T, A, r); };
    auto mu = [&](long double r) { return eos_mu0(e, T, A, r); };
    // Spinodals: dp0/drho > 0 below s1, < 0 on (s1, s2) around rho_c, > 0 above s2.
    long double s1, s2;
    if (!bisect(dp, 0.0L, rc, &s1)) return false;
    if (!bisect(dp, rc, rmax * (1.0L - 1e-18L), &s2)) return false;
    const long double lgs1 = logl(s1);
    auto roots = [&](long double P, long double *g, long double *l) {
        long double lg;
        bool ok = bisect([&](long double x) { return p(expl(x)) - P; }, lgs1 - 2000.0L, lgs1, &lg);
        ok = ok && bisect([&](long double r) { return p(r) - P; }, s2, rmax * (1.0L - 1e-18L), l);
        *g = expl(lg);
        return ok;
    };
    long double Phi = p(s1), Plo = p(s2);
    long double lo = Plo > 0.0L ? logl(Plo) : logl(Phi) - 1400.0L, hi = logl(Phi);
    // Along an isotherm d mu = dp / rho: below the saturation pressure the
    // liquid branch has the higher mu, above it the lower one.
    long double g = 0, l = 0;
    for (int it = 0; it < 200; ++it) {
        long double mid = 0.5L * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (!roots(expl(mid), &g, &l)) return false;
        if (mu(l) - mu(g) > 0.0L)
            lo = mid;
        else
            hi = mid;
    }
    if (!roots(expl(0.5L * (lo + hi)), &g, &l)) return false;
    *rho_g = g;
    *rho_l = l;
    return true;
}

}  // namespace cplbm
