// Host driver of the library's host thermodynamics (critical points, the
// Maxwell construction, alpha(T), p0 and psi') for the address and
// undefined-behaviour sanitizers, over every EOS and a range of T/Tc.
#include <cmath>
#include <cstdio>

#include "../paper_1906_09530_amd/csrc/thermo.hpp"

int main()
{
    using namespace cplbm;
    int bad = 0;
    for (int kind = EOS_VDW; kind <= EOS_CS; ++kind) {
        Eos e{kind, kind == EOS_VDW ? 9.0L / 49 : (kind == EOS_CS ? 1.0L : 2.0L / 49),
              kind == EOS_CS ? 4.0L : 2.0L / 21, 1.0L, 0.344L};
        long double Tc, rc, pc;
        if (!eos_critical(e, &Tc, &rc, &pc)) { ++bad; continue; }
        for (long double tr = 0.3L; tr < 0.99L; tr += 0.1L) {
            long double g, l;
            if (!eos_maxwell(e, tr, &g, &l)) { ++bad; continue; }
            const long double T = tr * Tc, A = e.a * eos_alpha(e, T, Tc);
            const long double d = eos_mu0(e, T, A, g) - eos_mu0(e, T, A, l);
            const long double q = eos_p0(e, T, A, g) - eos_p0(e, T, A, l) + eos_dp0(e, T, A, g);
            if (!std::isfinite((double)d) || !std::isfinite((double)q)) ++bad;
        }
        (void)eos_rho_max(e);
    }
    std::printf(bad ? "sanitized thermo: %d failures\n" : "sanitized thermo: ok\n", bad);
    return bad ? 1 : 0;
}
