// Host-side thermodynamics of the equations of state of Sec. 3.2 (arXiv:1906.09530):
// critical points, temperature functions alpha(T) and the Maxwell
// construction.  Long double, analytic derivatives, bracketed bisection.
#pragma once

namespace cplbm {

enum { EOS_VDW = 0, EOS_RK = 1, EOS_RKS = 2, EOS_PR = 3, EOS_CS = 4 };

struct Eos {
    int kind;
    long double a, b, R, omega;
};

// p0 = R T g(rho) - A h(rho), A = a alpha(T) (Eqs. 14, 16, 18, 20).
long double eos_p0(const Eos &e, long double T, long double A, long double rho);
// d p0 / d rho
long double eos_dp0(const Eos &e, long double T, long double A, long double rho);
// psi'(rho), the printed chemical potentials without the gradient term
// (Eqs. 15, 17, 19, 21).
long double eos_mu0(const Eos &e, long double T, long double A, long double rho);
// Upper end of the EOS domain: 1/b, or 4/b for Carnahan-Starling.
long double eos_rho_max(const Eos &e);

// alpha(T): 1/sqrt(T) (RK), the Soave and Peng-Robinson functions of T/T_c
// (RKS, PR), 1 otherwise.
long double eos_alpha(const Eos &e, long double T, long double Tc);

// Critical point with alpha(T_c) = 1 (RKS, PR) or alpha = T^-1/2 (RK).
// Returns false if the bracketing fails.
bool eos_critical(const Eos &e, long double *Tc, long double *rhoc, long double *pc);

// Coexistence densities at T = T_r T_c.  Returns false outside 0 < T_r < 1.
bool eos_maxwell(const Eos &e, long double T_r, long double *rho_g, long double *rho_l);

}  // namespace cplbm
