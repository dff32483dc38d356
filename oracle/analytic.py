"""Thermodynamics of the chemical-potential model in arbitrary precision.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Written from Sec. 3 of Wen et al. (arXiv:1906.09530) with mpmath at 50
digits, so that none of it depends on FP64 rounding:

* the equations of state and their chemical potentials (Eqs. 14-21) and the
  free-energy density psi = rho psi' - p0 (Eq. 9);
* the critical point of each EOS (needed for T_r = T/T_c, Sec. 3.2);
* the Maxwell equal-area coexistence densities (Sec. 5.1);
* the planar-interface profile (Eqs. 22-24), interface width and surface
  tension, and their transformation to the mesh space (Sec. 4.1, Eq. 33).
"""
import functools

import mpmath as mp

from .lib import EOS_CS, EOS_PR, EOS_RK, EOS_RKS, EOS_VDW, OracleParams

mp.mp.dps = 40
_TOL = mp.mpf(10) ** -28

# EOS constants used throughout the paper (Sec. 3.2, after Eq. 21).
DEFAULT_AB = {
    EOS_VDW: (mp.mpf(9) / 49, mp.mpf(2) / 21),
    EOS_RK: (mp.mpf(2) / 49, mp.mpf(2) / 21),
    EOS_RKS: (mp.mpf(2) / 49, mp.mpf(2) / 21),
    EOS_PR: (mp.mpf(2) / 49, mp.mpf(2) / 21),
    EOS_CS: (mp.mpf(1), mp.mpf(4)),
}
OMEGA_WATER = mp.mpf("0.344")
OMEGA_METHANE = mp.mpf("0.011")


def _bisect(f, lo, hi, tol=mp.mpf(10) ** -45, maxit=400):
    """Root of f on [lo, hi] by bisection; f(lo) and f(hi) must differ in sign."""
    flo, fhi = f(lo), f(hi)
    if flo == 0:
        return lo
    if fhi == 0:
        return hi
    if (flo > 0) == (fhi > 0):
        raise ValueError("no sign change on the bracket")
    for _ in range(maxit):
        mid = (lo + hi) / 2
        fm = f(mid)
        if fm == 0:
            return mid
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
        if abs(hi - lo) <= tol * max(1, abs(mid)):
            break
    return (lo + hi) / 2


class EOS:
    """One equation of state with its constants (a, b, R, omega)."""

    def __init__(self, eos, a=None, b=None, R=1, omega=OMEGA_WATER):
        self.eos = eos
        da, db = DEFAULT_AB[eos]
        self.a = mp.mpf(da if a is None else a)
        self.b = mp.mpf(db if b is None else b)
        self.R = mp.mpf(R)
        self.omega = mp.mpf(omega)
        self._crit = None
        self._maxwell = {}

    # -- temperature functions, Eqs. 16 (RK, RKS) and 18 (PR) -------------
    def alpha(self, T, Tc=None):
        if self.eos == EOS_RK:
            return 1 / mp.sqrt(T)
        if self.eos in (EOS_RKS, EOS_PR):
            w = self.omega
            if self.eos == EOS_RKS:
                m = mp.mpf("0.480") + mp.mpf("1.574") * w - mp.mpf("0.176") * w * w
            else:
                m = mp.mpf("0.37464") + mp.mpf("1.54226") * w - mp.mpf("0.26992") * w * w
            return (1 + m * (1 - mp.sqrt(T / Tc))) ** 2
        return mp.mpf(1)

    # -- bulk pressure, Eqs. 14, 16, 18, 20 --------------------------------
    def p0(self, rho, T, al):
        a, b, R = self.a, self.b, self.R
        if self.eos == EOS_VDW:
            return rho * R * T / (1 - b * rho) - a * rho ** 2
        if self.eos in (EOS_RK, EOS_RKS):
            return rho * R * T / (1 - b * rho) - a * al * rho ** 2 / (1 + b * rho)
        if self.eos == EOS_PR:
            return rho * R * T / (1 - b * rho) - a * al * rho ** 2 / (1 + 2 * b * rho - (b * rho) ** 2)
        e = b * rho / 4
        return rho * R * T * (1 + e + e ** 2 - e ** 3) / (1 - e) ** 3 - a * rho ** 2

    # -- bulk chemical potential psi'(rho), Eqs. 15, 17, 19, 21 -------------
    def mu0(self, rho, T, al):
        a, b, R = self.a, self.b, self.R
        if self.eos == EOS_VDW:
            return R * T * (mp.log(rho / (1 - b * rho)) + 1 / (1 - b * rho)) - 2 * a * rho
        if self.eos in (EOS_RK, EOS_RKS):
            return (R * T * mp.log(rho / (1 - b * rho)) + R * T / (1 - b * rho)
                    - a * al / b * mp.log(1 + b * rho) - a * al * rho / (1 + b * rho))
        if self.eos == EOS_PR:
            s2 = mp.sqrt(2)
            return (R * T * mp.log(rho / (1 - b * rho))
                    - a * al / (2 * s2 * b) * mp.log((s2 - 1 + b * rho) / (s2 + 1 - b * rho))
                    + R * T / (1 - b * rho) - a * al * rho / (1 + 2 * b * rho - (b * rho) ** 2))
        e = b * rho / 4
        return R * T * ((3 - e) / (1 - e) ** 3 + mp.log(rho) + 1) - 2 * a * rho

    # -- free-energy density consistent with mu0, from Eq. 9 ----------------
    def psi(self, rho, T, al):
        return rho * self.mu0(rho, T, al) - self.p0(rho, T, al)

    def rho_max(self):
        """Upper end of the EOS domain (1/b, or the CS packing limit 4/b)."""
        return 4 / self.b if self.eos == EOS_CS else 1 / self.b

    # -- critical point: dp/drho = d2p/drho2 = 0 ----------------------------
    def critical_point(self):
        """(T_c, rho_c, p_c).  alpha(T_c) = 1 for RKS and PR by construction
        of their temperature functions; RK keeps alpha = T^-1/2."""
        if self._crit is not None:
            return self._crit

        def al_at(T):
            return 1 / mp.sqrt(T) if self.eos == EOS_RK else mp.mpf(1)

        def eqs(rho, T):
            f = lambda r: self.p0(r, T, al_at(T))  # noqa: E731
            return [mp.diff(f, rho, 1), mp.diff(f, rho, 2)]

        a, b = self.a, self.b
        guess = {
            EOS_VDW: (1 / (3 * b), 8 * a / (27 * b)),
            EOS_PR: (mp.mpf("0.2531") / b, mp.mpf("0.1701") * a / b),
            EOS_RKS: (mp.mpf("0.2599") / b, mp.mpf("0.2027") * a / b),
            EOS_RK: (mp.mpf("0.2599") / b, (mp.mpf("0.2027") * a / b) ** (mp.mpf(2) / 3)),
            EOS_CS: (mp.mpf("0.5218") / b, mp.mpf("0.3773") * a / b),
        }[self.eos]
        rc, Tc = mp.findroot(eqs, guess, tol=mp.mpf(10) ** -40)
        pc = self.p0(rc, Tc, al_at(Tc))
        self._crit = (Tc, rc, pc)
        return self._crit

    def temperature(self, T_r):
        """Absolute temperature T = T_r T_c and alpha(T)."""
        Tc = self.critical_point()[0]
        T = mp.mpf(T_r) * Tc
        return T, self.alpha(T, Tc)

    # -- Maxwell equal-area construction (Sec. 5.1) --------------------------
    def spinodals(self, T, al):
        """The two zeros of dp0/drho below the critical temperature: dp0/drho
        is positive below s1, negative on (s1, s2) (which holds rho_c) and
        positive again above s2."""
        f = lambda r: self.p0(r, T, al)  # noqa: E731
        dp = lambda r: mp.diff(f, r)  # noqa: E731
        rc = self.critical_point()[1]
        lo = _bisect(lambda lr: dp(mp.exp(lr)), mp.log(rc) - 60, mp.log(rc))
        hi = _bisect(dp, rc, self.rho_max() * (1 - mp.mpf("1e-25")))
        return mp.exp(lo), hi

    def maxwell(self, T_r):
        """Coexistence densities (rho_g, rho_l): equal mu0 and equal p0."""
        key = float(T_r)
        if key not in self._maxwell:
            self._maxwell[key] = self._maxwell_solve(T_r)
        return self._maxwell[key]

    def _maxwell_solve(self, T_r):
        T, al = self.temperature(T_r)
        p = lambda r: self.p0(r, T, al)  # noqa: E731
        mu = lambda r: self.mu0(r, T, al)  # noqa: E731
        s1, s2 = self.spinodals(T, al)
        rmax = self.rho_max()

        def roots(P):
            # gas branch: p increases on (0, s1); liquid branch on (s2, rmax)
            g = _bisect(lambda lr: p(mp.exp(lr)) - P, mp.log(s1) - 700, mp.log(s1), tol=_TOL)
            l = _bisect(lambda r: p(r) - P, s2, rmax * (1 - mp.mpf("1e-40")), tol=_TOL)
            return mp.exp(g), l

        Phi = p(s1)
        Plo = max(p(s2), mp.mpf(0))
        # bisection on log P between the spinodal pressures.  Along the
        # isotherm d mu = dp / rho, so below the saturation pressure the
        # liquid root has the higher mu0 and above it the lower one.
        lo = mp.log(Plo) if Plo > 0 else mp.log(Phi) - 200
        hi = mp.log(Phi)
        while hi - lo > _TOL * max(1, abs(hi)):
            mid = (lo + hi) / 2
            g, l = roots(mp.exp(mid))
            if mu(l) - mu(g) > 0:
                lo = mid
            else:
                hi = mid
        return roots(mp.exp((lo + hi) / 2))

    # -- planar interface, Eqs. 22-24 ---------------------------------------
    def delta_omega(self, rho, T, al, rho_b, mu_b):
        """psi(rho) - psi(rho_b) - mu_b (rho - rho_b), the right side of Eq. 22."""
        return self.psi(rho, T, al) - self.psi(rho_b, T, al) - mu_b * (rho - rho_b)

    def interface(self, T_r):
        """Momentum-space interface quantities at kappa = 1: the profile
        y(rho) of Eq. 23 (origin at (rho_g + rho_l)/2), the width
        (rho_l - rho_g)/max rho' (rho' from Eq. 24) and the surface tension
        sigma = int kappa rho'^2 dy = int sqrt(2 kappa dOmega) drho."""
        T, al = self.temperature(T_r)
        rg, rl = self.maxwell(T_r)
        mub = self.mu0(rg, T, al)
        dO = lambda r: self.delta_omega(r, T, al, rg, mub)  # noqa: E731
        slope = lambda r: mp.sqrt(2 * dO(r))  # noqa: E731
        sigma = mp.quad(slope, [rg, (rg + rl) / 2, rl])
        # max slope: d(dOmega)/drho = mu0(rho) - mu_b = 0 at the maximum of dOmega
        s1, s2 = self.spinodals(T, al)
        rstar = _bisect(lambda r: self.mu0(r, T, al) - mub, s1, s2)
        width = (rl - rg) / slope(rstar)
        r0 = (rg + rl) / 2

        def y_of_rho(r):
            return mp.quad(lambda s: 1 / slope(s), [r0, r])

        return {"T": T, "alpha": al, "rho_g": rg, "rho_l": rl, "mu_b": mub,
                "sigma1": sigma, "width1": width, "y_of_rho": y_of_rho,
                "drho_dy": slope, "rho_star": rstar}

    def laplace_pair(self, T_r, radius, kappa_hat, k):
        """Bulk densities of a drop of radius R (mesh nodes) in equilibrium
        with its vapour: equal mu0 and k^2 [p0(rho_in) - p0(rho_out)] =
        sigma_mesh / R (Eq. 40 in the mesh space), with sigma_mesh =
        k sqrt(kappa_hat) sigma1."""
        it = self.interface(T_r)
        T, al = it["T"], it["alpha"]
        sig = k * mp.sqrt(kappa_hat) * it["sigma1"]
        p = lambda r: self.p0(r, T, al)  # noqa: E731
        mu = lambda r: self.mu0(r, T, al)  # noqa: E731
        sol = mp.findroot(lambda lg, rl: [mu(mp.exp(lg)) - mu(rl),
                                          k * k * (p(rl) - p(mp.exp(lg))) - sig / radius],
                          (mp.log(it["rho_g"]), it["rho_l"]), tol=mp.mpf(10) ** -40)
        return mp.exp(sol[0]), sol[1]


# MRT relaxation rates used in the paper (Sec. 2, after Eq. 4)
MRT_RATES = (1.64, 1.54, 1.9)


def params(eos, T_r, nx, ny, *, kappa, tau, k, mu_cap=float("inf"), cfd_alpha=1.0 / 3.0,
           bc_y=0, wall_ux=0.0, omega=None, a=None, b=None, R=1, collision=0, force=0,
           rates=MRT_RATES, wetting=0, mu_wall=0.0):
    """OracleParams for the C oracle, with T = T_r T_c and alpha(T) from this
    module's critical point.  collision: 0 BGK (Eq. 1), 1 MRT (Eq. 4) with
    rates (s_e, s_eps, s_q); force: 0 chemical potential (Eq. 12), 1
    pseudopotential comparison model (Sec. 5.1); wetting: walls hold the
    chemical potential at mu_wall (momentum units) instead of the
    neighbour-node value."""
    e = EOS(eos, a=a, b=b, R=R, omega=OMEGA_WATER if omega is None else omega)
    T, al = e.temperature(T_r)
    return OracleParams(nx=nx, ny=ny, bc_y=bc_y, eos=eos, wall_ux=wall_ux, a=float(e.a),
                        b=float(e.b), R=float(e.R), T=float(T), alpha_T=float(al),
                        kappa=kappa, tau=tau, k=k, mu_cap=mu_cap, cfd_alpha=cfd_alpha,
                        collision=collision, force=force, s_e=rates[0], s_eps=rates[1],
                        s_q=rates[2], wetting=wetting, mu_wall=mu_wall)


@functools.lru_cache(maxsize=None)
def coexistence(eos, T_r, omega=None):
    """Maxwell coexistence densities (rho_g, rho_l) as doubles, for the
    default constants of each EOS (Sec. 3.2): inputs of seeded test fields."""
    g, l = EOS(eos, omega=OMEGA_WATER if omega is None else omega).maxwell(T_r)
    return float(g), float(l)
