"""Pins of the oracle's thermodynamics (Sec. 3.2 and Sec. 5.1 of the paper).

Each test checks the oracle against something other than itself: a
thermodynamic identity, a textbook critical point, an independent quadrature,
a limit, or a number the paper prints.
"""
import json
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
from oracle import analytic as A

ALL = [A.EOS_VDW, A.EOS_RK, A.EOS_RKS, A.EOS_PR, A.EOS_CS]
NAMES = {A.EOS_VDW: "VdW", A.EOS_RK: "RK", A.EOS_RKS: "RKS", A.EOS_PR: "PR", A.EOS_CS: "CS"}


@pytest.mark.parametrize("eos", ALL)
def test_gibbs_duhem(eos):
    """Eq. 9 gives dp0/drho = rho d(psi')/drho: the printed chemical
    potentials (Eqs. 15, 17, 19, 21) must be consistent with their EOS
    (Eqs. 14, 16, 18, 20).  Any typo in either side breaks this."""
    e = A.EOS(eos)
    T, al = e.temperature(0.6)
    for frac in ["0.001", "0.05", "0.2", "0.5", "0.8"]:
        rho = mp.mpf(frac) * e.rho_max()
        dp = mp.diff(lambda r: e.p0(r, T, al), rho)
        dmu = mp.diff(lambda r: e.mu0(r, T, al), rho)
        assert abs(dp - rho * dmu) <= mp.mpf(10) ** -25 * (abs(dp) + 1e-30)


@pytest.mark.parametrize("eos", ALL)
def test_c_oracle_eos_matches_arbitrary_precision(eos):
    """The C oracle's p0 and psi' (the ones the scheme uses) agree with the
    50-digit versions that the identities above pin."""
    e = A.EOS(eos)
    T, al = e.temperature(0.55)
    Tc = e.critical_point()[0]
    assert oracle.alpha_T(eos, float(T), float(Tc), float(e.omega)) == pytest.approx(
        float(al), rel=1e-15)
    for frac in [1e-6, 1e-3, 0.03, 0.3, 0.7, 0.95]:
        rho = frac * float(e.rho_max())
        pc = oracle.p0(eos, float(e.a), float(e.b), 1.0, float(T), float(al), rho)
        mc = oracle.mu0(eos, float(e.a), float(e.b), 1.0, float(T), float(al), rho)
        pm = e.p0(mp.mpf(rho), T, al)
        mm = e.mu0(mp.mpf(rho), T, al)
        assert abs(pc - float(pm)) <= 1e-13 * max(abs(float(pm)), 1e-12)
        assert abs(mc - float(mm)) <= 1e-13 * max(abs(float(mm)), 1.0)


def test_eos_constants_are_the_printed_ones(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "paper_printed.json")))["eos_constants"]
    for eos, key in [(A.EOS_VDW, "VdW"), (A.EOS_PR, "PR"), (A.EOS_RKS, "RKS"), (A.EOS_CS, "CS")]:
        e = A.EOS(eos)
        assert e.a == mp.mpf(g[key]["a"][0]) / g[key]["a"][1]
        assert e.b == mp.mpf(g[key]["b"][0]) / g[key]["b"][1]
    assert A.OMEGA_WATER == mp.mpf(str(g["omega_water"]))


def test_critical_point_vdw_closed_form():
    """VdW: T_c = 8a/(27 R b), rho_c = 1/(3b), Z_c = 3/8."""
    e = A.EOS(A.EOS_VDW)
    Tc, rc, pc = e.critical_point()
    assert abs(Tc - 8 * e.a / (27 * e.b)) < mp.mpf(10) ** -30
    assert abs(rc - 1 / (3 * e.b)) < mp.mpf(10) ** -30
    assert abs(pc / (rc * Tc) - mp.mpf(3) / 8) < mp.mpf(10) ** -30


@pytest.mark.parametrize("eos", [A.EOS_RKS, A.EOS_RK])
def test_critical_point_redlich_kwong_closed_form(eos):
    """Redlich-Kwong family: b rho_c = 2^(1/3) - 1 and Z_c = 1/3; with
    Omega_b/Omega_a = 3 (2^(1/3) - 1)^2, R T_c = 3 (2^(1/3)-1)^2 a alpha/b,
    alpha(T_c) = 1 for RKS and T_c^(-1/2) for RK."""
    e = A.EOS(eos)
    Tc, rc, pc = e.critical_point()
    c = 2 ** (mp.mpf(1) / 3) - 1
    assert abs(e.b * rc - c) < mp.mpf(10) ** -30
    assert abs(pc / (rc * Tc) - mp.mpf(1) / 3) < mp.mpf(10) ** -30
    rhs = 3 * c * c * e.a / e.b
    lhs = Tc ** mp.mpf(1.5) if eos == A.EOS_RK else Tc
    assert abs(lhs / rhs - 1) < mp.mpf(10) ** -30


def test_critical_point_peng_robinson_textbook():
    """PR: Z_c = 0.3074013, Omega_a = 0.45723553, Omega_b = 0.07779607 (the
    standard Peng-Robinson constants), so T_c = (Omega_b/Omega_a) a/(R b)."""
    e = A.EOS(A.EOS_PR)
    Tc, rc, pc = e.critical_point()
    assert float(pc / (rc * Tc)) == pytest.approx(0.3074013087, rel=1e-9)
    assert float(Tc) == pytest.approx(0.0777960739 / 0.4572355289 * float(e.a / e.b), rel=1e-9)
    assert float(e.b * pc / Tc) == pytest.approx(0.0777960739, rel=1e-9)


def test_critical_point_carnahan_starling_literature():
    """CS with a van der Waals attraction: eta_c = b rho_c / 4 = 0.1304,
    Z_c = 0.3590, R T_c b / a = 0.3773 (literature values to 4 digits)."""
    e = A.EOS(A.EOS_CS)
    Tc, rc, pc = e.critical_point()
    assert float(e.b * rc / 4) == pytest.approx(0.1304, abs=1e-4)
    assert float(pc / (rc * Tc)) == pytest.approx(0.3590, abs=1e-4)
    assert float(Tc * e.b / e.a) == pytest.approx(0.3773, abs=1e-4)


@pytest.mark.parametrize("eos,T_r", [(A.EOS_VDW, 0.6), (A.EOS_PR, 0.5), (A.EOS_RKS, 0.4),
                                      (A.EOS_CS, 0.7), (A.EOS_CS, 0.35), (A.EOS_RK, 0.8)])
def test_maxwell_equal_area(eos, T_r):
    """Coexistence satisfies the equal-area rule in the specific volume,
    int_{v_l}^{v_g} p0 dv = p_sat (v_g - v_l), evaluated here by direct
    quadrature -- a route independent of the equal-mu condition the
    solver uses."""
    e = A.EOS(eos)
    T, al = e.temperature(T_r)
    rg, rl = e.maxwell(T_r)
    psat = e.p0(rl, T, al)
    assert abs(e.p0(rg, T, al) - psat) <= mp.mpf(10) ** -20 * abs(psat)
    vl, vg = 1 / rl, 1 / rg
    # split at the spinodals (kinks of the integrand's behaviour)
    s1, s2 = e.spinodals(T, al)
    pts = [vl, 1 / s2, 1 / s1, vg]
    integral = mp.quad(lambda v: e.p0(1 / v, T, al), pts)
    area = psat * (vg - vl)
    assert abs(integral - area) <= mp.mpf(10) ** -18 * abs(area)


def test_maxwell_near_critical_limit():
    """T_r -> 1: both branches approach rho_c, the gap closing like
    sqrt(1 - T_r) (mean-field exponent 1/2)."""
    e = A.EOS(A.EOS_PR)
    rc = e.critical_point()[1]
    gaps = []
    for d in ["1e-3", "1e-5"]:
        rg, rl = e.maxwell(1 - mp.mpf(d))
        assert rg < rc < rl
        gaps.append((rl - rg) / rc)
    ratio = gaps[0] / gaps[1]          # sqrt(1e-3 / 1e-5) = 10
    assert abs(ratio - 10) < 0.1
    assert gaps[1] < 0.05


@pytest.mark.parametrize("eos", ALL)
def test_corresponding_states(eos):
    """In reduced variables (b rho, T/T_c) each EOS of the paper depends on
    nothing else, so b*rho_g and b*rho_l at fixed T_r do not change when a and
    b are changed."""
    e1 = A.EOS(eos)
    e2 = A.EOS(eos, a=e1.a * 3, b=e1.b / 2)
    g1, l1 = e1.maxwell(0.65)
    g2, l2 = e2.maxwell(0.65)
    assert abs(e1.b * g1 / (e2.b * g2) - 1) < mp.mpf(10) ** -20
    assert abs(e1.b * l1 / (e2.b * l2) - 1) < mp.mpf(10) ** -20


def test_density_ratio_printed_at_T04(golden_dir):
    """Sec. 5.4: PR and RKS density ratios exceed 65,000 at T_r = 0.4."""
    g = json.load(open(os.path.join(golden_dir, "paper_printed.json")))["density_ratio_T04"]
    for eos in (A.EOS_PR, A.EOS_RKS):
        rg, rl = A.EOS(eos).maxwell(g["T_r"])
        assert rl / rg > g["min_ratio"]


def test_pr_domain_limit(golden_dir):
    """Sec. 5.6: the PR chemical potential diverges at rho = 1/b = 21/2."""
    g = json.load(open(os.path.join(golden_dir, "paper_printed.json")))["pr_domain_limit"]
    e = A.EOS(A.EOS_PR)
    assert 1 / e.b == mp.mpf(g["inv_b"][0]) / g["inv_b"][1]
    T, al = e.temperature(0.6)
    assert e.mu0(1 / e.b * (1 - mp.mpf("1e-12")), T, al) > 1
    p = A.params(A.EOS_PR, 0.6, 8, 8, kappa=0.1, tau=1.0, k=0.5, mu_cap=6.0)
    assert oracle.mu0_capped(p, 10.5) == 6.0          # at 1/b: the limit
    assert oracle.mu0_capped(p, 11.0) == 6.0          # beyond it: the limit
    assert oracle.mu0_capped(p, 10.49999999) == 6.0   # finite but above the limit
    assert oracle.mu0_capped(p, 5.0) == pytest.approx(float(e.mu0(mp.mpf(5), T, al)), rel=1e-14)


def test_interface_profile_first_integral():
    """Eq. 22 is the first integral of mu = psi'(rho) - kappa rho'' = mu_b.
    Integrate that second-order ODE from the profile's origin with the
    slope of Eq. 24 (mpmath Taylor ODE solver) and check that the
    trajectory follows the quadrature y(rho) of Eq. 23 and tends to the
    liquid density."""
    e = A.EOS(A.EOS_CS)
    it = e.interface(0.8)
    T, al, mub = it["T"], it["alpha"], it["mu_b"]
    r0 = (it["rho_g"] + it["rho_l"]) / 2
    with mp.workdps(20):
        _check_trajectory(e, it, T, al, mub, r0)


def _check_trajectory(e, it, T, al, mub, r0):
    sol = mp.odefun(lambda y, s: [s[1], e.mu0(s[0], T, al) - mub], 0,
                    [r0, it["drho_dy"](r0)])
    for y in [1, 3]:
        rho_y, d_y = sol(y)
        assert abs(it["y_of_rho"](rho_y) - y) < mp.mpf(10) ** -12
        assert abs(d_y - it["drho_dy"](rho_y)) < mp.mpf(10) ** -12
    rho_far = sol(12)[0]
    assert abs(rho_far - it["rho_l"]) < 1e-3 * it["rho_l"]


def test_surface_tension_two_routes():
    """sigma = kappa int rho'^2 dy (pressure-tensor mismatch, Sec. 5.3)
    computed along the ODE trajectory equals int sqrt(2 kappa dOmega) drho."""
    e = A.EOS(A.EOS_CS)
    it = e.interface(0.8)
    T, al, mub = it["T"], it["alpha"], it["mu_b"]
    r0 = (it["rho_g"] + it["rho_l"]) / 2
    with mp.workdps(20):
        sol = mp.odefun(lambda y, s: [s[1], e.mu0(s[0], T, al) - mub], 0,
                        [r0, it["drho_dy"](r0)])
        liquid_half = mp.quad(lambda y: sol(y)[1] ** 2, [0, 4, 10, 16])
    # by symmetry of the first integral the gas side mirrors the slope; use
    # the quadrature form on the gas half and the trajectory on the liquid half
    gas_half = mp.quad(lambda r: it["drho_dy"](r), [it["rho_g"], r0])
    total = liquid_half + gas_half
    assert abs(total / it["sigma1"] - 1) < 2e-3   # truncation of the tail at y = 16
