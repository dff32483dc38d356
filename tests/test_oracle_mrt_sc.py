"""Pins of the oracle's multiple-relaxation-time collision (Eq. 4) and of the
pseudopotential comparison model with k and the compact scheme (Sec. 5.1).

What fixes them, independently of how the oracle computes them:
* MRT: the moment basis is orthogonal and inverts; with every rate equal to
  1/tau it is the BGK collision of Eq. 1; it conserves mass and adds the
  momentum F; a shear wave decays at the viscosity c_s^2 (1/s_v - 1/2) that
  s_v = 1/tau gives (the closed form of the linearised Navier-Stokes mode);
  a flat interface converges to the same densities as SRT (the paper's
  MRT tau = 0.8 against SRT tau = 3.0 comparison).
* Pseudopotential: on smooth fields its force tends, at the compact scheme's
  sixth order, to c_s^2 grad rho - grad(k^2 p0), the limit the chemical-
  potential force of Eq. 12 also has at kappa = 0 (Gibbs-Duhem, Eq. 9).
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from oracle import analytic as A
from paper_1906_09530_amd import inputs

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
RATES = A.MRT_RATES


def test_mrt_basis_orthogonal_and_inverse():
    M = oracle.mrt_matrix()
    G = M @ M.T
    np.testing.assert_array_equal(G, np.diag(np.diag(G)))       # orthogonal rows
    np.testing.assert_array_equal(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])
    np.testing.assert_allclose(oracle.mrt_inverse(), np.linalg.inv(M), atol=1e-15)
    # the conserved rows are density and momentum (Eq. 3)
    np.testing.assert_array_equal(M[0], np.ones(9))
    np.testing.assert_array_equal(M[3], EX)
    np.testing.assert_array_equal(M[5], EY)
    # relaxation matrix slots: e and eps are even, q odd, p_xx and p_xy the
    # traceless stresses
    np.testing.assert_array_equal(M[7], EX ** 2 - EY ** 2)
    np.testing.assert_array_equal(M[8], EX * EY)


def test_mrt_equal_rates_is_bgk():
    """S = (1/tau) I on the non-conserved moments gives the BGK operator."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        fi = rng.uniform(0.01, 0.3, 9)
        rho = fi.sum()
        ux, uy = (EX * fi).sum() / rho, (EY * fi).sum() / rho
        Fx, Fy = rng.normal(0, 0.01, 2)
        tau = rng.uniform(0.55, 3.0)
        a = oracle.collide_node_mrt(fi, rho, ux, uy, Fx, Fy, tau, 1 / tau, 1 / tau, 1 / tau)
        b = oracle.collide_node(fi, rho, ux, uy, Fx, Fy, tau)
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


def test_mrt_conserves_mass_and_adds_the_force():
    rng = np.random.default_rng(4)
    for _ in range(20):
        fi = rng.uniform(0.01, 0.3, 9)
        rho = fi.sum()
        jx, jy = (EX * fi).sum(), (EY * fi).sum()
        Fx, Fy = rng.normal(0, 0.01, 2)
        fo = oracle.collide_node_mrt(fi, rho, jx / rho, jy / rho, Fx, Fy, 0.8, *RATES)
        assert fo.sum() == pytest.approx(rho, rel=1e-14)
        assert (EX * fo).sum() == pytest.approx(jx + Fx, abs=1e-15)
        assert (EY * fo).sum() == pytest.approx(jy + Fy, abs=1e-15)
        # the relaxed moments move toward equilibrium by their own rates
        M = oracle.mrt_matrix()
        eq = np.array([oracle.feq(i, rho, jx / rho, jy / rho) for i in range(9)])
        m, meq = M @ fi, M @ eq
        f0 = oracle.collide_node_mrt(fi, rho, jx / rho, jy / rho, 0.0, 0.0, 0.8, *RATES)
        s = np.array([0, RATES[0], RATES[1], 0, RATES[2], 0, RATES[2], 1 / 0.8, 1 / 0.8])
        np.testing.assert_allclose(M @ f0, m - s * (m - meq), atol=1e-14)


@pytest.mark.parametrize("collision", [0, 1])
def test_shear_wave_decays_at_the_viscosity(collision):
    """u_x = U sin(2 pi y / L) in a uniform fluid decays as exp(-nu q^2 t),
    nu = c_s^2 (tau - 1/2) (Sec. 2): BGK and MRT (s_v = 1/tau) alike."""
    L, tau, U = 128, 0.8, 1e-4
    nu = (tau - 0.5) / 3.0
    p = A.params(A.EOS_CS, 0.7, 4, L, kappa=0.1, tau=tau, k=0.2, collision=collision)
    _, l = A.coexistence(A.EOS_CS, 0.7)
    y = np.arange(L)
    rho = np.full((L, 4), l)
    ux = np.repeat((U * np.sin(2 * np.pi * y / L))[:, None], 4, axis=1)
    f = oracle.init(p, rho, ux, np.zeros_like(ux))
    amp = {}
    done = 0
    for t in (100, 600):
        oracle.run(p, f, t - done)
        done = t
        _, vx, _ = oracle.moments(p, f)
        amp[t] = 2 * np.mean(vx[:, 0] * np.sin(2 * np.pi * y / L))
    q = 2 * np.pi / L
    nu_meas = -math.log(amp[600] / amp[100]) / (q * q * 500)
    assert nu_meas == pytest.approx(nu, rel=2e-3)


def _slab(T_r, tau, collision, ny=128):
    g, l = A.coexistence(A.EOS_CS, T_r)
    p = A.params(A.EOS_CS, T_r, 4, ny, kappa=0.1, tau=tau, k=0.2, collision=collision)
    rho, ux, uy = inputs.slab(4, ny, g, l, 4.0)
    f = oracle.init(p, rho, ux, uy)
    st, steps, d = oracle.run_until_converged(p, f, 1e-12, 100, 300000)
    assert st == 0
    return oracle.moments(p, f)[0][:, 0]


def test_mrt_and_srt_reach_the_same_coexistence():
    """Sec. 5.1: MRT at tau = 0.8 and SRT at tau = 3.0 give the same flat
    interface.  In an x-uniform steady state the rest populations sit at
    equilibrium and the moving ones carry the momentum flux rho c_s^2 +
    F^2/(4 rho) whatever the relaxation rates, so the converged profiles
    agree to the convergence tolerance."""
    r_mrt = _slab(0.7, 0.8, 1)
    r_srt = _slab(0.7, 3.0, 0)
    np.testing.assert_allclose(r_mrt, r_srt, rtol=1e-8)


# ---- pseudopotential comparison model ------------------------------------

def _mp_p0(eos, T_r):
    e = A.EOS(eos)
    T, al = e.temperature(T_r)
    return lambda r: e.p0(r, T, al)


def _force_error(force, n, eos=A.EOS_CS, T_r=0.7, k=0.3):
    """Max |F_oracle - F_limit| / max |F_limit| for rho = rho0 (1 + 0.2 sin(2 pi x / n)),
    F_limit = c_s^2 rho' - k^2 p0'(rho) rho' evaluated exactly."""
    g, l = A.coexistence(eos, T_r)
    rho0 = 0.5 * (g + l)
    p = A.params(eos, T_r, n, 4, kappa=0.0, tau=1.0, k=k, force=force)
    x = np.arange(n)
    th = 2 * np.pi * x / n
    rho = np.repeat((rho0 * (1 + 0.2 * np.sin(th)))[None, :], 4, axis=0)
    drho = rho0 * 0.2 * np.cos(th) * 2 * np.pi / n
    P = _mp_p0(eos, T_r)
    dp = np.array([float(mp.diff(P, mp.mpf(float(r)))) for r in rho[0]])
    F_lim = drho / 3.0 - k * k * dp * drho
    f = oracle.init(p, rho, np.zeros_like(rho), np.zeros_like(rho))
    _, _, _, _, fx, fy = oracle.moments(p, f, want_force=True)
    assert np.abs(fy).max() == 0.0
    return np.abs(fx[0] - F_lim).max() / np.abs(F_lim).max()


@pytest.mark.parametrize("force", [0, 1])
def test_both_forces_tend_to_the_pressure_gradient(force):
    """Pseudopotential (force 1) and chemical-potential force at kappa = 0
    (force 0) both converge to c_s^2 grad rho - grad(k^2 p0) at sixth order."""
    e32, e64 = _force_error(force, 32), _force_error(force, 64)
    order = math.log2(e32 / e64)
    assert e64 < 1e-5
    assert order > 5.5, (e32, e64, order)


def test_pseudopotential_mass_and_psi():
    """psi^2 c_s^2 G / 2 + rho c_s^2 is the mesh pressure k^2 p0 (G = -1), and
    a drop run with the pseudopotential force conserves mass."""
    p = A.params(A.EOS_CS, 0.8, 32, 32, kappa=0.0, tau=1.0, k=0.3, force=1)
    P = _mp_p0(A.EOS_CS, 0.8)
    for r in (0.01, 0.1, 0.2, 0.3):
        psi = float(oracle.sc_psi(p, r))
        assert r / 3 - psi * psi / 6 == pytest.approx(0.09 * float(P(r)), rel=1e-12, abs=1e-16)
    g, l = A.coexistence(A.EOS_CS, 0.8)
    rho, ux, uy = inputs.droplet(32, 32, g, l, 9.0, 4.0)
    f = oracle.init(p, rho, ux, uy)
    m0 = f.sum()
    oracle.run(p, f, 200)
    assert np.isfinite(f).all()
    assert abs(f.sum() / m0 - 1) < 1e-13
