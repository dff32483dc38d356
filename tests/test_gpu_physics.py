"""Physics of the converged solver against the thermodynamics the paper fixes
(Sec. 5.1 coexistence, Sec. 5.3 Laplace's law), run as batches on the GPU.

The pins come from the oracle's arbitrary-precision thermodynamics (Maxwell
construction, planar-interface surface tension), not from the solver.  The
bounds follow what the BGK scheme with the exact-difference force reaches at
these settings (measured; the deviations are properties of the scheme, shared
by the oracle):

* flat slabs, CS, T/Tc = 0.5 ... 0.85, k = 0.2 ... 0.4, interfaces of 5 and 8
  nodes: liquid within 2e-5 of Maxwell everywhere (measured <= 8.3e-6), gas
  within 1e-3 at T/Tc = 0.85 (measured 1.1e-4) and above Maxwell by an amount
  that grows as T falls (3.7e-2 at 0.5);
* drops, T/Tc = 0.85 and 0.75, k = 0.2, 8-node interface, R = 32 ... 96
  (radius at least four interface widths): the pressure jump
  k^2 [p0(rho_in) - p0(rho_out)] times the equimolar radius is the same for
  every drop to 3 % (Laplace's law, measured 1.2 %).  Its slope is the
  surface tension by the integral method (Sec. 5.3) through the drop centre
  once the pressure tensor is the lattice's own: Eq. 10 gives
  P_N - P_T = kappa (d rho/dy)^2, and the forced lattice adds the momentum
  flux F F/(4 rho) of its bare velocity u = -F/(2 rho), normal to the
  interface (an exact identity of the steady state, pinned on the oracle).
  With both terms the slope matches the integral to 3 %; Eq. 10's term alone
  is about half of it.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import analytic as A
from paper_1906_09530_amd import inputs, lbm

pytestmark = pytest.mark.gpu

T_R, K, W = 0.85, 0.2, 8.0


def _settings(T_r=T_R):
    e = A.EOS(A.EOS_CS)
    it = e.interface(T_r)
    w1 = float(mp.re(it["width1"]))
    kappa = (W * K / w1) ** 2
    return e, it, kappa


def _converge(b, n, max_chunks=20):
    for _ in range(max_chunks):
        st, _, _, sts = b.run_until_converged(1e-12, 100, 50_000)
        if all(s != lbm.LBM_NOT_CONVERGED for s in sts):
            break
    assert all(s == lbm.LBM_OK for s in sts), sts


# (T/Tc, k, interface width W) of the flat-slab table; k = 0.3 with W = 8 and
# k = 0.4 with W >= 5 diverge at T/Tc <= 0.6 (stability of the explicit scheme)
SLABS = [(0.50, 0.2, 5.0), (0.50, 0.2, 8.0), (0.60, 0.2, 8.0), (0.70, 0.2, 8.0),
         (0.70, 0.3, 8.0), (0.85, 0.2, 8.0), (0.85, 0.4, 8.0)]


def test_flat_slabs_against_the_maxwell_densities():
    """Flat slabs, 64 x 384 (liquid in the middle half), CS, tau = 1,
    kappa = (W k / w1)^2, run as one batch to convergence.  Liquid within
    2e-5 of Maxwell everywhere (measured <= 8.3e-6); the gas within 1e-3 at
    T/Tc = 0.85 (measured 1.1e-4, 1.4e-4) and above Maxwell by an amount that
    grows as T falls (3.7e-2 at 0.5).  The offset is the jump of the mesh
    chemical potential between the two bulks that the discrete steady state
    leaves (pinned on the oracle); it shrinks as the interface widens in
    nodes.  Every slab stays flat."""
    e = A.EOS(A.EOS_CS)
    nx, ny = 64, 384
    ps, r0, ml = [], [], []
    for T_r, k, W in SLABS:
        w1 = float(mp.re(e.interface(T_r)["width1"]))
        g, l = A.coexistence(A.EOS_CS, T_r)
        ps.append(lbm.params(lbm.EOS_CS, T_r, nx, ny, kappa=(W * k / w1) ** 2, tau=1.0, k=k))
        r0.append(inputs.slab(nx, ny, g, l, W)[0])
        ml.append((g, l))
    b = lbm.Batch(ps, r0)
    _converge(b, len(ps))
    dev = {}
    print("\n T/Tc    k    W   kappa   rho_l-Maxwell  rho_g-Maxwell")
    for i, (T_r, k, W) in enumerate(SLABS):
        r = b.moments(i)[0]
        g, l = ml[i]
        dl, dg = r[ny // 2, 0] / l - 1, r[0, 0] / g - 1
        dev[(T_r, k, W)] = (dl, dg)
        print(" %.2f  %.1f  %.0f  %.4f   %+.2e      %+.2e" % (T_r, k, W, ps[i].kappa, dl, dg),
              flush=True)
        assert (r == r[:, :1]).all()      # stays flat
        assert abs(dl) <= 2e-5
        assert 0.0 < dg <= 0.1
    assert dev[(0.85, 0.2, 8.0)][1] <= 1e-3 and dev[(0.85, 0.4, 8.0)][1] <= 1e-3
    gas = [dev[(T, 0.2, 8.0)][1] for T in (0.5, 0.6, 0.7, 0.85)]
    assert all(a > b for a, b in zip(gas, gas[1:]))


def test_gas_density_reaches_maxwell_as_the_interface_is_resolved():
    """Sec. 5.1 with the mesh coefficient of Sec. 4 (a smaller k spreads the
    same transition region over more nodes): CS slabs at T/Tc = 0.7 and 0.6
    with kappa fixed and k = 0.2, 0.1, 0.05 (interfaces of 8, 16 and 32
    nodes), converged as one batch.  The gas offset from Maxwell -- the jump
    of the mesh chemical potential that the discrete balance leaves -- falls
    as about the inverse square of the interface width: measured 1.9e-3,
    5.2e-4, 1.8e-4 at 0.7 and 8.5e-3, 2.2e-3, 6.1e-4 at 0.6, so the gas meets
    Maxwell within 1e-3 at 16 nodes (0.7) and 32 nodes (0.6); the liquid is
    within 1e-5 in every case."""
    e = A.EOS(A.EOS_CS)
    cases = [(T, Wn) for T in (0.7, 0.6) for Wn in (8.0, 16.0, 32.0)]
    ps, r0, ml = [], [], []
    for T_r, Wn in cases:
        k = 0.2 * 8.0 / Wn
        w1 = float(mp.re(e.interface(T_r)["width1"]))
        g, l = A.coexistence(A.EOS_CS, T_r)
        ny = int(max(384, 24 * Wn)) // 8 * 8
        ps.append(lbm.params(lbm.EOS_CS, T_r, 64, ny, kappa=(Wn * k / w1) ** 2, tau=1.0, k=k))
        r0.append(inputs.slab(64, ny, g, l, Wn)[0])
        ml.append((g, l, ny))
    b = lbm.Batch(ps, r0)
    _converge(b, len(ps), max_chunks=40)
    off = {}
    print("\n T/Tc   W   gas - Maxwell   liquid - Maxwell")
    for i, (T_r, Wn) in enumerate(cases):
        r = b.moments(i)[0]
        g, l, ny = ml[i]
        dg, dl = r[0, 0] / g - 1, r[ny // 2, 0] / l - 1
        off[(T_r, Wn)] = dg
        print(" %.2f  %3.0f   %+.3e      %+.3e" % (T_r, Wn, dg, dl), flush=True)
        assert abs(dl) <= 1e-5
        assert dg > 0
    for T_r in (0.7, 0.6):
        a, bb, c = (off[(T_r, Wn)] for Wn in (8.0, 16.0, 32.0))
        assert a / bb > 2.5 and bb / c > 2.5          # about 1 / W^2
    assert off[(0.7, 16.0)] < 1e-3 and off[(0.7, 32.0)] < 1e-3 and off[(0.6, 32.0)] < 1e-3


def _integral_sigma(p, op, f, r):
    """Surface tension of a converged drop by the integral method along the
    vertical line through its centre (Sec. 5.3): Eq. 10's kappa (d rho/dy)^2
    and the forced lattice's normal momentum flux F_y^2/(4 rho), each summed
    over the line and halved (the line crosses the interface twice).  The
    derivative and the force come from the oracle on the GPU's state."""
    import oracle
    c = p.nx // 2
    dy = oracle.cfm_columns(op, r)[:, c]
    _, _, _, _, _, fy = oracle.moments(op, np.ascontiguousarray(f), want_force=True)
    s10 = p.kappa * float(np.sum(dy ** 2)) / 2
    sff = float(np.sum(fy[:, c] ** 2 / (4 * r[:, c]))) / 2
    return s10, sff


@pytest.mark.parametrize("T_r", [0.85, 0.75])
def test_drops_follow_laplaces_law(T_r):
    e, it, kappa = _settings(T_r)
    T, al = it["T"], it["alpha"]
    sigma = K * kappa ** 0.5 * float(mp.re(it["sigma1"]))
    g, l = A.coexistence(A.EOS_CS, T_r)
    radii = (32, 48, 64, 96)
    ps, r0 = [], []
    for R in radii:
        n = int(8 * ((2 * R + 12 * W) // 8 + 1))
        ps.append(lbm.params(lbm.EOS_CS, T_r, n, n, kappa=kappa, tau=1.0, k=K))
        r0.append(inputs.droplet(n, n, g, l, R, W)[0])
    b = lbm.Batch(ps, r0)
    _converge(b, len(radii))
    inv_r, dp, s10, sff = [], [], [], []
    print("\nT/Tc %.2f:  R0  equimolar R  rho_in   rho_out     k^2 dp0     k^2 dp0 R   "
          "sigma_Eq10  sigma_FF" % T_r)
    for i, p in enumerate(ps):
        r = b.moments(i)[0]
        n = p.nx
        rin, rout = r[n // 2, n // 2], r[0, 0]
        req = float(np.sqrt((r - rout).sum() / (np.pi * (rin - rout))))  # equimolar radius
        inv_r.append(1.0 / req)
        dp.append(K * K * float(mp.re(e.p0(mp.mpf(rin), T, al) - e.p0(mp.mpf(rout), T, al))))
        op = A.params(A.EOS_CS, T_r, n, n, kappa=kappa, tau=1.0, k=K)
        a, bb = _integral_sigma(p, op, b.get_state(i), r)
        s10.append(a)
        sff.append(bb)
        print("           %3d  %7.2f    %.5f  %.4e  %.4e  %.2e  %.4e  %.4e" % (
            radii[i], req, rin, rout, dp[-1], dp[-1] * req, a, bb))
    jump_r = np.array(dp) / np.array(inv_r)  # sigma implied by each drop
    slope = float(np.polyfit(inv_r, dp, 1)[0])
    s_int = float(np.mean(np.array(s10) + np.array(sff)))
    print("Laplace: dP R = %s (continuum sigma %.4e, ratio %.2f)" % (
        " ".join("%.4e" % v for v in jump_r), sigma, jump_r.mean() / sigma))
    print("slope %.4e; integral sigma: Eq. 10 %.4e + lattice F^2/(4 rho) %.4e = %.4e "
          "(slope / integral %.3f, slope / Eq. 10 term %.2f)" % (
              slope, np.mean(s10), np.mean(sff), s_int, slope / s_int, slope / np.mean(s10)),
          flush=True)
    assert np.all(np.diff(dp) < 0)                 # smaller drops, larger jump
    assert (jump_r.max() - jump_r.min()) <= 0.03 * jump_r.mean()
    assert abs(slope / s_int - 1) <= 0.03
    assert 1.3 < jump_r.mean() / sigma < 2.0


@pytest.mark.parametrize("eos,k", [(lbm.EOS_PR, 0.2), (lbm.EOS_RKS, 0.2), (lbm.EOS_VDW, 0.1)])
def test_laplaces_law_for_the_other_equations_of_state(eos, k):
    """Sec. 5.3 (Fig. 8): Laplace's law for the other EOS the paper tests, at
    T/Tc = 0.8, 8-node interfaces (k = 0.2; VdW at k = 0.1, where its drops
    stay finite), drops of R = 32 ... 96 converged as one batch: the
    pressure jump k^2 [p0(rho_in) - p0(rho_out)] times the equimolar radius
    is the same for every drop to 3 %, smaller drops carry larger jumps, and
    the slope of the jump against 1/R equals the surface tension of the
    integral method (Eq. 10's term plus the lattice's F^2/(4 rho), as for the
    CS drops) to 3 %: measured slope / integral 0.999 (PR), 1.000 (RKS),
    1.013 (VdW)."""
    T_r = 0.8
    e = A.EOS(eos)
    it = e.interface(T_r)
    T, al = it["T"], it["alpha"]
    kappa = (W * k / float(mp.re(it["width1"]))) ** 2
    g, l = A.coexistence(eos, T_r)
    radii = (32, 48, 64, 96)
    ps, r0 = [], []
    for R in radii:
        n = int(8 * ((2 * R + 12 * W) // 8 + 1))
        ps.append(lbm.params(eos, T_r, n, n, kappa=kappa, tau=1.0, k=k))
        r0.append(inputs.droplet(n, n, g, l, R, W)[0])
    b = lbm.Batch(ps, r0)
    _converge(b, len(radii))
    inv_r, dp, sig = [], [], []
    for i, p in enumerate(ps):
        r = b.moments(i)[0]
        n = p.nx
        rin, rout = r[n // 2, n // 2], r[0, 0]
        req = float(np.sqrt((r - rout).sum() / (np.pi * (rin - rout))))
        inv_r.append(1.0 / req)
        dp.append(k * k * float(mp.re(e.p0(mp.mpf(rin), T, al) - e.p0(mp.mpf(rout), T, al))))
        op = A.params(eos, T_r, n, n, kappa=kappa, tau=1.0, k=k)
        a, bb = _integral_sigma(p, op, b.get_state(i), r)
        sig.append(a + bb)
    jump_r = np.array(dp) / np.array(inv_r)
    slope = float(np.polyfit(inv_r, dp, 1)[0])
    s_int = float(np.mean(sig))
    sigma = k * kappa ** 0.5 * float(mp.re(it["sigma1"]))
    print("\nEOS %d: dP R = %s; slope %.4e, integral sigma %.4e (ratio %.3f), continuum %.4e" % (
        eos, " ".join("%.4e" % v for v in jump_r), slope, s_int, slope / s_int, sigma),
        flush=True)
    assert np.all(np.diff(dp) < 0)
    assert (jump_r.max() - jump_r.min()) <= 0.03 * jump_r.mean()
    assert abs(slope / s_int - 1) <= 0.03


# (EOS, T/Tc) of the superlarge-ratio slabs (Sec. 5.1, Fig. 4: k = 0.1)
RATIO_SLABS = [(lbm.EOS_PR, 0.25), (lbm.EOS_RKS, 0.25), (lbm.EOS_CS, 0.20), (lbm.EOS_CS, 0.17)]


def test_superlarge_density_ratio_slabs():
    """Flat slabs, 64 x 400, k = 0.1 (the paper's default), tau = 1, 8-node
    interface, run to max |drho| < 1e-12 per 100 steps: Maxwell ratios of
    5.6e11 (PR, T/Tc = 0.25), 1.0e12 (RKS, 0.25), 5.2e10 (CS, 0.20) and
    2.1e13 (CS, 0.17).  Every slab converges and stays flat; the liquid meets
    Maxwell to 1e-7 (measured <= 1.1e-8); the gas settles above Maxwell (the
    low-temperature offset of the scheme, 4.4-19x here), leaving converged
    density ratios above 1e10 (measured 7.9e10, 1.3e11, 1.2e10, 1.1e12).
    The absolute criterion says little about a gas of 1e-11, so each slab
    then runs 20,000 steps more and its gas density must change by less
    than 1e-8 of itself per 100 steps."""
    nx, ny, W, k = 64, 400, 8.0, 0.1
    ps, r0, ml = [], [], []
    for eos, T_r in RATIO_SLABS:
        e = A.EOS(eos)
        w1 = float(mp.re(e.interface(T_r)["width1"]))
        g, l = A.coexistence(eos, T_r)
        ps.append(lbm.params(eos, T_r, nx, ny, kappa=(W * k / w1) ** 2, tau=1.0, k=k))
        r0.append(inputs.slab(nx, ny, g, l, W)[0])
        ml.append((g, l))
    b = lbm.Batch(ps, r0)
    _converge(b, len(ps))
    drift = []
    for i, p in enumerate(ps):           # converged members have retired
        s = lbm.Solver(p, r0[i])
        s.set_state(b.get_state(i))
        gas0 = s.moments()[0][0, 0]
        s.step(20_000)
        drift.append(abs(s.moments()[0][0, 0] / gas0 - 1) / 200)
        s.close()
    print("\n gas drift per 100 steps after convergence: %s" % (
        " ".join("%.1e" % d for d in drift)))
    assert max(drift) < 1e-8
    print(" EOS  T/Tc  Maxwell ratio  rho_l-Maxwell  rho_g/Maxwell  ratio")
    for i, (eos, T_r) in enumerate(RATIO_SLABS):
        r = b.moments(i)[0]
        g, l = ml[i]
        rl, rg = r[ny // 2, 0], r[0, 0]
        print(" %d    %.2f  %.3e      %+.2e      %.2f          %.3e" % (
            eos, T_r, l / g, rl / l - 1, rg / g, rl / rg), flush=True)
        assert (r == r[:, :1]).all()
        assert abs(rl / l - 1) <= 1e-7
        assert 1.0 < rg / g < 25.0
        assert rl / rg > 1e10


def test_spurious_current_of_converged_drops():
    """Sec. 5.4, Fig. 9: static PR and RKS drops at T/Tc = 0.6, 0.5, 0.4 run
    to max |drho| < 1e-12 per 100 steps (192 x 192, R = 60, tanh width 10,
    tau = 1.5 as in the paper, k = 0.05, kappa for a 10-node interface,
    limit 6).  The largest speed |v| of the converged field (the spurious
    current) stays far below 1e-3 (measured 2.0e-4 PR, 3.0e-4 RKS at
    T/Tc = 0.4) and grows as the temperature falls, as in Fig. 9(a).  The
    converged density ratio at T/Tc = 0.4 exceeds 1e4 (measured 1.8e4 PR,
    2.8e4 RKS; the Maxwell ratios are 6.8e5 and 7.5e5): the drop's Laplace
    pressure and the scheme's gas offset, which grows at small k, keep it
    below the paper's 65,000.  With k = 0.07 the ratios reach 5.5e4 and 6.3e4
    but the spurious current 0.8e-3 and 1.3e-3; at k = 0.1 the RKS drops
    diverge for interfaces wider than 6 nodes (measured on the same meshes)."""
    cases = [(eos, T_r) for eos in (lbm.EOS_PR, lbm.EOS_RKS) for T_r in (0.6, 0.5, 0.4)]
    n, R, k, W = 192, 60.0, 0.05, 10.0
    ps, r0 = [], []
    for eos, T_r in cases:
        g, l = A.coexistence(eos, T_r)
        w1 = float(mp.re(A.EOS(eos).interface(T_r)["width1"]))
        ps.append(lbm.params(eos, T_r, n, n, kappa=(W * k / w1) ** 2, tau=1.5, k=k,
                             mu_cap=6.0))
        r0.append(inputs.droplet(n, n, g, l, R, 10.0)[0])
    b = lbm.Batch(ps, r0)
    _converge(b, len(ps), max_chunks=60)
    print("\n EOS  T/Tc  steps     max|v|      rho_in/rho_out   Maxwell ratio")
    vmax = {}
    for i, (eos, T_r) in enumerate(cases):
        r, vx, vy = b.moments(i)
        g, l = A.coexistence(eos, T_r)
        v = float(np.hypot(vx, vy).max())
        ratio = r[n // 2, n // 2] / r[0, 0]
        vmax[(eos, T_r)] = v
        print(" %d    %.1f   %7d   %.3e   %.3e        %.3e" % (
            eos, T_r, b.steps_taken(i), v, ratio, l / g), flush=True)
        assert v < 1e-3
        if T_r == 0.4:
            assert ratio > 1e4
    for eos in (lbm.EOS_PR, lbm.EOS_RKS):
        assert vmax[(eos, 0.4)] > vmax[(eos, 0.5)] > vmax[(eos, 0.6)]


def _line_width_and_sigma(p, op, f, r):
    """Interface width (rho_l - rho_g) / max |d rho/dy| and surface tension of a
    converged flat slab along one column: Eq. 10's kappa (d rho/dy)^2 and the
    lattice's F_y^2/(4 rho), summed over the column and halved (two
    interfaces).  The derivative and force come from the oracle on the GPU's
    state."""
    import oracle
    col = r[:, 0]
    dy = oracle.cfm_columns(op, r)[:, 0]
    _, _, _, _, _, fy = oracle.moments(op, np.ascontiguousarray(f), want_force=True)
    width = (col.max() - col.min()) / np.abs(dy).max()
    s10 = p.kappa * float(np.sum(dy ** 2)) / 2
    sff = float(np.sum(fy[:, 0] ** 2 / (4 * col))) / 2
    return width, s10, sff


# Figs. 6-7: six EOS at T/Tc = 0.6 (PRM: Peng-Robinson for methane); kappa
# fixed per EOS (a 4-node interface at k = 0.3; 3 nodes for van der Waals,
# whose liquid is denser and less stable), k = 0.05 ... 0.2
F67_EOS = [("VdW", lbm.EOS_VDW, 0.344, 3.0), ("RK", lbm.EOS_RK, 0.344, 4.0),
           ("RKS", lbm.EOS_RKS, 0.344, 4.0), ("PR", lbm.EOS_PR, 0.344, 4.0),
           ("PRM", lbm.EOS_PR, 0.011, 4.0), ("CS", lbm.EOS_CS, 0.344, 4.0)]
F67_K = (0.05, 0.1, 0.15, 0.2)


def test_interface_width_and_surface_tension_vs_k():
    """Sec. 5.2, Figs. 6-7: flat slabs of six EOS at T/Tc = 0.6 in mesh spaces
    k = 0.05 ... 0.2 at a fixed kappa per EOS.  The interface width in nodes
    goes as 1/k: width * k (the momentum-space width) is the same for every
    k to 8 %; the surface tension of the lattice divided by k (its
    momentum-space value) likewise.  Both exceed the continuum w1 sqrt(kappa)
    and sqrt(kappa) sigma1: the forced lattice's normal flux F^2/(4 rho) acts
    as an extra gradient coefficient of order c_s^4/(2 rho) (see the design
    notes); the measured values are printed."""
    T_r = 0.6
    cases, ps, r0, ops = [], [], [], []
    for name, eos, om, nodes in F67_EOS:
        e = A.EOS(eos, omega=om)
        it = e.interface(T_r)
        w1, s1 = float(mp.re(it["width1"])), float(mp.re(it["sigma1"]))
        g, l = (float(v) for v in e.maxwell(T_r))
        kap = (nodes * 0.3 / w1) ** 2
        for k in F67_K:
            w = w1 * kap ** 0.5 / k
            ny = 384 if k < 0.1 else 256
            cases.append((name, k, kap, w1, s1))
            ps.append(lbm.params(eos, T_r, 64, ny, kappa=kap, tau=1.0, k=k, omega=om))
            ops.append(A.params(eos, T_r, 64, ny, kappa=kap, tau=1.0, k=k, omega=om))
            r0.append(inputs.slab(64, ny, g, l, min(w, 16.0))[0])
    b = lbm.Batch(ps, r0)
    _converge(b, len(ps), max_chunks=40)
    print("\n EOS   k     width   width*k  w1 sqrt(kappa)  sigma_Eq10/k  sigma_lattice/k  "
          "sqrt(kappa) sigma1")
    res = {}
    for i, (name, k, kap, w1, s1) in enumerate(cases):
        r = b.moments(i)[0]
        width, s10, sff = _line_width_and_sigma(ps[i], ops[i], b.get_state(i), r)
        res.setdefault(name, []).append((width * k, (s10 + sff) / k, s10 / k))
        print(" %-4s %.2f  %6.2f   %.3f    %.3f           %.3e     %.3e        %.3e" % (
            name, k, width, width * k, w1 * kap ** 0.5, s10 / k, (s10 + sff) / k,
            kap ** 0.5 * s1), flush=True)
    for name, vals in res.items():
        wk = [v[0] for v in vals]
        sk = [v[1] for v in vals]
        assert max(wk) / min(wk) - 1 <= 0.08, (name, wk)
        assert max(sk) / min(sk) - 1 <= 0.08, (name, sk)


def test_pseudopotential_against_chemical_potential_slabs():
    """Sec. 5.1, Fig. 4: CS flat slabs, 64 x 256, k = 0.2, tau = 1, with the
    pseudopotential force (no kappa) and with the chemical-potential force
    (8-node interface), T/Tc = 0.5 ... 0.8.  Both keep the liquid within 1e-4
    of Maxwell; the gas of both settles above it, the pseudopotential's
    further (measured 2-5x), so the chemical-potential model stays closer to
    the Maxwell curve at every temperature, as the paper reports."""
    temps = (0.5, 0.6, 0.7, 0.8)
    k, W = 0.2, 8.0
    ps, r0, ml = [], [], []
    e = A.EOS(A.EOS_CS)
    for force in (lbm.FORCE_SC, lbm.FORCE_CP):
        for T_r in temps:
            g, l = A.coexistence(A.EOS_CS, T_r)
            w1 = float(mp.re(e.interface(T_r)["width1"]))
            kap = 0.0 if force == lbm.FORCE_SC else (W * k / w1) ** 2
            ps.append(lbm.params(lbm.EOS_CS, T_r, 64, 256, kappa=kap, tau=1.0, k=k, force=force))
            r0.append(inputs.slab(64, 256, g, l, 4.0)[0])
            ml.append((g, l))
    b = lbm.Batch(ps, r0)
    _converge(b, len(ps), max_chunks=40)
    print("\n force  T/Tc  rho_l-Maxwell  rho_g-Maxwell")
    off = {}
    for i, p in enumerate(ps):
        r = b.moments(i)[0]
        g, l = ml[i]
        dl, dg = r[128, 0] / l - 1, r[0, 0] / g - 1
        name = "SC" if p.force == lbm.FORCE_SC else "CP"
        off[(name, p.T_r)] = dg
        print(" %s     %.1f   %+.2e      %+.2e" % (name, p.T_r, dl, dg), flush=True)
        assert abs(dl) <= 1e-4
        assert dg > 0
    for T_r in temps:
        assert off[("SC", T_r)] > off[("CP", T_r)]


def _spreading(Re, k, W, collision, rates, steps=3600):
    """A drop of diameter D = 100 falling at U = 0.1 onto a film 30 nodes
    thick in a 1000 x 300 box between walls (Sec. 5.5: PR, T/Tc = 0.6,
    limit 6, tau from Re = U D / nu); the spreading radius r is half the
    width of the liquid run through the impact point on the row two nodes
    above the film, at t* = U (t - t_impact) / D."""
    nx, ny, D, U, film = 1000, 300, 100.0, 0.1, 30
    tau = 3 * U * D / Re + 0.5
    w1 = float(mp.re(A.EOS(A.EOS_PR).interface(0.6)["width1"]))
    g, l = A.coexistence(A.EOS_PR, 0.6)
    p = lbm.params(lbm.EOS_PR, 0.6, nx, ny, kappa=(W * k / w1) ** 2, tau=tau, k=k, mu_cap=6.0,
                   bc_y=1, collision=collision, rates=rates)
    y0 = film + D / 2 + 5.0
    rho0, ux0, uy0 = inputs.splash(nx, ny, g, l, D / 2, W, film=film, drop_center=(nx / 2, y0),
                                   drop_uy=-U)
    s = lbm.Solver(p, rho0, ux0, uy0)
    t_imp = (y0 - D / 2 - film) / U
    half = 0.5 * (g + l)
    pts = []
    for n in range(100, steps + 1, 100):
        s.step(100)
        row = s.moments()[0][film + 2, :]
        assert np.isfinite(row).all()
        liq = row > half
        c = nx // 2
        if not liq[c]:
            continue
        a, b = c, c
        while a > 0 and liq[a - 1]:
            a -= 1
        while b < nx - 1 and liq[b + 1]:
            b += 1
        pts.append((U * (n - t_imp) / D, (b - a + 1) / 2.0 / D))
    s.close()
    return pts


@pytest.mark.parametrize("Re,k,W,collision,rates", [
    (40, 0.1, 6.0, lbm.COLLISION_BGK, lbm.MRT_RATES),
    (150, 0.1, 8.0, lbm.COLLISION_MRT, (1.64, 1.54, 1.2))])
def test_drop_spreading_law(Re, k, W, collision, rates):
    """Sec. 5.5, Fig. 11: after impact the spreading radius follows
    r/D ~ C sqrt(U t / D) with C near 1.3 (the two-dimensional value the
    paper quotes).  Measured C = (r/D)/sqrt(t*) over t* = 0.5 ... 1.5 lies in
    1.25 ... 1.5 at Re = 40 (BGK) and Re = 150 (MRT), and the power-law
    exponent fitted over t* = 0.1 ... 1.5 in 0.55 ... 0.7.  Re = 400 (the
    paper's Fig. 14) diverges in the first 100 steps with every setting tried
    (BGK and MRT, k = 0.05 and 0.1, limit 6)."""
    pts = _spreading(Re, k, W, collision, rates)
    C = [r / np.sqrt(t) for t, r in pts if 0.5 <= t <= 1.5]
    sel = [(t, r) for t, r in pts if 0.1 <= t <= 1.5]
    expo, logc = np.polyfit(np.log([t for t, _ in sel]), np.log([r for _, r in sel]), 1)
    print("\nRe %d: t* r/D: %s" % (Re, " ".join("%.2f:%.3f" % q for q in pts[1:24:3])))
    print("Re %d: C over t* 0.5-1.5: %.3f ... %.3f; fit exponent %.3f, C %.3f" % (
        Re, min(C), max(C), expo, np.exp(logc)), flush=True)
    assert 1.2 <= min(C) and max(C) <= 1.55
    assert 0.5 <= expo <= 0.72


def _splash_run(Re, collision, rates, cap, steps, check=100, watch=None):
    """The splash of _spreading (k = 0.1, 6-node interfaces) with the drop's
    velocity following its tanh profile; returns (steps run before the
    density went non-finite or `steps`, the largest density seen in the
    first `watch` steps, the final density or None)."""
    nx, ny, D, U, film, k, W = 1000, 300, 100.0, 0.1, 30, 0.1, 6.0
    w1 = float(mp.re(A.EOS(A.EOS_PR).interface(0.6)["width1"]))
    g, l = A.coexistence(A.EOS_PR, 0.6)
    p = lbm.params(lbm.EOS_PR, 0.6, nx, ny, kappa=(W * k / w1) ** 2, tau=3 * U * D / Re + 0.5,
                   k=k, mu_cap=cap, bc_y=1, collision=collision, rates=rates)
    rho0, ux0, uy0 = inputs.splash(nx, ny, g, l, D / 2, W, film=film,
                                   drop_center=(nx / 2, film + D / 2 + 5.0), drop_uy=-U,
                                   smooth_velocity=True)
    s = lbm.Solver(p, rho0, ux0, uy0)
    peak, done = 0.0, 0
    try:
        while done < steps:
            if watch and done < watch:
                s.step(check)
                peak = max(peak, float(s.moments()[0].max()))
                done += check
            else:
                s.run_until_converged(0.0, check_every=check, max_steps=steps - done)
                done = steps
        rho = s.moments()[0]
        # mass conservation: to round-off, which drifts by up to ~1e-16 of
        # the mass per step (the nine equilibria sum to rho in floating point
        # only to the last bits)
        assert abs(rho.sum() / rho0.sum() - 1.0) < 1e-11
    except lbm.LBMError:
        done, rho = s.steps_taken, None
    s.close()
    return done, peak, rho


def test_upper_limit_carries_the_high_reynolds_splash():
    """Sec. 5.6 and Fig. 14: the drop of Sec. 5.5 (PR, T/Tc = 0.6, density
    ratio 853) at Re = 400 with MRT.  On impact the liquid is compressed past
    1/b = 10.5, where psi' of Eq. 19 has no value; with the upper limit 6 the
    run goes on (mass conserved to round-off), the sheet thrown up from the
    impact breaks into separate liquid pieces (secondary droplets) by
    t* = 4.5, and the film and drop stay finite; without the limit the same
    run goes non-finite within the first 200 steps, as the paper describes.
    At Re = 150 the limit also carries BGK, and at Re = 400 MRT holds where
    BGK does not (the paper's remark that MRT is the more stable).  The
    ghost-moment rate s_q is 1.2 here: with the printed 1.9 this run goes
    non-finite within 100 steps."""
    mrt, bgk = lbm.COLLISION_MRT, lbm.COLLISION_BGK
    rates = (1.64, 1.54, 1.2)
    done, peak, rho = _splash_run(400, mrt, rates, 6.0, 4700, check=50, watch=1000)
    print("\nRe 400 MRT, limit 6: %d steps, peak density %.3f" % (done, peak), flush=True)
    assert done == 4700 and rho is not None
    assert peak > 10.5
    g, l = A.coexistence(A.EOS_PR, 0.6)
    from scipy import ndimage
    pieces = ndimage.label(rho > 0.5 * (g + l))[1]
    print("liquid pieces at t* = 4.5: %d" % pieces, flush=True)
    assert pieces >= 3
    done_nolim = _splash_run(400, mrt, rates, math.inf, 2000)[0]
    done_bgk = _splash_run(400, bgk, lbm.MRT_RATES, 6.0, 2000)[0]
    print("Re 400 without the limit: non-finite after %d steps; BGK with the limit: %d" % (
        done_nolim, done_bgk), flush=True)
    assert done_nolim <= 300 and done_bgk <= 300
    assert _splash_run(150, bgk, lbm.MRT_RATES, 6.0, 3000)[0] == 3000
    assert _splash_run(150, bgk, lbm.MRT_RATES, math.inf, 2000)[0] <= 300


def test_re150_splash_in_a_moving_frame():
    """Sec. 5.5, Fig. 12: the Re = 150 splash (PR, T/Tc = 0.6, D = 100,
    U = 0.1, 1000 x 300 between walls, MRT) in the rest frame and in a frame
    moving at the paper's reference speed 0.03 (walls sliding along).  At
    t* = 0.6, 1.9, 4.5 and 7.5 the moving-frame liquid, shifted back by
    0.03 t (a whole number of nodes at these steps), has the rest frame's
    number of separate liquid pieces and its volume within 0.1 %, and the
    outlines differ by a small fraction of a node on average (the number of
    nodes on one side only, over the number of outline nodes): measured
    0.05, 0.24, 0.56 and 0.90 at the four times."""
    from scipy import ndimage
    nx, ny, D, U, film, k, W, Re = 1000, 300, 100.0, 0.1, 30, 0.1, 8.0, 150
    w1 = float(mp.re(A.EOS(A.EOS_PR).interface(0.6)["width1"]))
    g, l = A.coexistence(A.EOS_PR, 0.6)
    half = 0.5 * (g + l)
    y0 = film + D / 2 + 5.0
    marks = (600, 2000, 4600, 7600)
    out = {}
    for uf in (0.0, 0.03):
        p = lbm.params(lbm.EOS_PR, 0.6, nx, ny, kappa=(W * k / w1) ** 2,
                       tau=3 * U * D / Re + 0.5, k=k, mu_cap=6.0, bc_y=1, wall_ux=uf,
                       collision=lbm.COLLISION_MRT, rates=(1.64, 1.54, 1.2))
        rho0, ux0, uy0 = inputs.splash(nx, ny, g, l, D / 2, W, film=film,
                                       drop_center=(nx / 2, y0), drop_uy=-U, frame_ux=uf)
        s = lbm.Solver(p, rho0, ux0, uy0)
        done = 0
        for m in marks:
            s.step(m - done)
            done = m
            out[(uf, m)] = s.moments()[0]
            assert np.isfinite(out[(uf, m)]).all()
        s.close()
    for m, bound in zip(marks, (0.2, 0.6, 1.5, 2.0)):
        a = out[(0.0, m)] > half
        b = np.roll(out[(0.03, m)], -round(0.03 * m), axis=1) > half
        outline = (a & ~ndimage.binary_erosion(a)).sum()
        disp = (a ^ b).sum() / outline
        pa, pb = ndimage.label(a)[1], ndimage.label(b)[1]
        print("\nt* %.1f: pieces %d / %d, volume %d / %d, outline %d, differing/outline %.3f" % (
            U * (m - (y0 - D / 2 - film) / U) / D, pa, pb, a.sum(), b.sum(), outline, disp),
            flush=True)
        assert pa == pb
        assert abs(int(a.sum()) - int(b.sum())) <= 1e-3 * a.sum()
        assert disp <= bound


def test_contact_angle_follows_the_wall_chemical_potential():
    """Wetting walls (the chemical-potential boundary the paper takes from
    its ref. [45]): a CS drop (T/Tc = 0.7, k = 0.2, 5-node interface) resting
    on the bottom wall of a 192 x 96 box whose walls hold the chemical
    potential at mu_b + dmu, mu_b the coexistence value.  The contact angle
    (from the drop's base half-width a and height h on its axis,
    theta = 2 atan(h / a) for a circular cap) is 90 degrees at dmu = 0 and
    moves monotonically, and nearly linearly, with dmu: a lower wall
    potential wets (the force -rho grad mu draws liquid toward it).
    Measured after 300,000 steps: 68, 80, 91, 100, 110 degrees for
    dmu = -0.2 ... 0.2 (3 million steps give the same angles to a degree)."""
    T_r, k, nx, ny = 0.7, 0.2, 192, 96
    e = A.EOS(A.EOS_CS)
    T, al = e.temperature(T_r)
    g, l = A.coexistence(A.EOS_CS, T_r)
    mub = float(e.mu0(mp.mpf(g), T, al))
    w1 = float(mp.re(e.interface(T_r)["width1"]))
    kap = (5 * k / w1) ** 2
    dmus = (-0.2, -0.1, 0.0, 0.1, 0.2)
    ps = [lbm.params(lbm.EOS_CS, T_r, nx, ny, kappa=kap, tau=1.0, k=k, bc_y=1, wetting=1,
                     mu_wall=mub + d) for d in dmus]
    rho = inputs.droplet(nx, ny, g, l, 32.0, 5.0, center=(nx / 2, -0.5))[0]
    b = lbm.Batch(ps, [rho] * len(ps))
    b.step(300_000)
    half = 0.5 * (g + l)
    theta = []
    print("\n dmu     base a  height h  contact angle")
    for i, d in enumerate(dmus):
        r = b.moments(i)[0]
        assert np.isfinite(r).all()
        a = (r[0] > half).sum() / 2.0
        h = (r[:, nx // 2] > half).sum()
        theta.append(2 * np.degrees(np.arctan(h / a)))
        print(" %+.2f   %5.1f   %3d       %.1f" % (d, a, h, theta[-1]), flush=True)
    assert all(t1 < t2 for t1, t2 in zip(theta, theta[1:]))
    assert abs(theta[2] - 90.0) <= 3.0
    assert theta[0] < 75.0 and theta[-1] > 105.0
