"""Physics of the converged solver against the thermodynamics the paper fixes
(Sec. 5.1 coexistence, Sec. 5.3 Laplace's law), run as batches on the GPU.

The pins come from the oracle's arbitrary-precision thermodynamics (Maxwell
construction, planar-interface surface tension), not from the solver.  The
bounds follow what the BGK scheme with the exact-difference force reaches at
these settings (measured; the deviations are properties of the scheme, shared
by the oracle):

* flat slab, CS, T/Tc = 0.85, k = 0.2, 8-node interface: liquid within 1e-4 of
  Maxwell, gas within 1e-3 (measured 4e-6 and 1.1e-4);
* drops, same settings, R = 32 ... 96 (radius at least four interface
  widths): the pressure jump k^2 [p0(rho_in) - p0(rho_out)] times the
  equimolar radius is the same for every drop to 3 % (Laplace's law, measured
  1.2 %); the surface tension it implies exceeds the continuum
  sigma = k sqrt(kappa) sigma_1 by 1.77x.  The flat interface shows why: the
  forced lattice carries a bare velocity u = -F/(2 rho) inside the interface,
  whose momentum flux F F/(4 rho) adds normal stress; summed over the
  interface it is of the size of the excess (it predicts 2.2x).
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import analytic as A
from paper_1906_09530_amd import inputs, lbm

pytestmark = pytest.mark.gpu

T_R, K, W = 0.85, 0.2, 8.0


def _settings():
    e = A.EOS(A.EOS_CS)
    it = e.interface(T_R)
    w1 = float(mp.re(it["width1"]))
    kappa = (W * K / w1) ** 2
    return e, it, kappa


def _converge(b, n, max_chunks=20):
    for _ in range(max_chunks):
        st, _, _, sts = b.run_until_converged(1e-12, 100, 50_000)
        if all(s != lbm.LBM_NOT_CONVERGED for s in sts):
            break
    assert all(s == lbm.LBM_OK for s in sts), sts


def test_flat_slab_meets_the_maxwell_densities():
    _, _, kappa = _settings()
    g, l = A.coexistence(A.EOS_CS, T_R)
    nx, ny = 64, 384
    p = lbm.params(lbm.EOS_CS, T_R, nx, ny, kappa=kappa, tau=1.0, k=K)
    b = lbm.Batch([p], [inputs.slab(nx, ny, g, l, W)[0]])
    _converge(b, 1)
    r = b.moments(0)[0]
    rl, rg = r[ny // 2, 0], r[0, 0]
    print("\nslab T/Tc %.2f: rho_l %+.2e, rho_g %+.2e relative to Maxwell" % (
        T_R, rl / l - 1, rg / g - 1), flush=True)
    assert abs(rl / l - 1) <= 1e-4
    assert abs(rg / g - 1) <= 1e-3
    assert (r == r[:, :1]).all()  # stays flat


def test_drops_follow_laplaces_law():
    e, it, kappa = _settings()
    T, al = it["T"], it["alpha"]
    sigma = K * kappa ** 0.5 * float(mp.re(it["sigma1"]))
    g, l = A.coexistence(A.EOS_CS, T_R)
    radii = (32, 48, 64, 96)
    ps, r0 = [], []
    for R in radii:
        n = int(8 * ((2 * R + 12 * W) // 8 + 1))
        ps.append(lbm.params(lbm.EOS_CS, T_R, n, n, kappa=kappa, tau=1.0, k=K))
        r0.append(inputs.droplet(n, n, g, l, R, W)[0])
    b = lbm.Batch(ps, r0)
    _converge(b, len(radii))
    inv_r, dp = [], []
    for i, p in enumerate(ps):
        r = b.moments(i)[0]
        n = p.nx
        rin, rout = r[n // 2, n // 2], r[0, 0]
        req = float(np.sqrt((r - rout).sum() / (np.pi * (rin - rout))))  # equimolar radius
        inv_r.append(1.0 / req)
        dp.append(K * K * float(mp.re(e.p0(mp.mpf(rin), T, al) - e.p0(mp.mpf(rout), T, al))))
    jump_r = np.array(dp) / np.array(inv_r)  # sigma implied by each drop
    print("\nLaplace: dP R = %s (continuum sigma %.4e)" % (
        " ".join("%.4e" % v for v in jump_r), sigma), flush=True)
    assert np.all(np.diff(dp) < 0)                 # smaller drops, larger jump
    assert (jump_r.max() - jump_r.min()) <= 0.03 * jump_r.mean()
    assert 1.3 < jump_r.mean() / sigma < 2.0
