"""Host side of the warm-start workloads (no device call): the drawn drops stay
in their ranges, the Peng-Robinson drops have resolved interfaces, and the
training features and targets assembled on the host follow the network's
definition in the oracle (the definition the library's warm-start field is
checked against on the GPU)."""
import mpmath as mp
import numpy as np
import pytest

from oracle import analytic as A
from oracle import mlp as ref
from paper_1906_09530_amd import lbm, warmstart


@pytest.mark.parametrize("wl", sorted(warmstart.WORKLOADS))
def test_members_are_seeded_and_stay_in_their_ranges(wl):
    r = warmstart.WORKLOADS[wl]["ranges"]
    ms = warmstart.members(5, 192, wl)
    assert ms == warmstart.members(5, 192, wl)
    assert ms != warmstart.members(55, 192, wl)
    for m in ms:
        assert r["t_lo"] <= m["T_r"] < r["t_hi"]
        assert r["r_lo"] <= m["r_frac"] < r["r_hi"]
        assert r["k_lo"] <= m["k"] < r["k_hi"]
    # the draws spread over the ranges
    t = np.array([m["T_r"] for m in ms])
    assert t.min() < r["t_lo"] + 0.1 * (r["t_hi"] - r["t_lo"])
    assert t.max() > r["t_hi"] - 0.1 * (r["t_hi"] - r["t_lo"])


def test_pr_drops_have_resolved_interfaces():
    """Mesh interface width w1 sqrt(kappa) / k (Sec. 5.3) between 8 and 13.5
    nodes over the whole (T/Tc, k) box: w1 grows with T, so the corners
    bound it."""
    w = warmstart.WORKLOADS["pr"]
    r = w["ranges"]
    e = A.EOS(A.EOS_PR)
    w_lo = float(mp.re(e.interface(r["t_lo"])["width1"])) * w["kappa"] ** 0.5 / r["k_hi"]
    w_hi = float(mp.re(e.interface(r["t_hi"])["width1"])) * w["kappa"] ** 0.5 / r["k_lo"]
    assert 8.0 <= w_lo < w_hi <= 13.5
    p = warmstart.drop_params(warmstart.members(5, 1, "pr")[0], 128, "pr")
    assert (p.eos, p.mu_cap, p.kappa, p.tau) == (lbm.EOS_PR, 6.0, 0.003, 1.0)
    assert (p.a, p.b, p.omega) == (2.0 / 49.0, 2.0 / 21.0, 0.344)


@pytest.mark.parametrize("wl", sorted(warmstart.WORKLOADS))
def test_training_features_follow_the_network_definition(wl):
    m = warmstart.members(55, 1, wl)[0]
    n = 64
    radius = m["r_frac"] * n
    d, th = warmstart.geometry(n, radius, np.arange(n * n))
    x = warmstart.features(m, radius, d, th, wl)
    xr = ref.drop_features(m["T_r"], radius, warmstart.WORKLOADS[wl]["kappa"], m["k"], n, n)
    assert x.dtype == np.float32 and x.shape == (n * n, 7)
    np.testing.assert_allclose(x, xr, rtol=1e-6, atol=1e-6)


def test_sample_targets_are_log_density_fraction_and_polar_velocity():
    """A density geometric between the Maxwell pair with exponent s gives the
    density target s; a purely radial velocity of size 2e-3 gives (2, 0) in
    units of 1e-3."""
    m = warmstart.members(5, 1, "pr")[0]
    n = 32
    p = warmstart.drop_params(m, n, "pr")
    g, l = lbm.maxwell(p)
    s = np.linspace(0.0, 1.0, n * n).reshape(n, n)
    rho = g ** (1.0 - s) * l ** s
    y, x = np.meshgrid(np.arange(n) - n / 2.0, np.arange(n) - n / 2.0, indexing="ij")
    ang = np.arctan2(y, x)
    ux, uy = 2e-3 * np.cos(ang), 2e-3 * np.sin(ang)
    feats, t = warmstart.samples(m, p, 10.0, rho, ux, uy, stride=2, wl="pr")
    nodes = (np.arange(0, n, 2)[:, None] * n + np.arange(0, n, 2)[None, :]).ravel()
    assert feats.shape == (len(nodes), 7) and t.shape == (len(nodes), 3)
    np.testing.assert_allclose(t[:, 0], s.ravel()[nodes], rtol=0, atol=1e-6)
    np.testing.assert_allclose(t[:, 1], 2.0, rtol=1e-6)
    np.testing.assert_allclose(t[:, 2], 0.0, atol=1e-6)
