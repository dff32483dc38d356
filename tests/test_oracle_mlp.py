"""Pins of the FP64 warm-start network reference (oracle/mlp.py) against
things other than itself: central finite differences of the loss, closed
forms of special cases, Adam's known first steps, bfloat16 rounding of
exactly representable halfway cases and torch's own conversion."""
import numpy as np
import pytest

from oracle import mlp


def _net(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, mlp.N_PARAMS)


def _data(seed, n=12):
    rng = np.random.default_rng(seed + 100)
    return rng.normal(0.0, 1.0, (n, mlp.N_IN)), rng.normal(0.0, 1.0, (n, mlp.N_OUT))


def test_parameter_count():
    assert mlp.N_PARAMS == 7 * 128 + 128 + 128 * 128 + 128 + 3 * 128 + 3 == 17923


def test_gradient_matches_central_differences_everywhere():
    """Every component of the backpropagated gradient against a central
    difference of the loss with step 1e-5 (error O(h^2) ~ 1e-10)."""
    w = _net(1)
    x, t = _data(1)
    _, g = mlp.grad(w, x, t)
    h = 1e-5
    fd = np.empty_like(w)
    for i in range(w.size):
        wp = w.copy()
        wp[i] += h
        wm = w.copy()
        wm[i] -= h
        fd[i] = (mlp.loss(wp, x, t) - mlp.loss(wm, x, t)) / (2 * h)
    scale = np.abs(g).max()
    assert np.abs(g - fd).max() <= 1e-7 * scale
    # each block is exercised (no block of zeros hiding a dropped term)
    for a in mlp.unpack(g):
        assert np.abs(a).max() > 1e-6 * scale


def test_gradient_with_silent_hidden_layer():
    """W2 = 0, b2 = 0: a2 = 0, so y = b3 for every sample, dL/db3 =
    2 mean(b3 - t) per output, dL/dW3 = 0, dL/dW1 = dL/db1 = 0 (W2 blocks the
    path) and dL/db2 = W3^T dL/db3 (tanh'(0) = 1)."""
    w = _net(2)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(w)
    W2[:] = 0.0
    b2[:] = 0.0
    x, t = _data(2)
    y, _, _ = mlp.forward(w, x)
    assert np.all(y == b3)
    _, g = mlp.grad(w, x, t)
    gW1, gb1, gW2, gb2, gW3, gb3 = mlp.unpack(g)
    np.testing.assert_allclose(gb3, 2.0 * np.mean(b3 - t, axis=0), rtol=1e-14)
    assert np.all(gW3 == 0.0) and np.all(gW1 == 0.0) and np.all(gb1 == 0.0)
    np.testing.assert_allclose(gb2, gb3 @ W3, rtol=1e-12, atol=1e-15)


def test_adam_first_steps_move_by_the_learning_rate():
    """With bias correction, step 1 gives m_hat = g and v_hat = g^2, so each
    parameter moves by -lr g / (|g| + eps); a constant gradient keeps that
    on step 2."""
    rng = np.random.default_rng(3)
    w = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr = 1e-3
    w1, m, v = mlp.adam(w, g, m, v, 1, lr)
    assert np.allclose(w1 - w, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    w2, m, v = mlp.adam(w1, g, m, v, 2, lr)
    assert np.allclose(w2 - w1, -lr * g / (np.abs(g) + 1e-8), rtol=1e-10, atol=0)


def test_bf16_rounding_halfway_cases():
    ulp = 2.0 ** -7  # spacing of bfloat16 just above 1
    vals = np.array([1.0, 1.0 + ulp / 2, 1.0 + 1.5 * ulp, 1.0 + ulp / 2 + 2.0 ** -20,
                     -(1.0 + 1.5 * ulp), 3.0, 0.0])
    want = np.array([1.0, 1.0, 1.0 + 2 * ulp, 1.0 + ulp, -(1.0 + 2 * ulp), 3.0, 0.0])
    np.testing.assert_array_equal(mlp.bf16(vals), want)


def test_bf16_matches_torch_conversion():
    import torch
    x = np.random.default_rng(4).normal(0, 10, 10000).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)


def test_bf16_forward_is_close_to_fp64():
    w = _net(5, scale=0.1)
    x, _ = _data(5, n=200)
    y, _, _ = mlp.forward(w, x)
    yb = mlp.forward_bf16(w, x)
    assert np.abs(yb - y).max() < 2e-2 * max(1.0, np.abs(y).max())
    assert np.abs(yb - y).max() > 0.0


def test_density_map_and_mass_match():
    g, l = 1e-4, 0.5
    np.testing.assert_allclose(mlp.density_from_output(np.array([0.0, 1.0]), g, l), [g, l],
                               rtol=1e-14)
    f = mlp.drop_features(0.5, 20.0, 0.1, 0.25, 64, 64)
    d = f[:, 4] * mlp.FEATURE_SCALE[4]
    y = 0.5 * (1.0 - np.tanh(d / 3.0))
    rho = mlp.density_from_output(y, g, l).reshape(64, 64)
    # angle features: node (x, y) = (40, 32) lies on theta = 0, (32, 40) on pi/2
    assert f[32 * 64 + 40, 5] == pytest.approx(1.0) and f[32 * 64 + 40, 6] == pytest.approx(0.0)
    assert f[40 * 64 + 32, 5] == pytest.approx(1.0) and abs(f[40 * 64 + 32, 6]) < 1e-12
    assert f[40 * 64 + 40, 5] == pytest.approx(-1.0)  # theta = pi/4
    target = rho.sum() * (1.0 + 1e-3)
    r2 = mlp.mass_match(rho, target, g, l)
    assert r2.sum() == pytest.approx(target, rel=1e-14)
    far = np.abs(d.reshape(64, 64)) > 30
    assert np.all(r2[far] == rho[far]) or np.abs(r2[far] - rho[far]).max() < 1e-12 * l
    # the features: centre node has r - R = -R; normalisation as documented
    assert f[32 * 64 + 32, 4] == pytest.approx(-20.0 / 8.0)
    assert f[0, 0] == pytest.approx(0.0) and f[0, 1] == pytest.approx((20 / 256 - 0.25) / 0.1)


def test_velocity_from_output_rotates_the_polar_components():
    th = np.array([0.0, np.pi / 2, np.pi, -np.pi / 2])
    y = np.zeros((4, 3))
    y[:, 1] = 2.0   # radial outwards, 2e-3
    ux, uy = mlp.velocity_from_output(y, th)
    np.testing.assert_allclose(ux, [2e-3, 0.0, -2e-3, 0.0], atol=1e-18)
    np.testing.assert_allclose(uy, [0.0, 2e-3, 0.0, -2e-3], atol=1e-18)
    y[:, 1], y[:, 2] = 0.0, 1.0  # azimuthal, counter-clockwise
    ux, uy = mlp.velocity_from_output(y, th)
    np.testing.assert_allclose(ux, [0.0, -1e-3, 0.0, 1e-3], atol=1e-18)
    np.testing.assert_allclose(uy, [1e-3, 0.0, -1e-3, 0.0], atol=1e-18)


def test_symmetric_outputs_are_even_and_odd_under_reflection():
    w = _net(6, scale=0.2)
    x, _ = _data(6, n=40)
    xm = x.copy()
    xm[:, -1] = -xm[:, -1]
    for bf16 in (False, True):
        y, ym = mlp.symmetric_outputs(w, x, bf16), mlp.symmetric_outputs(w, xm, bf16)
        np.testing.assert_allclose(ym[:, :2], y[:, :2], rtol=0, atol=1e-15)
        np.testing.assert_allclose(ym[:, 2], -y[:, 2], rtol=0, atol=1e-15)


def test_reach_weight_blends_to_the_maxwell_gas_at_rest():
    """Weight 1 near the drop, 0 beyond reach + 10 (distances checked on
    nodes along the x axis through the centre, where r - R is exact), 1/2
    at r - R = reach, non-increasing in r; scaled outputs give the Maxwell
    gas density (to round-off) and zero velocity where it is 0, which mass
    matching leaves there."""
    n, R, reach = 128, 20.0, 25.0
    w = mlp.reach_weight(R, n, n, reach).reshape(n, n)
    row = w[n // 2]                            # y = n/2: r = |x - n/2|
    d = np.abs(np.arange(n) - n / 2.0) - R
    assert np.all(row[d <= reach - 10] == 1.0) and np.all(row[d >= reach + 10] == 0.0)
    assert row[n // 2 + 45] == 0.5             # r - R = 25 = reach
    assert row[n // 2 + 40] == 0.75 and row[n // 2 + 50] == 0.25
    dd, _ = mlp.drop_geometry(R, n, n)
    order = np.argsort(dd, kind="stable")
    assert np.all(np.diff(w.ravel()[order]) <= 0.0)
    assert np.all(mlp.reach_weight(R, n, n, np.inf) == 1.0)
    g, l = 1e-5, 0.7
    y = np.full((n * n, 3), 0.3)
    y[:, 0] = 0.5 * (1.0 - np.tanh(dd / 3.0))
    yw = y * w.ravel()[:, None]
    rho = mlp.density_from_output(yw[:, 0], g, l)
    far = w.ravel() == 0.0
    np.testing.assert_allclose(rho[far], g, rtol=1e-15)   # exp(ln g) to round-off
    ux, uy = mlp.drop_velocity(yw, R, n, n)
    assert np.all(ux.ravel()[far] == 0.0) and np.all(uy.ravel()[far] == 0.0)
    r2 = mlp.mass_match(rho.reshape(n, n), rho.sum() * 1.001, g, l)
    np.testing.assert_allclose(r2.ravel()[far], g, rtol=1e-14)
