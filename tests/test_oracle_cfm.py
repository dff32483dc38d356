"""Pins of the oracle's compact finite-difference derivative (Sec. 4.3,
Eqs. 37-39): brute-force dense solves, the closed-form Fourier response,
convergence order and exact invariants."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _dense(n, al, a, b):
    """Eq. 37 written out as full n x n periodic matrices (h = 1)."""
    L = np.eye(n)
    Rm = np.zeros((n, n))
    for i in range(n):
        L[i, (i - 1) % n] += al
        L[i, (i + 1) % n] += al
        Rm[i, (i + 1) % n] += a / 2
        Rm[i, (i - 1) % n] -= a / 2
        Rm[i, (i + 2) % n] += b / 4
        Rm[i, (i - 2) % n] -= b / 4
    return L, Rm


def test_sixth_order_coefficients_printed(golden_dir):
    """Eq. 38 at alpha = 1/3 gives the printed coefficients of Eq. 39."""
    g = json.load(open(os.path.join(golden_dir, "paper_printed.json")))["cfm_sixth_order"]
    al = Fraction(*g["alpha"])
    assert Fraction(2, 3) * (al + 2) == Fraction(*g["a"])
    assert Fraction(1, 3) * (4 * al - 1) == Fraction(*g["b"])
    # and the oracle with alpha = 1/3 solves exactly the system of Eq. 39
    n = 12
    u = np.random.default_rng(3).standard_normal(n)
    L, Rm = _dense(n, 1 / 3, 14 / 9, 1 / 9)
    np.testing.assert_allclose(oracle.cfm_line(u, 1 / 3), np.linalg.solve(L, Rm @ u),
                               rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [3, 4, 5, 7, 8, 13, 16])
@pytest.mark.parametrize("al", [1 / 3, 1 / 4])
def test_dense_brute_force(n, al):
    a, b = 2 * (al + 2) / 3, (4 * al - 1) / 3
    u = np.random.default_rng(n).standard_normal(n)
    L, Rm = _dense(n, al, a, b)
    ref = np.linalg.solve(L, Rm @ u)
    np.testing.assert_allclose(oracle.cfm_line(u, al), ref, rtol=0, atol=2e-15 * n)


@pytest.mark.parametrize("al", [1 / 3, 1 / 4])
@pytest.mark.parametrize("n", [64, 100, 257])
def test_fourier_response(al, n):
    """For u_j = exp(i theta j) the scheme returns i k'(theta) u_j with
    k'(theta) = (a sin theta + (b/2) sin 2 theta) / (1 + 2 alpha cos theta)."""
    a, b = 2 * (al + 2) / 3, (4 * al - 1) / 3
    j = np.arange(n)
    for m in [1, 5, n // 4, n // 2 - 1]:
        th = 2 * np.pi * m / n
        kp = (a * np.sin(th) + b / 2 * np.sin(2 * th)) / (1 + 2 * al * np.cos(th))
        ph = 2 * np.pi * ((m * j) % n) / n      # exact phase reduction
        np.testing.assert_allclose(oracle.cfm_line(np.cos(ph), al), -kp * np.sin(ph),
                                   rtol=0, atol=2e-14)
        np.testing.assert_allclose(oracle.cfm_line(np.sin(ph), al), kp * np.cos(ph),
                                   rtol=0, atol=2e-14)


@pytest.mark.parametrize("al,order", [(1 / 4, 4), (1 / 3, 6)])
def test_convergence_order(al, order):
    """Formal order 4 at alpha = 1/4 and 6 at alpha = 1/3 (Sec. 4.3) on a
    smooth periodic function."""
    errs = []
    ns = [16, 32]
    for n in ns:
        h = 2 * np.pi / n
        x = h * np.arange(n)
        u = np.exp(np.sin(x))
        du = np.cos(x) * u
        errs.append(np.abs(oracle.cfm_line(u, al) / h - du).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 0.3


def test_constant_and_sum_invariants():
    """D(const) = 0 exactly (antisymmetric stencil); sum_i (Du)_i = 0 to
    round-off (the periodic derivative has zero mean)."""
    for al in (1 / 3, 1 / 4):
        np.testing.assert_array_equal(oracle.cfm_line(np.full(40, 3.7), al), 0.0)
        u = np.random.default_rng(7).standard_normal(97)
        assert abs(oracle.cfm_line(u, al).sum()) < 1e-13


def test_second_derivative_by_repetition():
    """Applying the scheme twice (Sec. 4.3) gives the response -k'(theta)^2."""
    n, al = 128, 1 / 3
    a, b = 2 * (al + 2) / 3, (4 * al - 1) / 3
    j = np.arange(n)
    for m in [3, 20, 63]:
        th = 2 * np.pi * m / n
        kp = (a * np.sin(th) + b / 2 * np.sin(2 * th)) / (1 + 2 * al * np.cos(th))
        d2 = oracle.cfm_line(oracle.cfm_line(np.cos(th * j), al), al)
        np.testing.assert_allclose(d2, -kp * kp * np.cos(th * j), rtol=0, atol=1e-13)


@pytest.mark.parametrize("al", [1 / 3, 1 / 4])
@pytest.mark.parametrize("ny", [16, 40, 64])
def test_wall_columns_closed_form(al, ny):
    """Between walls (half a node beyond the first and last rows) a column is
    differentiated on its even extension (the neighbour-node condition of
    Sec. 5.5).  u(y) = cos(theta (y + 1/2)) with theta = pi m / ny is even
    about both walls, so its extension is one Fourier mode of the 2 ny line:
    the scheme returns exactly -k'(theta) sin(theta (y + 1/2)), and applied
    twice -k'(theta)^2 u.  A mirror shifted by one node, or an odd extension,
    breaks both."""
    from oracle import analytic as A
    a, b = 2 * (al + 2) / 3, (4 * al - 1) / 3
    nx = 3
    p = A.params(A.EOS_CS, 0.7, nx, ny, kappa=0.0, tau=1.0, k=1.0, cfd_alpha=al, bc_y=1)
    y = np.arange(ny)
    for m in [1, 3, ny // 2, ny - 1]:
        th = np.pi * m / ny
        kp = (a * np.sin(th) + b / 2 * np.sin(2 * th)) / (1 + 2 * al * np.cos(th))
        ph = np.pi * ((m * (2 * y + 1)) % (4 * ny)) / (2 * ny)   # theta (y + 1/2), reduced
        u = np.repeat(np.cos(ph)[:, None], nx, axis=1)
        d1 = oracle.cfm_columns(p, u)
        d2 = oracle.cfm_columns(p, u, second=True)
        np.testing.assert_allclose(d1[:, 0], -kp * np.sin(ph), rtol=0, atol=4e-14)
        np.testing.assert_allclose(d2[:, 1], -kp * kp * np.cos(ph), rtol=0, atol=4e-14)
    # and the extension's dense system (2 ny periodic line) on a random column
    u = np.random.default_rng(ny).standard_normal((ny, nx))
    L, Rm = _dense(2 * ny, al, a, b)
    for x in range(nx):
        ext = np.concatenate([u[:, x], u[::-1, x]])
        ref = np.linalg.solve(L, Rm @ ext)[:ny]
        np.testing.assert_allclose(oracle.cfm_columns(p, u)[:, x], ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("al", [1 / 3, 1 / 4])
@pytest.mark.parametrize("ny", [16, 40])
def test_wetting_wall_columns_closed_form(al, ny):
    """A wetting wall holds the chemical potential at its value u_w: the
    column of u - u_w is extended oddly about both wall planes.
    u(y) = u_w + sin(theta (y + 1/2)), theta = pi m / ny, is odd about both
    walls around u_w, so its extension is one Fourier mode of the 2 ny line
    and the scheme returns exactly k'(theta) cos(theta (y + 1/2)); a random
    column matches the dense solve of the explicitly extended line."""
    from oracle import analytic as A
    a, b = 2 * (al + 2) / 3, (4 * al - 1) / 3
    nx, u_w = 3, 0.37
    p = A.params(A.EOS_CS, 0.7, nx, ny, kappa=0.0, tau=1.0, k=1.0, cfd_alpha=al, bc_y=1,
                 wetting=1, mu_wall=u_w)
    y = np.arange(ny)
    for m in [1, 2, ny // 2, ny - 1]:
        th = np.pi * m / ny
        kp = (a * np.sin(th) + b / 2 * np.sin(2 * th)) / (1 + 2 * al * np.cos(th))
        ph = np.pi * ((m * (2 * y + 1)) % (4 * ny)) / (2 * ny)
        u = np.repeat((u_w + np.sin(ph))[:, None], nx, axis=1)
        d = oracle.cfm_columns_wall_value(p, u, u_w)
        np.testing.assert_allclose(d[:, 1], kp * np.cos(ph), rtol=0, atol=4e-14)
    u = np.random.default_rng(ny + 1).standard_normal((ny, nx))
    L, Rm = _dense(2 * ny, al, a, b)
    for x in range(nx):
        ext = np.concatenate([u[:, x] - u_w, -(u[::-1, x] - u_w)])
        ref = np.linalg.solve(L, Rm @ ext)[:ny]
        np.testing.assert_allclose(oracle.cfm_columns_wall_value(p, u, u_w)[:, x], ref,
                                   rtol=0, atol=1e-13)
