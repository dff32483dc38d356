"""CPU-side checks of libcplbm: the ABI it exports, its host thermodynamics
against the oracle, and parameter validation (no device call is made)."""
import ctypes as C
import math
import os
import re

import mpmath as mp
import numpy as np
import pytest

from oracle import analytic as A
from paper_1906_09530_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(lbm_\w+)\s*\(", src))
    return names


def test_library_exports_every_declared_entry_point():
    lib = lbm.load()
    names = _declared()
    assert "lbm_init" in names and "lbm_step" in names and "lbm_moments" in names
    assert "lbm_run_until_converged" in names
    for n in sorted(names):
        assert hasattr(lib, n), n


@pytest.mark.parametrize("eos", [0, 1, 2, 3, 4])
def test_critical_point_matches_oracle(eos):
    p = lbm.params(eos, 0.5, 16, 16, kappa=0.0, tau=1.0, k=1.0)
    Tc, rc, pc = lbm.critical_point(p)
    T2, r2, p2 = A.EOS(eos).critical_point()
    assert Tc == pytest.approx(float(T2), rel=1e-14)
    assert rc == pytest.approx(float(r2), rel=1e-14)
    assert pc == pytest.approx(float(p2), rel=1e-13)


@pytest.mark.parametrize("eos,T_r", [(0, 0.6), (1, 0.8), (2, 0.4), (3, 0.3), (3, 0.5),
                                      (4, 0.15), (4, 0.7), (4, 0.95), (3, 0.99)])
def test_maxwell_matches_oracle(eos, T_r):
    p = lbm.params(eos, T_r, 16, 16, kappa=0.0, tau=1.0, k=1.0)
    g, l = lbm.maxwell(p)
    g2, l2 = A.EOS(eos).maxwell(T_r)
    assert g == pytest.approx(float(g2), rel=1e-13)
    assert l == pytest.approx(float(l2), rel=1e-13)


def test_maxwell_rejects_supercritical():
    p = lbm.params(3, 1.2, 16, 16, kappa=0.0, tau=1.0, k=1.0)
    with pytest.raises(lbm.LBMError):
        lbm.maxwell(p)


def _init_status(p, rho):
    ctx = C.c_void_p()
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    st = lbm.load().lbm_init(C.byref(p), rho.ctypes.data, None, None, 0, None, None,
                             C.byref(ctx))
    assert ctx.value is None
    return st, lbm.load().lbm_last_error(None).decode()


@pytest.mark.parametrize("field,value", [("tau", 0.5), ("tau", 0.3), ("k", 0.0), ("kappa", -1.0),
                                          ("nx", 7), ("ny", 5001), ("nx", 4098),
                                          ("ny", 8204), ("ny", 1 << 21), ("nx", 1 << 21),
                                          ("cfd_alpha", 0.3),
                                          ("bc_y", 2), ("eos", 9), ("mu_cap", math.nan),
                                          ("T_r", -0.1), ("wall_ux", math.inf)])
def test_init_rejects_invalid_parameters(field, value):
    p = lbm.params(4, 0.7, 16, 16, kappa=0.1, tau=1.0, k=0.2)
    setattr(p, field, value)
    st, msg = _init_status(p, np.full((16, 16), 0.1))
    assert st == lbm.LBM_E_INVALID and msg
    assert lbm.workspace_bytes(p) == 0


@pytest.mark.parametrize("bad", [0.0, -0.1, math.nan, math.inf])
def test_init_rejects_bad_density(bad):
    p = lbm.params(4, 0.7, 16, 16, kappa=0.1, tau=1.0, k=0.2)
    rho = np.full((16, 16), 0.1)
    rho[3, 5] = bad
    st, _ = _init_status(p, rho)
    assert st == lbm.LBM_E_DOMAIN


def test_init_domain_check_depends_on_the_upper_limit():
    """rho >= 1/b is refused only when the limit of Sec. 5.6 is off."""
    p = lbm.params(3, 0.6, 16, 16, kappa=0.002, tau=1.0, k=0.1)
    rho = np.full((16, 16), 1.0)
    rho[8, 8] = 10.6
    st, msg = _init_status(p, rho)
    assert st == lbm.LBM_E_DOMAIN and "domain" in msg
    p.mu_cap = 6.0
    assert lbm.workspace_bytes(p) > 9 * 2 * 16 * 16 * 8


def _batch_status(plist, rhos):
    n = len(plist)
    arr = (lbm.Params * n)(*plist)
    rhos = [np.ascontiguousarray(r, dtype=np.float64) for r in rhos]
    ptrs = (C.c_void_p * n)(*[r.ctypes.data for r in rhos])
    b = C.c_void_p()
    st = lbm.load().lbm_batch_create(n, arr, ptrs, None, None, C.byref(b))
    assert b.value is None
    return st, lbm.load().lbm_batch_last_error(None).decode()


@pytest.mark.parametrize("nx,ny", [(60, 64), (64, 60), (56, 64), (1032, 64), (64, 2048)])
def test_batch_rejects_sizes_outside_its_range(nx, ny):
    good = lbm.params(4, 0.7, 64, 64, kappa=0.1, tau=1.0, k=0.2)
    bad = lbm.params(4, 0.7, nx, ny, kappa=0.1, tau=1.0, k=0.2)
    st, msg = _batch_status([good, bad], [np.full((64, 64), 0.1), np.full((ny, nx), 0.1)])
    assert st == lbm.LBM_E_INVALID and "simulation 1" in msg


def test_batch_validates_each_simulation():
    good = lbm.params(4, 0.7, 64, 64, kappa=0.1, tau=1.0, k=0.2)
    bad = lbm.params(4, 0.7, 64, 64, kappa=0.1, tau=0.4, k=0.2)
    st, msg = _batch_status([good, bad, good], [np.full((64, 64), 0.1)] * 3)
    assert st == lbm.LBM_E_INVALID and "simulation 1" in msg and "tau" in msg
    rho = np.full((64, 64), 0.1)
    rho[1, 2] = -1.0
    st, msg = _batch_status([good, good], [np.full((64, 64), 0.1), rho])
    assert st == lbm.LBM_E_DOMAIN and "simulation 1" in msg
    st, _ = _batch_status([], [])
    assert st == lbm.LBM_E_INVALID


@pytest.mark.parametrize("eos,T_r", [(0, 0.6), (1, 0.8), (2, 0.5), (3, 0.5), (4, 0.7)])
def test_eos_values_match_oracle(eos, T_r):
    """lbm_eos_values (host long double) against the oracle's mpmath EOS."""
    p = lbm.params(eos, T_r, 16, 16, kappa=0.0, tau=1.0, k=1.0)
    e = A.EOS(eos)
    T, al = e.temperature(T_r)
    g, l = e.maxwell(T_r)
    for r in (float(g), 0.5 * float(g + l), float(l)):
        p0, mu0 = lbm.eos_values(p, r)
        # p0 is a difference of two terms that nearly cancel on the liquid
        # branch: compare on the scale of the repulsive term
        scale = abs(float(r * e.R * T / (1 - e.b * r)))
        assert abs(p0 - float(e.p0(mp.mpf(r), T, al))) <= 1e-13 * scale
        assert mu0 == pytest.approx(float(e.mu0(mp.mpf(r), T, al)), rel=1e-12, abs=1e-15)
    with pytest.raises(lbm.LBMError):
        lbm.eos_values(p, float(e.rho_max()) * 1.01)


@pytest.mark.parametrize("nx,ny", [(4100, 16), (5000, 32), (1 << 20, 8), (16, 5000), (24, 8192),
                                   (16, 9216), (32, 16384), (8192, 8192), (8, 40000),
                                   (8, 1 << 20)])
def test_long_lines_are_accepted(nx, ny):
    """Rows beyond 4096 nodes (a multiple of 4, over windowed segments) and
    columns beyond 4096 (a multiple of 8, over tiles of rows with windows)
    size a workspace."""
    p = lbm.params(4, 0.7, nx, ny, kappa=0.1, tau=1.0, k=0.2, bc_y=1)
    assert lbm.workspace_bytes(p) >= 9 * 2 * 8 * nx * ny
