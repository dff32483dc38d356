"""ctypes front of ``cplbm_oracle.c`` (test infrastructure only).

Every function here marshals numpy arrays and forwards to the C oracle; the
arithmetic lives in the C file, which cites the paper for each step.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cplbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# the same source with OpenMP over lines and nodes (bitwise equal results)
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")

EOS_VDW, EOS_RK, EOS_RKS, EOS_PR, EOS_CS = 0, 1, 2, 3, 4


class OracleParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("bc_y", C.c_int32), ("eos", C.c_int32),
        ("wall_ux", C.c_double), ("a", C.c_double), ("b", C.c_double), ("R", C.c_double),
        ("T", C.c_double), ("alpha_T", C.c_double), ("kappa", C.c_double),
        ("tau", C.c_double), ("k", C.c_double), ("mu_cap", C.c_double),
        ("cfd_alpha", C.c_double), ("collision", C.c_int32), ("force", C.c_int32),
        ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double),
        ("wetting", C.c_int32), ("mu_wall", C.c_double),
    ]


def build(force=False):
    """Compile the oracle with gcc (IEEE order, no FMA contraction): the serial
    library and the OpenMP one."""
    for out, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
            tmp = out + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared"] + extra +
                                  ["-o", tmp, SRC, "-lm"])
            os.replace(tmp, out)
    return LIB


_lib = None
_libs = {}


def threads(n=None):
    """Switch every oracle call to the OpenMP build on n threads (n = None or
    0: all cores), or back to the serial build (n = 1).  Returns the threads
    the calls now use."""
    global _lib
    want_omp = n is None or n != 1
    _lib = _open(LIB_OMP if want_omp else LIB)
    return _lib.orc_threads(0 if n is None else int(n))


def load():
    global _lib
    if _lib is None:
        _lib = _open(LIB)
    return _lib


def _open(path):
    if path not in _libs:
        build()
        lib = C.CDLL(path)
        d, i32, i64, P = C.c_double, C.c_int, C.c_int64, C.c_void_p
        pp = C.POINTER(OracleParams)
        for name, res, args in [
            ("orc_threads", i32, [i32]),
            ("orc_alpha_T", d, [i32, d, d, d]),
            ("orc_p0", d, [i32, d, d, d, d, d, d]),
            ("orc_mu0", d, [i32, d, d, d, d, d, d]),
            ("orc_mu0_capped", d, [pp, d]),
            ("orc_cfm_line", None, [i32, d, P, P]),
            ("orc_cfm_columns", None, [pp, P, P, i32]),
            ("orc_cfm_columns_wall_value", None, [pp, P, d, P]),
            ("orc_feq", d, [i32, d, d, d]),
            ("orc_node_moments", None, [P, P, P, P]),
            ("orc_collide_node", None, [P, d, d, d, d, d, d, P]),
            ("orc_mrt_matrix", None, [P]),
            ("orc_mrt_inverse", None, [P]),
            ("orc_collide_node_mrt", None, [P, d, d, d, d, d, d, d, d, d, P]),
            ("orc_sc_psi", d, [pp, d]),
            ("orc_stream", None, [pp, P, P, P]),
            ("orc_init", None, [pp, P, P, P, P]),
            ("orc_step", None, [pp, P]),
            ("orc_run", None, [pp, P, i64]),
            ("orc_moments", None, [pp, P, P, P, P, P, P, P]),
            ("orc_run_until_converged", i32, [pp, P, d, i64, i64, C.POINTER(i64),
                                              C.POINTER(d)]),
        ]:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _libs[path] = lib
    return _libs[path]


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


def _nullable(a):
    return None if a is None else _ptr(a)


def alpha_T(eos, T, Tc, omega):
    return load().orc_alpha_T(eos, T, Tc, omega)


def p0(eos, a, b, R, T, al, rho):
    f = load().orc_p0
    return np.vectorize(lambda r: f(eos, a, b, R, T, al, float(r)))(rho)


def mu0(eos, a, b, R, T, al, rho):
    f = load().orc_mu0
    return np.vectorize(lambda r: f(eos, a, b, R, T, al, float(r)))(rho)


def mu0_capped(p, rho):
    f = load().orc_mu0_capped
    return np.vectorize(lambda r: f(C.byref(p), float(r)))(rho)


def cfm_line(u, alpha):
    u = np.ascontiguousarray(u, dtype=np.float64)
    d = np.empty_like(u)
    load().orc_cfm_line(len(u), alpha, _ptr(u), _ptr(d))
    return d


def cfm_columns(p, u, second=False):
    """d/dy (or the scheme applied twice) of the field u[ny][nx] as the
    oracle's step takes it (even extension between walls)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    d = np.empty_like(u)
    load().orc_cfm_columns(C.byref(p), _ptr(u), _ptr(d), int(second))
    return d


def cfm_columns_wall_value(p, u, u_w):
    """d/dy of the field u[ny][nx] held at u_w on the walls (odd extension of
    u - u_w), as the oracle's step differentiates the chemical potential
    between wetting walls."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    d = np.empty_like(u)
    load().orc_cfm_columns_wall_value(C.byref(p), _ptr(u), float(u_w), _ptr(d))
    return d


def feq(i, rho, ux, uy):
    return load().orc_feq(i, rho, ux, uy)


def collide_node(fi, rho, ux, uy, Fx, Fy, tau):
    fi = np.ascontiguousarray(fi, dtype=np.float64)
    out = np.empty(9)
    load().orc_collide_node(_ptr(fi), rho, ux, uy, Fx, Fy, tau, _ptr(out))
    return out


def mrt_matrix():
    M = np.empty((9, 9))
    load().orc_mrt_matrix(_ptr(M))
    return M


def mrt_inverse():
    M = np.empty((9, 9))
    load().orc_mrt_inverse(_ptr(M))
    return M


def collide_node_mrt(fi, rho, ux, uy, Fx, Fy, tau, s_e, s_eps, s_q):
    fi = np.ascontiguousarray(fi, dtype=np.float64)
    out = np.empty(9)
    load().orc_collide_node_mrt(_ptr(fi), rho, ux, uy, Fx, Fy, tau, s_e, s_eps, s_q, _ptr(out))
    return out


def sc_psi(p, rho):
    f = load().orc_sc_psi
    return np.vectorize(lambda r: f(C.byref(p), float(r)))(rho)


def stream(p, fstar, rho):
    fstar = np.ascontiguousarray(fstar, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    out = np.full_like(fstar, np.nan)
    load().orc_stream(C.byref(p), _ptr(fstar), _ptr(rho), _ptr(out))
    return out


def init(p, rho0, ux0, uy0):
    f = np.empty((9, p.ny, p.nx))
    args = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho0, ux0, uy0)]
    load().orc_init(C.byref(p), *[_ptr(a) for a in args], _ptr(f))
    return f


def step(p, f):
    load().orc_step(C.byref(p), _ptr(f))
    return f


def run(p, f, nsteps):
    load().orc_run(C.byref(p), _ptr(f), int(nsteps))
    return f


def moments(p, f, want_force=False):
    """rho, v = u + F/(2 rho), and (optionally) mu, Fx, Fy of the state f."""
    sh = (p.ny, p.nx)
    rho, vx, vy, mu, fx, fy = (np.empty(sh) for _ in range(6))
    load().orc_moments(C.byref(p), _ptr(f), _ptr(rho), _ptr(vx), _ptr(vy),
                       _ptr(mu), _ptr(fx), _ptr(fy))
    if want_force:
        return rho, vx, vy, mu, fx, fy
    return rho, vx, vy


def run_until_converged(p, f, tol, every, max_steps):
    steps = C.c_int64(0)
    delta = C.c_double(0.0)
    st = load().orc_run_until_converged(C.byref(p), _ptr(f), tol, int(every), int(max_steps),
                                        C.byref(steps), C.byref(delta))
    return st, steps.value, delta.value
