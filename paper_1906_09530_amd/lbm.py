"""ctypes binding of libcplbm (the C ABI declared in include/lbm.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  Host data are numpy float64 arrays; device data are torch
tensors (float64, contiguous, on the GPU), whose pointers are passed as-is.
If the library is not built, ``load()`` raises -- there is no fallback.
"""
import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcplbm.so")

LBM_OK, LBM_NOT_CONVERGED = 0, 1
LBM_E_INVALID, LBM_E_DOMAIN, LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_NONFINITE = -1, -2, -3, -4, -5
EOS_VDW, EOS_RK, EOS_RKS, EOS_PR, EOS_CS = 0, 1, 2, 3, 4

# EOS constants of Sec. 3.2 (a, b), R = 1
EOS_AB = {EOS_VDW: (9 / 49, 2 / 21), EOS_RK: (2 / 49, 2 / 21), EOS_RKS: (2 / 49, 2 / 21),
          EOS_PR: (2 / 49, 2 / 21), EOS_CS: (1.0, 4.0)}


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("bc_y", C.c_int32), ("eos", C.c_int32),
        ("a", C.c_double), ("b", C.c_double), ("R", C.c_double), ("omega", C.c_double),
        ("T_r", C.c_double), ("kappa", C.c_double), ("tau", C.c_double), ("k", C.c_double),
        ("mu_cap", C.c_double), ("cfd_alpha", C.c_double), ("wall_ux", C.c_double),
        ("collision", C.c_int32), ("force", C.c_int32),
        ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double),
        ("wetting", C.c_int32), ("mu_wall", C.c_double),
    ]


COLLISION_BGK, COLLISION_MRT = 0, 1
COLUMN_STREAM = 1  # lbm_set_column_shape chunk: strips streamed down the columns
FORCE_CP, FORCE_SC = 0, 1
# MRT relaxation rates s_e, s_eps, s_q of the paper (Sec. 2, after Eq. 4)
MRT_RATES = (1.64, 1.54, 1.9)


def params(eos, T_r, nx, ny, *, kappa, tau, k, mu_cap=math.inf, cfd_alpha=1.0 / 3.0, bc_y=0,
           wall_ux=0.0, omega=0.344, a=None, b=None, R=1.0, collision=COLLISION_BGK,
           force=FORCE_CP, rates=MRT_RATES, wetting=0, mu_wall=0.0):
    da, db = EOS_AB[eos]
    return Params(nx=nx, ny=ny, bc_y=bc_y, eos=eos, a=da if a is None else a,
                  b=db if b is None else b, R=R, omega=omega, T_r=T_r, kappa=kappa, tau=tau,
                  k=k, mu_cap=mu_cap, cfd_alpha=cfd_alpha, wall_ux=wall_ux,
                  collision=collision, force=force, s_e=rates[0], s_eps=rates[1],
                  s_q=rates[2], wetting=wetting, mu_wall=mu_wall)


class LBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (status_string(status), msg))
        self.status = status


_lib = None


def load():
    """Load libcplbm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcplbm.so is not built (run python -m paper_1906_09530_amd.build)")
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes the library bind to that one copy, so device buffers and
    # streams are shared with torch (a second runtime copy would be loaded if
    # the order were reversed, and torch could then not see the GPU).
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, d, i32, i64 = C.c_void_p, C.c_double, C.c_int, C.c_int64
    pp = C.POINTER(Params)
    pd = C.POINTER(C.c_double)
    sigs = {
        "lbm_critical_point": (i32, [pp, pd, pd, pd]),
        "lbm_maxwell": (i32, [pp, pd, pd]),
        "lbm_workspace_bytes": (C.c_size_t, [pp]),
        "lbm_init": (i32, [pp, P, P, P, i32, P, P, C.POINTER(P)]),
        "lbm_step": (i32, [P, i64]),
        "lbm_moments": (i32, [P, P, P, P, i32]),
        "lbm_force_fields": (i32, [P, P, P, P, i32]),
        "lbm_run_until_converged": (i32, [P, d, i64, i64, C.POINTER(i64), pd]),
        "lbm_get_state": (i32, [P, P, i32]),
        "lbm_set_state": (i32, [P, P, i32]),
        "lbm_time_passes": (i32, [P, i64, pd]),
        "lbm_set_graph_steps": (i32, [P, i64]),
        "lbm_time_step_kernels": (i32, [P, i64, pd, C.POINTER(C.c_int)]),
        "lbm_eos_values": (i32, [pp, d, pd, pd]),
        "lbm_autotune": (i32, [P, i32, C.POINTER(C.c_int), C.POINTER(C.c_int), pd,
                            C.POINTER(C.c_int)]),
        "lbm_set_column_shape": (i32, [P, i32, i32]),
        "lbm_set_collision_variant": (i32, [P, i32]),
        "lbm_step_noalloc": (i32, [pp, P, i64, P]),
        "lbm_steps_taken": (i64, [P]),
        "lbm_synchronize": (i32, [P]),
        "lbm_destroy": (None, [P]),
        "lbm_last_error": (C.c_char_p, [P]),
        "lbm_status_string": (C.c_char_p, [i32]),
        "lbm_batch_create": (i32, [i32, pp, C.POINTER(P), C.POINTER(P), C.POINTER(P),
                                   C.POINTER(P)]),
        "lbm_batch_set_column_shape": (i32, [P, i32, i32]),
        "lbm_batch_autotune": (i32, [P, i32, C.POINTER(C.c_int), C.POINTER(C.c_int), pd,
                                     C.POINTER(C.c_int)]),
        "lbm_batch_step": (i32, [P, i64]),
        "lbm_batch_run_until_converged": (i32, [P, d, i64, i64, i32, C.POINTER(i64), pd,
                                                C.POINTER(C.c_int32)]),
        "lbm_batch_moments": (i32, [P, i32, P, P, P]),
        "lbm_batch_get_state": (i32, [P, i32, P]),
        "lbm_batch_steps": (i64, [P, i32]),
        "lbm_batch_destroy": (None, [P]),
        "lbm_batch_last_error": (C.c_char_p, [P]),
        "lbm_mlp_create": (i32, [P, P, C.POINTER(P)]),
        "lbm_mlp_get_params": (i32, [P, P]),
        "lbm_mlp_set_params": (i32, [P, P]),
        "lbm_mlp_forward": (i32, [P, P, i64, P, i32]),
        "lbm_mlp_loss_grad": (i32, [P, P, P, i64, C.POINTER(C.c_float), P]),
        "lbm_mlp_train": (i32, [P, P, P, i64, P, i64, i64, C.c_float, C.c_float, C.c_float,
                                C.c_float, P]),
        "lbm_mlp_steps": (i64, [P]),
        "lbm_mlp_set_reach": (i32, [P, d]),
        "lbm_warm_start_drop": (i32, [P, pp, d, d, d, d, i32, P, P, P]),
        "lbm_set_velocity": (i32, [P, P, P, i32]),
        "lbm_batch_set_velocity": (i32, [P, i32, P, P]),
        "lbm_mlp_destroy": (None, [P]),
        "lbm_mlp_last_error": (C.c_char_p, [P]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(s):
    return load().lbm_status_string(s).decode()


def _check(st, ctx=None, ok=(LBM_OK,)):
    if st not in ok:
        raise LBMError(st, load().lbm_last_error(ctx).decode())
    return st


def critical_point(p):
    Tc, rc, pc = C.c_double(), C.c_double(), C.c_double()
    _check(load().lbm_critical_point(C.byref(p), C.byref(Tc), C.byref(rc), C.byref(pc)))
    return Tc.value, rc.value, pc.value


def maxwell(p):
    g, l = C.c_double(), C.c_double()
    _check(load().lbm_maxwell(C.byref(p), C.byref(g), C.byref(l)))
    return g.value, l.value


def eos_values(p, rho):
    """(p0(rho), psi'(rho)) at p.T_r, momentum units (Eqs. 14-21)."""
    a, b = C.c_double(), C.c_double()
    _check(load().lbm_eos_values(C.byref(p), float(rho), C.byref(a), C.byref(b)))
    return a.value, b.value


def workspace_bytes(p):
    return load().lbm_workspace_bytes(C.byref(p))


def _is_device(a):
    return a is not None and hasattr(a, "data_ptr") and getattr(a, "is_cuda", False)


def _ptr(a):
    """Pointer of a host numpy array or a device torch tensor (float64, contiguous)."""
    if a is None:
        return None
    if _is_device(a):
        import torch
        assert a.dtype == torch.float64 and a.is_contiguous()
        return a.data_ptr()
    assert isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data


NOALLOC_MAX_NODES = 262144


def step_noalloc(p, f, nsteps, stream=None):
    """lbm_step_noalloc: advance the device state f (a float64 torch tensor of
    9 * nx * ny, contiguous) by nsteps in place, with no device allocation."""
    assert _is_device(f)
    _check(load().lbm_step_noalloc(C.byref(p), _ptr(f), int(nsteps), stream), None)


class Solver:
    """One simulation (an lbm_ctx)."""

    def __init__(self, p, rho0, ux0=None, uy0=None, stream=None, device_ws=None):
        lib = load()
        self.p = p
        self.shape = (p.ny, p.nx)
        on_dev = _is_device(rho0)
        if not on_dev:
            rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
            ux0 = None if ux0 is None else np.ascontiguousarray(ux0, dtype=np.float64)
            uy0 = None if uy0 is None else np.ascontiguousarray(uy0, dtype=np.float64)
        self._keep = (rho0, ux0, uy0, device_ws)
        ctx = C.c_void_p()
        st = lib.lbm_init(C.byref(p), _ptr(rho0), _ptr(ux0), _ptr(uy0), int(on_dev), stream,
                          None if device_ws is None else device_ws.data_ptr(), C.byref(ctx))
        _check(st, None)
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            load().lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(load().lbm_step(self.ctx, int(n)), self.ctx)

    def synchronize(self):
        _check(load().lbm_synchronize(self.ctx), self.ctx)

    @property
    def steps_taken(self):
        return load().lbm_steps_taken(self.ctx)

    def _outs(self, k, device):
        if device:
            import torch
            return [torch.empty(self.shape, dtype=torch.float64, device="cuda") for _ in range(k)]
        return [np.empty(self.shape) for _ in range(k)]

    def moments(self, device=False):
        """(rho, vx, vy) with v = u + F/(2 rho)."""
        r, vx, vy = self._outs(3, device)
        _check(load().lbm_moments(self.ctx, _ptr(r), _ptr(vx), _ptr(vy), int(device)), self.ctx)
        return r, vx, vy

    def force_fields(self, device=False):
        """(mu, Fx, Fy): mesh chemical potential (Eq. 33) and force (Eq. 12)."""
        mu, fx, fy = self._outs(3, device)
        _check(load().lbm_force_fields(self.ctx, _ptr(mu), _ptr(fx), _ptr(fy), int(device)),
               self.ctx)
        return mu, fx, fy

    def run_until_converged(self, tol, check_every=100, max_steps=10 ** 7):
        steps, delta = C.c_int64(), C.c_double()
        st = load().lbm_run_until_converged(self.ctx, tol, int(check_every), int(max_steps),
                                            C.byref(steps), C.byref(delta))
        _check(st, self.ctx, ok=(LBM_OK, LBM_NOT_CONVERGED))
        return st, steps.value, delta.value

    def time_passes(self, n):
        """Average device ms of the three passes of a step over n steps."""
        out = (C.c_double * 3)()
        _check(load().lbm_time_passes(self.ctx, int(n), out), self.ctx)
        return list(out)

    def set_graph_steps(self, n):
        """Replay whole runs of n steps (rounded up to even) from captured
        HIP graphs in step() and run_until_converged(); 0 launches kernel by
        kernel."""
        _check(load().lbm_set_graph_steps(self.ctx, int(n)), self.ctx)

    def time_step_kernels(self, n):
        """Average ms of each kernel over n real steps (events around every
        launch inside the sequence): row pass A, column pass B, collision."""
        ms = (C.c_double * 3)()
        cnt = C.c_int()
        _check(load().lbm_time_step_kernels(self.ctx, int(n), ms, C.byref(cnt)), self.ctx)
        return list(ms)[:cnt.value]

    def autotune(self, repeats=20):
        """Pick the fastest column-pass shape and collision variant; returns
        {(width, chunk): ms} (chunk 0: the general reduction kernel; chunk < 0:
        tiles with windows; chunk COLUMN_STREAM: streamed strips; (0, v):
        collision variant v)."""
        w = (C.c_int * 27)()
        ch = (C.c_int * 27)()
        ms = (C.c_double * 27)()
        n = C.c_int()
        _check(load().lbm_autotune(self.ctx, int(repeats), w, ch, ms, C.byref(n)), self.ctx)
        return {(w[i], ch[i]): ms[i] for i in range(n.value)}

    def set_collision_variant(self, variant):
        """0: one pass reading f twice; 1: one pass, f in registers; 2: over
        896-node row segments with derivative windows (rows of more than 896
        nodes; the only variant beyond 4096)."""
        _check(load().lbm_set_collision_variant(self.ctx, int(variant)), self.ctx)

    def set_column_shape(self, width, chunk):
        """Strip width and chunk of the column pass (chunk 0: general
        reduction kernel; negative: tiles with windows; COLUMN_STREAM: strips
        of 8, 16 or 32 columns streamed down the columns in tiles)."""
        _check(load().lbm_set_column_shape(self.ctx, int(width), int(chunk)), self.ctx)

    def get_state(self, device=False):
        if device:
            import torch
            f = torch.empty((9,) + self.shape, dtype=torch.float64, device="cuda")
        else:
            f = np.empty((9,) + self.shape)
        _check(load().lbm_get_state(self.ctx, _ptr(f), int(device)), self.ctx)
        return f

    def set_velocity(self, vx=None, vy=None):
        """Fluid velocity v = u + F/(2 rho) of the current density (None: rest)."""
        dev = _is_device(vx) or _is_device(vy)
        if not dev:
            vx = None if vx is None else np.ascontiguousarray(vx, dtype=np.float64)
            vy = None if vy is None else np.ascontiguousarray(vy, dtype=np.float64)
        self._vkeep = (vx, vy)
        _check(load().lbm_set_velocity(self.ctx, _ptr(vx), _ptr(vy), int(dev)), self.ctx)

    def set_state(self, f):
        dev = _is_device(f)
        if not dev:
            f = np.ascontiguousarray(f, dtype=np.float64)
        _check(load().lbm_set_state(self.ctx, _ptr(f), int(dev)), self.ctx)


def _bcheck(st, b=None, ok=(LBM_OK,)):
    if st not in ok:
        raise LBMError(st, load().lbm_batch_last_error(b).decode())
    return st


class Batch:
    """Independent simulations stepped together (an lbm_batch): one launch per
    pass covers every active simulation; converged ones drop out."""

    def __init__(self, plist, rho0s, ux0s=None, uy0s=None):
        lib = load()
        n = len(plist)
        if len(rho0s) != n:
            raise ValueError("one initial density per simulation")
        self.plist = list(plist)
        self.n = n
        arr = (Params * n)(*plist)

        def host(a):
            return None if a is None else np.ascontiguousarray(a, dtype=np.float64)

        rho0s = [host(a) for a in rho0s]
        ux0s = [None] * n if ux0s is None else [host(a) for a in ux0s]
        uy0s = [None] * n if uy0s is None else [host(a) for a in uy0s]
        self._keep = (arr, rho0s, ux0s, uy0s)

        def ptrs(lst):
            return (C.c_void_p * n)(*[None if a is None else a.ctypes.data for a in lst])

        b = C.c_void_p()
        st = lib.lbm_batch_create(n, arr, ptrs(rho0s), ptrs(ux0s), ptrs(uy0s), C.byref(b))
        _bcheck(st, None)
        self.b = b

    def close(self):
        if getattr(self, "b", None):
            load().lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_column_shape(self, col_elems, chunk):
        _bcheck(load().lbm_batch_set_column_shape(self.b, int(col_elems), int(chunk)), self.b)

    def autotune(self, repeats=20):
        """Pick the fastest batched column-pass shape; {(col_elems, chunk): ms}."""
        ce, ch, ms, k = (C.c_int * 4)(), (C.c_int * 4)(), (C.c_double * 4)(), C.c_int()
        _bcheck(load().lbm_batch_autotune(self.b, int(repeats), ce, ch, ms, C.byref(k)), self.b)
        return {(ce[i], ch[i]): ms[i] for i in range(k.value)}

    def step(self, n=1):
        _bcheck(load().lbm_batch_step(self.b, int(n)), self.b)

    def run_until_converged(self, tol, check_every=100, max_steps=10 ** 7, use_graph=True):
        """Returns (status, steps[], delta[], per-simulation status[])."""
        steps = (C.c_int64 * self.n)()
        delta = (C.c_double * self.n)()
        sts = (C.c_int32 * self.n)()
        st = load().lbm_batch_run_until_converged(self.b, tol, int(check_every), int(max_steps),
                                                  int(bool(use_graph)), steps, delta, sts)
        _bcheck(st, self.b, ok=(LBM_OK, LBM_NOT_CONVERGED, LBM_E_NONFINITE))
        return st, list(steps), list(delta), list(sts)

    def steps_taken(self, sim):
        return load().lbm_batch_steps(self.b, int(sim))

    def set_velocity(self, sim, vx=None, vy=None):
        """Fluid velocity of simulation sim (host arrays; None: rest)."""
        vx = None if vx is None else np.ascontiguousarray(vx, dtype=np.float64)
        vy = None if vy is None else np.ascontiguousarray(vy, dtype=np.float64)
        _bcheck(load().lbm_batch_set_velocity(self.b, int(sim), _ptr(vx), _ptr(vy)), self.b)

    def moments(self, sim):
        p = self.plist[sim]
        r, vx, vy = (np.empty((p.ny, p.nx)) for _ in range(3))
        _bcheck(load().lbm_batch_moments(self.b, int(sim), r.ctypes.data, vx.ctypes.data,
                                         vy.ctypes.data), self.b)
        return r, vx, vy

    def get_state(self, sim):
        p = self.plist[sim]
        f = np.empty((9, p.ny, p.nx))
        _bcheck(load().lbm_batch_get_state(self.b, int(sim), f.ctypes.data), self.b)
        return f


MLP_PARAMS = 17923
MLP_INPUTS, MLP_OUTPUTS = 7, 3


def _mcheck(st, m=None, ok=(LBM_OK,)):
    if st not in ok:
        raise LBMError(st, load().lbm_mlp_last_error(m).decode())
    return st


def _dev_ptr(a, dtype):
    import torch
    assert a.is_cuda and a.dtype == dtype and a.is_contiguous()
    return a.data_ptr()


class MLP:
    """The warm-start network (an lbm_mlp): FP32 parameters on the device,
    trained and evaluated by the library's kernels.  Samples and targets are
    torch device tensors (float32); parameters and gradients cross as numpy
    float32 arrays."""

    def __init__(self, params, stream=None):
        lib = load()
        params = np.ascontiguousarray(params, dtype=np.float32)
        assert params.shape == (MLP_PARAMS,)
        m = C.c_void_p()
        _mcheck(lib.lbm_mlp_create(params.ctypes.data, stream, C.byref(m)), None)
        self.m = m

    def close(self):
        if getattr(self, "m", None):
            load().lbm_mlp_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.empty(MLP_PARAMS, dtype=np.float32)
        _mcheck(load().lbm_mlp_get_params(self.m, out.ctypes.data), self.m)
        return out

    def set_params(self, params):
        params = np.ascontiguousarray(params, dtype=np.float32)
        _mcheck(load().lbm_mlp_set_params(self.m, params.ctypes.data), self.m)

    def forward(self, x, bf16=False):
        """(n, 3) outputs of samples x (n, 7), device tensors."""
        import torch
        n = x.shape[0]
        y = torch.empty((n, MLP_OUTPUTS), dtype=torch.float32, device=x.device)
        _mcheck(load().lbm_mlp_forward(self.m, _dev_ptr(x, torch.float32), n,
                                       _dev_ptr(y, torch.float32), int(bool(bf16))), self.m)
        return y

    def loss_grad(self, x, t):
        import torch
        loss = C.c_float()
        g = np.empty(MLP_PARAMS, dtype=np.float32)
        _mcheck(load().lbm_mlp_loss_grad(self.m, _dev_ptr(x, torch.float32),
                                         _dev_ptr(t, torch.float32), x.shape[0], C.byref(loss),
                                         g.ctypes.data), self.m)
        return loss.value, g

    def train(self, x, t, order, batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """Adam steps over consecutive minibatches of `order` (device int32,
        a multiple of batch long); returns the per-step losses."""
        import torch
        iters = order.shape[0] // batch
        losses = np.empty(iters, dtype=np.float32)
        _mcheck(load().lbm_mlp_train(self.m, _dev_ptr(x, torch.float32),
                                     _dev_ptr(t, torch.float32), x.shape[0],
                                     _dev_ptr(order, torch.int32), batch, iters, lr, beta1,
                                     beta2, eps, losses.ctypes.data), self.m)
        return losses

    @property
    def steps(self):
        return load().lbm_mlp_steps(self.m)

    def set_reach(self, reach):
        """Distance from the interface up to which warm-start fields use the
        network (math.inf: everywhere)."""
        _mcheck(load().lbm_mlp_set_reach(self.m, float(reach)), self.m)

    def warm_start_drop(self, p, radius, target_mass, center=None, bf16=True):
        """Warm-start (rho, vx, vy) of a drop: device tensors (ny, nx), float64
        (v is the fluid velocity, for set_velocity)."""
        import torch
        cx, cy = (p.nx / 2.0, p.ny / 2.0) if center is None else center
        out = [torch.empty((p.ny, p.nx), dtype=torch.float64, device="cuda") for _ in range(3)]
        _mcheck(load().lbm_warm_start_drop(self.m, C.byref(p), cx, cy, radius, target_mass,
                                           int(bool(bf16)),
                                           *[_dev_ptr(a, torch.float64) for a in out]), self.m)
        return tuple(out)
