"""Learned warm start of static drops (orchestration over the C ABI).

The solver converges drops from the tanh start of Eq. 41 (Sec. 5.3, zero
velocity); the converged states become training samples of the network of
include/lbm_warmstart.h, which the library trains with its own FP32 kernels;
the trained network then proposes the initial density and velocity of new
drops (BF16 inference, density mass matched to the tanh start), and both
starts are run to the same convergence criterion.  The solver, the
training, the inference and the warm-start fields run in the library's
kernels; this module draws the workload, forms the training samples on the
host from the converged fields (seven normalised features per sampled node,
and as targets the normalised log density and the radial and azimuthal
velocity: a few elementwise numpy operations on every second node) and
keeps the books.

Workloads (square periodic meshes; T/Tc, radius fraction and k drawn per
drop, tau = 1):

* "cs": Carnahan-Starling drops (a = 1, b = 4, R = 1), kappa = 0.1,
  T/Tc in [0.35, 0.6], k in [0.15, 0.3], radius in [0.15, 0.35] N, tanh
  width 5;
* "pr": Peng-Robinson drops (a = 2/49, b = 2/21, R = 1, omega = 0.344),
  T/Tc in [0.3, 0.5], kappa = 0.003, k in [0.045, 0.055] (interfaces of
  8-13 nodes, w1 sqrt(kappa) / k), the chemical-potential limit at 6,
  radius in [0.22, 0.35] N (drops of 20-25 nodes at T/Tc < 0.39 can diverge
  in the first few hundred steps from the tanh start), tanh width 10.
"""
import math
import time

import numpy as np

from . import inputs, lbm

FEATURE_CENTER = np.array([0.5, 0.25, 0.1, 0.25, 0.0, 0.0, 0.0])
FEATURE_SCALE = np.array([0.25, 0.1, 0.1, 0.1, 8.0, 1.0, 1.0])
R_REF = 256.0
U_SCALE = 1e-3
WORKLOADS = {
    "cs": dict(eos=lbm.EOS_CS, kappa=0.1, tau=1.0, width=5.0, mu_cap=math.inf,
               ranges=dict(t_lo=0.35, t_hi=0.6, r_lo=0.15, r_hi=0.35, k_lo=0.15, k_hi=0.3)),
    "pr": dict(eos=lbm.EOS_PR, kappa=0.003, tau=1.0, width=10.0, mu_cap=6.0,
               ranges=dict(t_lo=0.3, t_hi=0.5, r_lo=0.22, r_hi=0.35, k_lo=0.045, k_hi=0.055)),
}


def members(seed, count, wl="cs"):
    return inputs.warmstart_members(seed, count, **WORKLOADS[wl]["ranges"])


def drop_params(member, n, wl="cs"):
    w = WORKLOADS[wl]
    return lbm.params(w["eos"], member["T_r"], n, n, kappa=w["kappa"], tau=w["tau"],
                      k=member["k"], mu_cap=w["mu_cap"])


def tanh_start(p, radius, wl="cs"):
    g, l = lbm.maxwell(p)
    return inputs.droplet(p.nx, p.ny, g, l, radius, WORKLOADS[wl]["width"])[0]


def _host(a):
    if a is None:
        return None
    return a.cpu().numpy() if hasattr(a, "cpu") else a


def converge(plist, rho0s, tol, every, max_steps, log=None, v0s=None):
    """Run every drop to max |rho(t) - rho(t - every)| < tol as one batch;
    returns (batch, steps, status, seconds).  rho0s: host or device arrays.
    Each drop starts with zero bare velocity (the start of Eq. 41) unless
    v0s[i] is a pair (vx, vy) of fluid velocities ((None, None): at rest)."""
    import torch
    b = lbm.Batch(plist, [_host(r) for r in rho0s])
    for i, v in enumerate(v0s or []):
        if v is not None:
            b.set_velocity(i, _host(v[0]), _host(v[1]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, part = 0, 50_000
    while done < max_steps:
        st, _, _, sts = b.run_until_converged(tol, every, min(part, max_steps - done))
        done += part
        active = sum(1 for x in sts if x == lbm.LBM_NOT_CONVERGED)
        if log:
            log("    %d steps, %d of %d active, %.1f s" % (min(done, max_steps), active,
                                                          len(plist), time.perf_counter() - t0))
        if active == 0:
            break
    secs = time.perf_counter() - t0
    return b, [b.steps_taken(i) for i in range(len(plist))], list(sts), secs


def geometry(n, radius, nodes):
    """(r - R, theta) of flat node indices `nodes` of an n x n mesh."""
    y, x = np.divmod(nodes, n)
    dx, dy = x - n / 2.0, y - n / 2.0
    return np.sqrt(dx * dx + dy * dy) - radius, np.arctan2(dy, dx)


def features(member, radius, d, theta, wl="cs"):
    """Normalised features (len(d), 7)."""
    f = np.empty((len(d), 7))
    f[:, 0] = member["T_r"]
    f[:, 1] = radius / R_REF
    f[:, 2] = WORKLOADS[wl]["kappa"]
    f[:, 3] = member["k"]
    f[:, 4] = d
    f[:, 5] = np.cos(4.0 * theta)
    f[:, 6] = np.sin(4.0 * theta)
    return ((f - FEATURE_CENTER) / FEATURE_SCALE).astype(np.float32)


def samples(member, p, radius, rho, ux, uy, stride=2, wl="cs"):
    """Training samples of a converged state (density and fluid velocity):
    the nodes with both coordinates multiples of `stride`; targets are the
    normalised log density and the radial and azimuthal velocity in units of
    U_SCALE."""
    n = p.nx
    g, l = lbm.maxwell(p)
    ys, xs = np.meshgrid(np.arange(0, n, stride), np.arange(0, n, stride), indexing="ij")
    nodes = (ys * n + xs).ravel()
    d, th = geometry(n, radius, nodes)
    r, u, v = rho.ravel()[nodes], ux.ravel()[nodes], uy.ravel()[nodes]
    c, s = np.cos(th), np.sin(th)
    t = np.empty((len(nodes), 3))
    t[:, 0] = (np.log(r) - np.log(g)) / (np.log(l) - np.log(g))
    t[:, 1] = (u * c + v * s) / U_SCALE
    t[:, 2] = (-u * s + v * c) / U_SCALE
    return features(member, radius, d, th, wl), t.astype(np.float32)


def training_set(seed, count, n, tol, every, max_steps, log=None, stride=2, wl="cs",
                 r_scale=1.0):
    """Converge `count` drops of workload `wl` at n x n from the tanh start
    and return (x, t, info).  r_scale scales the drawn radii (drops of the
    size a smaller mesh holds, on a mesh as large as the evaluation's)."""
    ms = members(seed, count, wl)
    plist = [drop_params(m, n, wl) for m in ms]
    radii = [r_scale * m["r_frac"] * n for m in ms]
    b, steps, sts, secs = converge(plist, [tanh_start(p, R, wl) for p, R in zip(plist, radii)],
                                   tol, every, max_steps, log)
    xs, ts = [], []
    for i, (m, p, R) in enumerate(zip(ms, plist, radii)):
        if sts[i] != lbm.LBM_OK:
            continue
        x, t = samples(m, p, R, *b.moments(i), stride=stride, wl=wl)
        xs.append(x)
        ts.append(t)
    b.close()
    return np.concatenate(xs), np.concatenate(ts), {
        "workload": wl, "drops": count, "n": n, "converged": sum(1 for s in sts if s == lbm.LBM_OK),
        "not_converged": [dict(T_r=round(m["T_r"], 4), k=round(m["k"], 4), radius=round(R, 1),
                               status=lbm.status_string(st), steps=s)
                          for m, R, st, s in zip(ms, radii, sts, steps) if st != lbm.LBM_OK],
        "steps_max": max(steps), "seconds": round(secs, 2)}


def train_network(x, t, *, seed=11, phases=((6000, 2e-3), (6000, 4e-4)), batch=4096,
                  density_weight=10.0):
    """Train a fresh network on (x, t) with Adam, one run of minibatches per
    (iterations, learning rate) phase.  The density output is trained scaled
    by density_weight (it needs more relative accuracy than the velocity) and
    the weight is folded back into the last layer afterwards, so the returned
    network predicts the quantities of include/lbm_warmstart.h.  Returns
    (MLP, losses of the last phase, seconds)."""
    import torch
    net = lbm.MLP(inputs.network_init(seed))
    tw = np.array(t, dtype=np.float32)
    tw[:, 0] *= density_weight
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    td = torch.from_numpy(tw).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (iters, lr) in enumerate(phases):
        order = torch.from_numpy(inputs.minibatch_order(seed + 1 + i, len(tw), batch, iters))
        losses = net.train(xd, td, order.cuda(), batch, lr=lr)
    secs = time.perf_counter() - t0
    w = net.get_params()
    off_w3 = 7 * 128 + 128 + 128 * 128 + 128  # W3 row 0, then b3[0] after W3
    w[off_w3:off_w3 + 128] /= density_weight
    w[off_w3 + 3 * 128] /= density_weight
    net.set_params(w)
    return net, losses, secs


def compare(net, seed, count, n, tol, every, max_steps, log=None, bf16=True, r_scale=1.0,
            modes=None, wl="cs", at_rest=True, reach=math.inf):
    """Unseen drops at n x n from the tanh start (Eq. 41, zero velocity) and
    from the warm start (same mass, predicted density and fluid velocity),
    run to the same criterion; the tanh start with the fluid at rest is run
    too, for reference.  A drop whose proposed density cannot be mass
    matched falls back to the tanh start.  Returns per-drop steps, wall
    times (the warm start's includes building its fields) and the largest
    differences between the converged states of the two starts (over the
    drops that converged from both; None if none did).  r_scale
    scales the drawn radii (to keep a larger mesh's drops within the radii the
    network was trained on).  modes: inference precisions to evaluate (bf16
    flags, default [bf16]); the tanh runs are shared, the top-level results
    are those of the first mode and "by_inference" holds every mode's.
    at_rest=False leaves out the tanh start with the fluid at rest.  reach:
    distance from the interface up to which the warm start uses the network
    (the Maxwell gas at rest beyond, lbm_mlp_set_reach; net keeps it)."""
    import torch
    modes = [bf16] if modes is None else list(modes)
    ms = members(seed, count, wl)
    plist = [drop_params(m, n, wl) for m in ms]
    radii = [r_scale * m["r_frac"] * n for m in ms]
    tanh0 = [tanh_start(p, R, wl) for p, R in zip(plist, radii)]
    bt, steps_t, sts_t, secs_t = converge(plist, tanh0, tol, every, max_steps, log)
    steps_r = None
    if at_rest:
        br, steps_r, _, _ = converge(plist, tanh0, tol, every, max_steps, log,
                                     [(None, None)] * count)
        br.close()
    by = {}
    net.set_reach(reach)
    for mode in modes:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho0, v0, fallback = [], [], 0
        for p, R, r in zip(plist, radii, tanh0):
            try:
                rho, vx, vy = net.warm_start_drop(p, R, float(r.sum()), bf16=mode)
                rho0.append(rho)
                v0.append((vx, vy))
            except lbm.LBMError:
                rho0.append(r)
                v0.append(None)
                fallback += 1
        torch.cuda.synchronize()
        secs_ws = time.perf_counter() - t0
        bw, steps_w, sts_w, secs_w = converge(plist, rho0, tol, every, max_steps, log, v0)
        drho, dv = [], []
        for i in range(len(plist)):
            if sts_t[i] != lbm.LBM_OK or sts_w[i] != lbm.LBM_OK:
                continue  # compared where both starts converged
            r1, vx1, vy1 = bt.moments(i)
            r2, vx2, vy2 = bw.moments(i)
            drho.append(float(np.abs(r1 - r2).max() / r1.max()))
            dv.append(float(max(np.abs(vx1 - vx2).max(), np.abs(vy1 - vy2).max())))
        mass = [float(abs(_host(w).sum() - r.sum()) / r.sum()) for w, r in zip(rho0, tanh0)]
        bw.close()
        by["bf16" if mode else "fp32"] = {
            "steps_warm": steps_w, "status_warm": sts_w, "fallbacks": fallback,
            "seconds_warm": round(secs_w + secs_ws, 3), "seconds_warm_fields": round(secs_ws, 4),
            "max_rel_drho": max(drho, default=None), "max_abs_dv": max(dv, default=None),
            "max_rel_mass_gap": max(mass),
        }
    bt.close()
    first = by["bf16" if modes[0] else "fp32"]
    out = {
        "workload": wl, "drops": count, "n": n, "tol": tol, "check_every": every,
        "inference": "bf16" if modes[0] else "fp32", "reach": reach,
        "steps_tanh": steps_t, "steps_tanh_at_rest": steps_r, "status_tanh": sts_t,
        "seconds_tanh": round(secs_t, 3),
    }
    out.update(first)
    out["by_inference"] = by
    return out
