"""Learned warm start of static drops (orchestration over the C ABI).

The solver converges drops from the tanh start of Eq. 41 (Sec. 5.3); the
converged profiles become training samples of the network of
include/lbm_warmstart.h, which the library trains with its own FP32 kernels;
the trained network then proposes the initial density of new drops (BF16
inference, mass matched to the tanh start), and both starts are run to the
same convergence criterion.  Every numerical step (solver, training,
inference, warm-start field) runs in the library's kernels; this module only
draws the workload, assembles the samples and keeps the books.

Workload: Carnahan-Starling drops (a = 1, b = 4, R = 1) in square periodic
meshes, kappa = 0.1, tau = 1, T/Tc, radius fraction and k drawn per drop.
"""
import time

import numpy as np

from . import inputs, lbm

KAPPA, TAU, WIDTH = 0.1, 1.0, 5.0
FEATURE_CENTER = np.array([0.5, 0.25, 0.1, 0.25, 0.0])
FEATURE_SCALE = np.array([0.25, 0.1, 0.1, 0.1, 8.0])
R_REF = 256.0
RANGES = dict(t_lo=0.35, t_hi=0.6, r_lo=0.15, r_hi=0.35, k_lo=0.15, k_hi=0.3)


def drop_params(member, n):
    return lbm.params(lbm.EOS_CS, member["T_r"], n, n, kappa=KAPPA, tau=TAU, k=member["k"])


def tanh_start(p, radius):
    g, l = lbm.maxwell(p)
    return inputs.droplet(p.nx, p.ny, g, l, radius, WIDTH)[0]


def converge(plist, rho0s, tol, every, max_steps, log=None):
    """Run every drop to max |rho(t) - rho(t - every)| < tol as one batch;
    returns (batch, steps, status, seconds).  rho0s: host or device arrays."""
    import torch
    host = [r.cpu().numpy() if hasattr(r, "cpu") else r for r in rho0s]
    b = lbm.Batch(plist, host)
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


def features(member, n, radius, r):
    """Normalised features (len(r), 5) of nodes at distance r from the centre."""
    f = np.empty((len(r), 5))
    f[:, 0] = member["T_r"]
    f[:, 1] = radius / R_REF
    f[:, 2] = KAPPA
    f[:, 3] = member["k"]
    f[:, 4] = r - radius
    return ((f - FEATURE_CENTER) / FEATURE_SCALE).astype(np.float32)


def samples(member, p, radius, rho):
    """Training samples of a converged drop: the row through the centre;
    target = normalised log density (ln rho - ln rho_g) / (ln rho_l - ln rho_g)."""
    n = p.nx
    g, l = lbm.maxwell(p)
    row = rho[p.ny // 2]
    r = np.abs(np.arange(n, dtype=np.float64) - n / 2.0)
    t = (np.log(row) - np.log(g)) / (np.log(l) - np.log(g))
    return features(member, n, radius, r), t.astype(np.float32)


def training_set(seed, count, n, tol, every, max_steps, log=None):
    """Converge `count` drops at n x n and return (x, t, info)."""
    members = inputs.warmstart_members(seed, count, **RANGES)
    plist = [drop_params(m, n) for m in members]
    radii = [m["r_frac"] * n for m in members]
    b, steps, sts, secs = converge(plist, [tanh_start(p, R) for p, R in zip(plist, radii)], tol,
                                   every, max_steps, log)
    xs, ts = [], []
    for i, (m, p, R) in enumerate(zip(members, plist, radii)):
        if sts[i] != lbm.LBM_OK:
            continue
        rho, _, _ = b.moments(i)
        x, t = samples(m, p, R, rho)
        xs.append(x)
        ts.append(t)
    b.close()
    return np.concatenate(xs), np.concatenate(ts), {
        "drops": count, "n": n, "converged": sum(1 for s in sts if s == lbm.LBM_OK),
        "steps_max": max(steps), "seconds": round(secs, 2)}


def train_network(x, t, *, seed=11, iters=3000, batch=2048, lr=2e-3):
    """Train a fresh network on (x, t) with Adam; returns (MLP, losses, s)."""
    import torch
    net = lbm.MLP(inputs.network_init(seed))
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    order = torch.from_numpy(inputs.minibatch_order(seed + 1, len(t), batch, iters)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = net.train(xd, td, order, batch, lr=lr)
    secs = time.perf_counter() - t0
    return net, losses, secs


def compare(net, seed, count, n, tol, every, max_steps, log=None):
    """Unseen drops at n x n from the tanh start and from the warm start (same
    mass), run to the same criterion.  Returns per-drop steps, wall times
    (warm start includes building its fields) and the largest differences
    between the two converged fields."""
    import torch
    members = inputs.warmstart_members(seed, count, **RANGES)
    plist = [drop_params(m, n) for m in members]
    radii = [m["r_frac"] * n for m in members]
    tanh0 = [tanh_start(p, R) for p, R in zip(plist, radii)]
    bt, steps_t, sts_t, secs_t = converge(plist, tanh0, tol, every, max_steps, log)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    warm0 = [net.warm_start_drop(p, R, float(r.sum())) for p, R, r in zip(plist, radii, tanh0)]
    torch.cuda.synchronize()
    secs_ws = time.perf_counter() - t0
    bw, steps_w, sts_w, secs_w = converge(plist, warm0, tol, every, max_steps, log)
    drho, dv = [], []
    for i, p in enumerate(plist):
        r1, vx1, vy1 = bt.moments(i)
        r2, vx2, vy2 = bw.moments(i)
        drho.append(float(np.abs(r1 - r2).max() / r1.max()))
        dv.append(float(max(np.abs(vx1 - vx2).max(), np.abs(vy1 - vy2).max())))
    mass = [float(abs(w.sum().item() - r.sum()) / r.sum()) for w, r in zip(warm0, tanh0)]
    bt.close()
    bw.close()
    return {
        "drops": count, "n": n, "tol": tol, "check_every": every,
        "steps_tanh": steps_t, "steps_warm": steps_w,
        "status_tanh": sts_t, "status_warm": sts_w,
        "seconds_tanh": round(secs_t, 3), "seconds_warm": round(secs_w + secs_ws, 3),
        "seconds_warm_fields": round(secs_ws, 4),
        "max_rel_drho": max(drho), "max_abs_dv": max(dv), "max_rel_mass_gap": max(mass),
    }
