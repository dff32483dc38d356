"""Benchmark of the solver's time step on one MI355X.

Workload: a static drop in a 1024 x 1024 periodic D2Q9 FP64 mesh, Peng-Robinson
EOS (a = 2/49, b = 2/21, R = 1, omega = 0.344) at T/T_c = 0.5, radius 200,
tanh initial interface of width 10 between the Maxwell densities
(Sec. 5.3, Eq. 41), tau = 0.8, upper limit of the chemical potential 6
(Sec. 5.6), k = 0.1, kappa = 0.004, sixth-order compact scheme.

One "step" is one lattice-Boltzmann time step of the whole mesh (the three
kernels of the solver).  Prints one JSON line with MLUPS (whole job) of this
workload, its kernels timed inside the step sequence (HIP events around every
launch), a report of the drop after the run (largest speed, bulk densities
against the Maxwell pair, pressure jump times radius), the roofline entry of
the dominant kernel on the 4096 x 2048 splash between walls (a working set of
~1.4 GB, far beyond the 256 MB last-level cache, so the bytes come from HBM),
and the CPU oracle timed on a bounded sample of the drop, on one core and on
all cores.  The "sweep" entry times a batched
sweep of simulations of uneven size to convergence against running each on
its own (the plain method); the "warm_start" entry trains the warm-start
network on solver-converged drops and compares steps and time to converge
from its proposal and from the tanh start.

    python bench.py [--gpus 1] [--steps 20000] [--warmup 200] [--sweep small|full|none]
                    [--warmstart small|full|cs-small|cs-full|none] [--splash hbm|full|none]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (D2Q9 FP64) + % peak HBM BW; sweep/warm-start time-to-converge vs plain"
HBM_PEAK_GBS = 8000.0
# Bytes per node of each kernel (FP64) as this design moves them:
#   row pass A: read the three density groups of the state (3 x 8), write rho
#     and the row part of mu (2 x 8)
#   column pass B: read rho and the row part of mu; write mu, F_y (strips
#     streamed down long columns add their windows: 168 rows above and
#     below, ~2.6 B per node at 2048 rows)
#   row pass C: read f (9 x 8), mu, F_y; write f (9 x 8) and its three
#     density groups (3 x 8); over row segments (long rows) it also reads
#     rho (8), and the window's 52 nodes past each end of an 896-node
#     segment add ~2 B of rho and mu reads
# and, for the roofline, the algorithmic count of the collide-and-stream
# kernel: read f and the two force or chemical-potential inputs, write f
# (72 + 24 + 72 = 168 B per lattice update); the floor of any scheme is f
# read and written once (144 B per update).
PASS_NAMES = ["rows_rho", "cols_mu", "rows_collide"]
PASS_BYTES = [40, 32, 184]
SEG_NAMES = ["rows_rho", "cols_mu", "collide_seg"]
SEG_BYTES = [40, 32, 192]
COLLIDE_ALG_BYTES = 168
FLOOR_BYTES = 144

NX = NY = 1024
CFG = dict(T_r=0.5, kappa=0.004, tau=0.8, k=0.1, mu_cap=6.0, radius=200.0, width=10.0)


KERNEL_SOURCES = ["kernels.hip", "kernels_iir.hip", "kernels.hpp", "physics.hpp", "lnx.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_splash4096x2048.json")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1906_09530_amd", "csrc", s), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return t["bytes_per_launch"].get(kernel)


# Batched sweep (Sec. 5.1 coexistence curve, Sec. 5.3 Laplace's law): square
# periodic CS meshes, half flat slabs, half static drops, T/Tc uniform in
# [0.35, 0.95], each run until max |rho(t) - rho(t - 100)| < 1e-12.
SWEEP = dict(seed=4, kappa=0.1, k=0.2, tau=1.0, width=5.0, tol=1e-12, check_every=100,
             max_steps=3_000_000)
SWEEP_SETS = {"small": dict(count=16, sizes=(64, 128, 256)),
              "full": dict(count=64, sizes=(64, 128, 256, 512))}


def sweep_cases(lbm, inputs, which):
    cfg = SWEEP_SETS[which]
    members = inputs.sweep_members(SWEEP["seed"], cfg["count"], sizes=cfg["sizes"])
    cases = []
    for m in members:
        n = m["n"]
        p = lbm.params(lbm.EOS_CS, m["T_r"], n, n, kappa=SWEEP["kappa"], tau=SWEEP["tau"],
                       k=SWEEP["k"])
        g, l = lbm.maxwell(p)
        if m["kind"] == "slab":
            rho0, _, _ = inputs.slab(n, n, g, l, SWEEP["width"])
        else:
            rho0, _, _ = inputs.droplet(n, n, g, l, m["radius"], SWEEP["width"])
        cases.append((m, p, rho0))
    return cases


def sweep_bench(lbm, inputs, which):
    """Time to converge every member: one batch (graph-replayed chunks,
    autotuned column shape) against one context per member run one after the
    other (the plain method).  Each plain run uses the batch's column-pass
    chunk, so both evolve bitwise alike and take the same steps."""
    import torch
    cases = sweep_cases(lbm, inputs, which)
    n = len(cases)
    tol, every, cap = SWEEP["tol"], SWEEP["check_every"], SWEEP["max_steps"]
    b = lbm.Batch([c[1] for c in cases], [c[2] for c in cases])
    tune = b.autotune(10)
    col_elems, chunk = min(tune, key=tune.get)
    print("sweep %s: %d members, batch column shape %s" % (which, n, (col_elems, chunk)),
          file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, part = 0, 100_000
    while done < cap:
        st, _, _, sts = b.run_until_converged(tol, every, min(part, cap - done), use_graph=True)
        done += part
        active = sum(1 for x in sts if x == lbm.LBM_NOT_CONVERGED)
        print("  batch: %d steps, %d active, %.1f s" % (done, active, time.perf_counter() - t0),
              file=sys.stderr, flush=True)
        if active == 0:
            break
    t_batch = time.perf_counter() - t0
    steps_b = [b.steps_taken(i) for i in range(n)]
    status_b = list(sts)
    b.close()

    t_seq, steps_s, status_s = 0.0, [], []
    for i, (m, p, rho0) in enumerate(cases):
        s = lbm.Solver(p, rho0)
        s.set_column_shape(col_elems // p.ny, chunk)
        s.synchronize()
        t0 = time.perf_counter()
        st, k, _ = s.run_until_converged(tol, every, cap)
        s.synchronize()
        t_seq += time.perf_counter() - t0
        steps_s.append(k)
        status_s.append(st)
        s.close()
        if i % 8 == 7 or i == n - 1:
            print("  plain: %d of %d done, %.1f s" % (i + 1, n, t_seq), file=sys.stderr,
                  flush=True)
    lups = sum(c[1].nx * c[1].ny * k for c, k in zip(cases, steps_b))
    return {
        "set": which, "members": n, "sizes": list(SWEEP_SETS[which]["sizes"]),
        "eos": "CS", "T_r_range": [0.35, 0.95], "kappa": SWEEP["kappa"], "k": SWEEP["k"],
        "tau": SWEEP["tau"], "tol": tol, "check_every": every,
        "batched_s": round(t_batch, 3), "plain_sequential_s": round(t_seq, 3),
        "speedup": round(t_seq / t_batch, 3),
        "all_converged": all(x == lbm.LBM_OK for x in status_b),
        "same_steps_as_plain": steps_b == steps_s and status_b == status_s,
        "steps_min_max": [min(steps_b), max(steps_b)],
        "lattice_updates": lups,
        "batched_MLUPS": round(lups / t_batch / 1e6, 1),
        "plain_MLUPS": round(lups / t_seq / 1e6, 1),
        "column_shape": [col_elems, chunk],
    }


# Learned warm start: Peng-Robinson drops ("pr": T/Tc 0.3-0.5, kappa = 0.003,
# k near 0.05) or Carnahan-Starling drops ("cs": T/Tc 0.35-0.6, kappa = 0.1),
# tau = 1; training drops converged by the solver, then unseen drops run from
# the tanh start and from the warm start to the same criterion.
# Training drops not converged within 1,000,000 steps are left out of the
# training set.  The full Peng-Robinson set (up to 850,000 steps per start on
# 512^2) runs BF16 inference only and leaves out the tanh start with the
# fluid at rest, to stay within minutes; its warm start uses the network
# within 80 nodes of the interface (the 256^2 training meshes reach about
# 125 nodes from their drops) and the Maxwell gas at rest beyond 90.  The
# "full512" set trains on 64 drops of the same radii on 512^2 meshes (the
# evaluation's size, whose gas far field the network then sees) and uses the
# network everywhere on the same 32 unseen drops.
WARM = {"small": dict(wl="pr", train=96, train_n=128, eval=8, eval_n=128),
        "full": dict(wl="pr", train=192, train_n=256, eval=32, eval_n=512, modes=(True,),
                     at_rest=False, reach=80.0),
        "full512": dict(wl="pr", train=64, train_n=512, train_r_scale=0.5, eval=32, eval_n=512,
                        eval_r_scale=0.5, modes=(True,), at_rest=False),
        "cs-small": dict(wl="cs", train=96, train_n=128, eval=8, eval_n=128),
        "cs-full": dict(wl="cs", train=192, train_n=256, eval=32, eval_n=512)}


def warmstart_bench(which):
    from paper_1906_09530_amd import lbm, warmstart
    cfg = WARM[which]
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    log("warm start %s: converging %d training drops at %d^2" % (which, cfg["train"],
                                                               cfg["train_n"]))
    x, t, info = warmstart.training_set(5, cfg["train"], cfg["train_n"], 1e-12, 100, 1_000_000,
                                        log=log, wl=cfg["wl"],
                                        r_scale=cfg.get("train_r_scale", 1.0))
    net, losses, secs = warmstart.train_network(x, t)
    log("  trained in %.1f s (final loss %.3e)" % (secs, float(losses[-20:].mean())))
    # radii of the unseen drops drawn from the training drops' range
    # BF16 inference (the network's deployed precision) and FP32 beside it
    res = warmstart.compare(net, 55, cfg["eval"], cfg["eval_n"], 1e-12, 100, 3_000_000, log=log,
                            modes=cfg.get("modes", (True, False)),
                            r_scale=cfg.get("eval_r_scale", cfg["train_n"] / cfg["eval_n"]),
                            wl=cfg["wl"],
                            at_rest=cfg.get("at_rest", True),
                            reach=cfg.get("reach", math.inf))
    net.close()
    ok = lbm.LBM_OK

    def totals(warm):
        """Steps of both starts summed over the drops that converged from
        both, and their count."""
        both = [i for i, (a, b) in enumerate(zip(res["status_tanh"], warm["status_warm"]))
                if a == ok and b == ok]
        st = sum(res["steps_tanh"][i] for i in both)
        sw = sum(warm["steps_warm"][i] for i in both)
        return st, sw, round(sw / st, 4) if st else None, len(both)

    st, sw, ratio, compared = totals(res)
    rr = warmstart.WORKLOADS[cfg["wl"]]["ranges"]
    other = {}
    for k, v in res["by_inference"].items():
        t_k, w_k, r_k, c_k = totals(v)
        other[k] = {"compared_drops": c_k, "steps_tanh": t_k, "steps_warm": w_k,
                    "steps_ratio": r_k, "seconds_warm": v["seconds_warm"],
                    "fallbacks": v["fallbacks"],
                    "all_converged": all(x == ok for x in v["status_warm"]),
                    "max_rel_drho_vs_tanh_solution": v["max_rel_drho"]}
    return {
        "set": which, "workload": cfg["wl"], "training": info, "samples": int(len(t)),
        "train_s": round(secs, 2),
        "eval_drops": cfg["eval"], "eval_n": cfg["eval_n"],
        "eval_radius_range": [round(rr[r] * cfg["train_n"] * cfg.get("train_r_scale", 1.0), 1)
                              for r in ("r_lo", "r_hi")],
        "tol": 1e-12, "check_every": 100,
        "inference": res["inference"],
        "reach": None if math.isinf(res["reach"]) else res["reach"],  # None: everywhere
        "compared_drops": compared, "steps_tanh": st, "steps_warm": sw, "steps_ratio": ratio,
        "steps_tanh_fluid_at_rest": (None if res["steps_tanh_at_rest"] is None
                                     else sum(res["steps_tanh_at_rest"])),
        "status_tanh": {lbm.status_string(s): res["status_tanh"].count(s)
                        for s in sorted(set(res["status_tanh"]))},
        "status_warm": {lbm.status_string(s): res["status_warm"].count(s)
                        for s in sorted(set(res["status_warm"]))},
        "seconds_tanh": res["seconds_tanh"], "seconds_warm": res["seconds_warm"],
        "all_converged": all(s == 0 for s in res["status_tanh"] + res["status_warm"]),
        "fallbacks": res["fallbacks"],
        "max_rel_drho_vs_tanh_solution": res["max_rel_drho"],
        "max_abs_dv_vs_tanh_solution": res["max_abs_dv"],
        "by_inference": other,
    }


def strict_json(obj):
    """obj with every non-finite float replaced by None (None in the output
    line stands for "not a number"), so the line is strict JSON."""
    if isinstance(obj, float):
        return obj if math.isfinite(obj) else None
    if isinstance(obj, dict):
        return {k: strict_json(v) for k, v in obj.items()}
    if isinstance(obj, (list, tuple)):
        return [strict_json(v) for v in obj]
    return obj


def copy_bandwidth(torch, nbytes, reps=20):
    """Read + write GB/s of the runtime's own device-to-device copy of
    nbytes / 2 (so that it moves nbytes per dispatch): the rate a plain
    streaming kernel reaches on this device.  A copy whose buffers fit in the
    last-level cache (256 MB) is partly served from it when repeated; one of
    1 GiB is not."""
    n = nbytes // 16
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 2 * n * 8 / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9


SPLASH = dict(nx=4096, ny=2048, T_r=0.6, kappa=0.1, k=0.2, tau=0.6, mu_cap=6.0, radius=100.0,
              width=5.0, film=40, drop_uy=-0.05, frame_ux=0.05, steps=10000)


def splash_bench(torch, lbm, inputs):
    """Drop falling on a liquid film between walls, 4096 x 2048 (CS), in the
    rest frame and in a frame moving at +0.05 with the walls sliding along:
    MLUPS of each (autotuned, chunks of 1000 steps with the moments read after
    each), mass at start and end, and the Galilean check (the moving-frame
    density shifted back by frame_ux x steps nodes against the rest frame)."""
    import numpy as np
    c = SPLASH
    nx, ny = c["nx"], c["ny"]
    res, runs = {}, []
    for frame in (0.0, c["frame_ux"]):
        p = lbm.params(lbm.EOS_CS, c["T_r"], nx, ny, kappa=c["kappa"], tau=c["tau"], k=c["k"],
                       mu_cap=c["mu_cap"], bc_y=1, wall_ux=frame)
        g, l = lbm.maxwell(p)
        rho0, ux0, uy0 = inputs.splash(nx, ny, g, l, c["radius"], c["width"], film=c["film"],
                                       drop_uy=c["drop_uy"], frame_ux=frame)
        d = [torch.from_numpy(a).cuda() for a in (rho0, ux0, uy0)]
        s = lbm.Solver(p, *d)
        s.autotune(5)
        mass0 = float(rho0.sum())
        done, t_step = 0, 0.0
        finite = True
        while done < c["steps"]:
            n = min(1000, c["steps"] - done)
            t0 = time.perf_counter()
            s.step(n)
            s.synchronize()
            t_step += time.perf_counter() - t0
            done += n
            r = s.moments()[0]
            finite = bool(np.isfinite(r).all())
            print("splash frame %.2f: %d steps, finite %s" % (frame, done, finite),
                  file=sys.stderr, flush=True)
            if not finite:
                break
        s.close()
        res[frame] = r
        runs.append({"frame_ux": frame, "steps": done, "finite": finite, "mass_start": mass0,
                     "mass_end": float(r.sum()), "seconds": round(t_step, 3),
                     "MLUPS": round(nx * ny * done / t_step / 1e6, 1)})
    out = dict(c, workload="drop splashing on a film between walls, CS", runs=runs)
    if all(r["finite"] for r in runs):
        shift = int(round(c["frame_ux"] * c["steps"]))
        moved = np.roll(res[c["frame_ux"]], -shift, axis=1)
        half = 0.5 * (g + l)
        out["galilean"] = {
            "shift_nodes": shift,
            "max_abs_drho": float(np.abs(moved - res[0.0]).max()),
            "nodes_across_mid_density_contour": int(((res[0.0] > half) != (moved > half)).sum()),
            "nodes": nx * ny}
    return out


def splash_hbm(torch, lbm, inputs, steps=300, kernel_steps=200):
    """The 4096 x 2048 splash between walls at rest (Sec. 5.5), autotuned: a
    whole-step rate over `steps` steps (events on the solver's stream) and each
    kernel timed inside the step sequence over `kernel_steps` steps.  Its
    working set (two f buffers, two density-group buffers and the planes,
    ~1.4 GB) is far beyond the last-level cache, so it is the HBM point."""
    import numpy as np
    c = SPLASH
    nx, ny = c["nx"], c["ny"]
    p = lbm.params(lbm.EOS_CS, c["T_r"], nx, ny, kappa=c["kappa"], tau=c["tau"], k=c["k"],
                   mu_cap=c["mu_cap"], bc_y=1)
    g, l = lbm.maxwell(p)
    rho0, ux0, uy0 = inputs.splash(nx, ny, g, l, c["radius"], c["width"], film=c["film"],
                                   drop_uy=c["drop_uy"])
    stream = torch.cuda.current_stream()
    d = [torch.from_numpy(a).cuda() for a in (rho0, ux0, uy0)]
    s = lbm.Solver(p, *d, stream=stream.cuda_stream)
    s.step(20)
    tune = s.autotune(5)
    # the collision variant the autotuner kept (2: over row segments)
    variant = min((k for k in tune if k[0] == 0), key=tune.get)[1]
    s.step(20)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    s.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / steps
    ms = s.time_step_kernels(kernel_steps)
    r = s.moments()[0]
    finite = bool(np.isfinite(r).all())
    s.close()
    names = SEG_NAMES if variant == 2 else PASS_NAMES
    nbytes = SEG_BYTES if variant == 2 else PASS_BYTES
    N = nx * ny
    dom = int(np.argmax(ms))
    return {"workload": "drop splashing on a 40-node film between walls, CS, 4096x2048, "
                        "T/Tc=0.6, R=100, tau=0.6, k=0.2, kappa=0.1",
            "nx": nx, "ny": ny, "finite": finite, "steps": steps, "collision_variant": variant,
            "column_shape": column_shape(tune),
            "ms_per_step": round(ms_step, 6), "MLUPS": round(N / (ms_step * 1e-3) / 1e6, 1),
            "floor_equivalent_GB_s": round(FLOOR_BYTES * N / (ms_step * 1e-3) / 1e9, 1),
            "kernels": {names[i]: {"avg_ms": round(ms[i], 6),
                                   "design_bytes_per_node": nbytes[i],
                                   "design_GB_s": round(nbytes[i] * N / (ms[i] * 1e-3) / 1e9, 1)}
                        for i in range(len(ms))},
            "dominant": names[dom], "dominant_ms": ms[dom]}


def column_shape(tune):
    """The column-pass shape the autotuner kept, as [width, chunk] (chunk
    LBM_COLUMN_STREAM = 1: strips streamed down the columns; negative: tiles
    with windows; 0: the reduction kernel)."""
    return list(min((k for k in tune if k[0] > 0), key=tune.get))


def small_mesh_bench(torch, lbm, inputs, steps=2000):
    """The 64 x 64 periodic CS drop (T/Tc = 0.7, kappa = 0, k = 1, fourth-order
    compact scheme, tau = 1, R = 16, tanh width 4, 1e-6 noise) for its 2000
    steps, its kernels launched one by one and replayed from captured HIP
    graphs of 100 steps (same results bit for bit): on a mesh this small the
    three kernels of a step take a few microseconds each and launch overhead
    sets the rate."""
    p = lbm.params(lbm.EOS_CS, 0.7, 64, 64, kappa=0.0, tau=1.0, k=1.0, cfd_alpha=0.25)
    rho_g, rho_l = lbm.maxwell(p)
    rho0, ux0, uy0 = inputs.droplet(64, 64, rho_g, rho_l, 16.0, 4.0, seed=1, noise=1e-6)
    out = {"workload": "64x64 periodic CS drop, T/Tc=0.7, kappa=0, k=1, 4th-order CFM, tau=1, "
                       "R=16, W=4", "steps": steps}
    states = []
    for name, G in (("eager", 0), ("graph100", 100)):
        sv = lbm.Solver(p, rho0, ux0, uy0)
        sv.set_graph_steps(G)
        sv.step(200)
        sv.synchronize()
        best = math.inf
        for _ in range(3):
            t0 = time.perf_counter()
            sv.step(steps)
            sv.synchronize()
            best = min(best, time.perf_counter() - t0)
        states.append(sv.get_state())
        sv.close()
        us = best / steps * 1e6
        out[name] = {"us_per_step": round(us, 3), "MLUPS": round(64 * 64 / us, 1)}
    out["graph_equals_eager_bitwise"] = bool((states[0] == states[1]).all())
    return out


def large_mesh_bench(torch, lbm, inputs, steps=200):
    """A 16384 x 8192 splash between walls (134 M nodes, ~36 GB of device
    state): rows of 16384 nodes run every row pass over windowed segments,
    columns of 8192 the factorised solve with 8-node chunks.  Whole-step rate
    over `steps` steps after autotuning."""
    nx, ny = 16384, 8192
    c = SPLASH
    p = lbm.params(lbm.EOS_CS, c["T_r"], nx, ny, kappa=c["kappa"], tau=c["tau"], k=c["k"],
                   mu_cap=c["mu_cap"], bc_y=1)
    g, l = lbm.maxwell(p)
    rho0, ux0, uy0 = inputs.splash(nx, ny, g, l, 4 * c["radius"], c["width"],
                                   film=4 * c["film"], drop_uy=c["drop_uy"])
    stream = torch.cuda.current_stream()
    d = [torch.from_numpy(a).cuda() for a in (rho0, ux0, uy0)]
    del rho0, ux0, uy0
    s = lbm.Solver(p, *d, stream=stream.cuda_stream)
    del d
    s.step(10)
    tune = s.autotune(2)
    s.step(10)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    s.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    kms = s.time_step_kernels(20)
    finite = bool(torch.isfinite(torch.as_tensor(s.moments(device=True)[0])).all())
    ws = lbm.workspace_bytes(p)
    s.close()
    return {"workload": "drop splashing on a 160-node film between walls, CS, 16384x8192, "
                        "T/Tc=0.6, R=400, tau=0.6, k=0.2, kappa=0.1",
            "nx": nx, "ny": ny, "steps": steps, "finite": finite,
            "device_bytes": ws, "ms_per_step": round(ms, 4),
            "MLUPS": round(nx * ny / (ms * 1e-3) / 1e6, 1),
            "column_shape": column_shape(tune),
            "kernels_ms": {n: round(t, 4) for n, t in zip(SEG_NAMES, kms)}}


def workload_params(lbm):
    return lbm.params(lbm.EOS_PR, CFG["T_r"], NX, NY, kappa=CFG["kappa"], tau=CFG["tau"],
                      k=CFG["k"], mu_cap=CFG["mu_cap"])


def cpu_baseline(budget_s=12.0, all_cores=True):
    """The oracle on the host on the first steps of the same workload until
    about `budget_s` of work: single-threaded, then (all_cores) its OpenMP
    build (bitwise the same results) on every core this process may use.
    Its inputs are built from the oracle's own coexistence densities."""
    import oracle
    from oracle import analytic as A
    from paper_1906_09530_amd import inputs
    op = A.params(A.EOS_PR, CFG["T_r"], NX, NY, kappa=CFG["kappa"], tau=CFG["tau"], k=CFG["k"],
                  mu_cap=CFG["mu_cap"])
    g, l = (float(v) for v in A.EOS(A.EOS_PR).maxwell(CFG["T_r"]))
    rho0, ux0, uy0 = inputs.droplet(NX, NY, g, l, CFG["radius"], CFG["width"])

    def timed(threads):
        used = oracle.threads(threads)
        f = oracle.init(op, rho0, ux0, uy0)
        steps, t0 = 0, time.perf_counter()
        while True:
            oracle.step(op, f)
            steps += 1
            el = time.perf_counter() - t0
            if el >= budget_s:
                break
        return NX * NY * steps / el / 1e6, steps, el, used

    try:
        one, s1, e1, _ = timed(1)
        if not all_cores:
            return {"value": one, "unit": "MLUPS", "cores": 1, "kind": "oracle",
                    "sample": "first %d steps of the same 1024x1024 PR drop, single-threaded C "
                              "oracle (%.1f s)" % (s1, e1)}
        # every core this process may use, within the thread count the
        # environment allows (OMP_NUM_THREADS)
        cores = len(os.sched_getaffinity(0))
        env = os.environ.get("OMP_NUM_THREADS", "")
        if env.isdigit() and int(env) > 0:
            cores = min(cores, int(env))
        many, s2, e2, used = timed(cores)
    finally:
        oracle.threads(1)
    return {"value": many, "unit": "MLUPS", "cores": used, "kind": "oracle",
            "single_core_value": one,
            "sample": "first %d steps of the same 1024x1024 PR drop, C oracle on %d threads "
                      "(OpenMP over lines and nodes, %.1f s); single-threaded: %d steps in %.1f s"
                      % (s2, used, e2, s1, e1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--pass-steps", type=int, default=1000,
                    help="steps timed per kernel with HIP events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--warmstart", choices=sorted(WARM) + ["none"], default="small",
                    help="learned warm start vs tanh start (steps and time to converge): 96 "
                         "training drops at 128^2, 8 unseen at 128^2 (small); 192 at 256^2, 32 "
                         "unseen at 512^2 (full, minutes); Peng-Robinson drops, or "
                         "Carnahan-Starling drops with the cs- prefix; or none")
    ap.add_argument("--sweep", choices=["small", "full", "none"], default="small",
                    help="batched sweep vs one run per member (time to converge): 16 members "
                         "up to 256^2 (small), 64 members up to 512^2 (full, minutes), or none")
    ap.add_argument("--splash", choices=["hbm", "full", "none"], default="hbm",
                    help="the 4096 x 2048 splash between walls: its whole-step rate and "
                         "in-sequence kernel times, the roofline point (hbm, default); also "
                         "the 10,000-step run in two frames (full, about 20 s more); or none")
    ap.add_argument("--large", choices=["16384x8192", "none"], default="16384x8192",
                    help="a 16384 x 8192 splash between walls, 200 steps (rows over windowed "
                         "segments; ~36 GB of device state), or none")
    ap.add_argument("--small", choices=["64", "none"], default="64",
                    help="the 64 x 64 drop of 2000 steps, launched kernel by kernel and from "
                         "captured graphs (64, default), or none")
    ap.add_argument("--kernel-steps", type=int, default=200,
                    help="steps over which each kernel is timed inside the sequence")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (a kernel of known "
                         "traffic, to calibrate FETCH_SIZE/WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.copy_calib:
        import torch
        n = args.copy_calib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(10):
            b.copy_(a)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / 10
        print(json.dumps({"copy_calib_bytes_per_dispatch": n * 8,
                          "copy_GB_s_read_plus_write": round(2 * n * 8 / (ms * 1e-3) / 1e9, 1)}),
              flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver is a single-GPU build "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1906_09530_amd import inputs, lbm

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    p = workload_params(lbm)
    rho_g, rho_l = lbm.maxwell(p)
    rho0, ux0, uy0 = inputs.droplet(NX, NY, rho_g, rho_l, CFG["radius"], CFG["width"])
    d = [torch.from_numpy(a).cuda() for a in (rho0, ux0, uy0)]
    s = lbm.Solver(p, *d, stream=stream.cuda_stream)

    print("warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
    s.step(args.warmup)
    torch.cuda.synchronize()
    tune = s.autotune(20)
    print("column-strip widths (ms): %s" % tune, file=sys.stderr, flush=True)

    print("timed %d steps" % args.steps, file=sys.stderr, flush=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    done = 0
    chunk = 2000
    while done < args.steps:
        n = min(chunk, args.steps - done)
        s.step(n)
        done += n
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps
    mlups = NX * NY / (ms_per_step * 1e-3) / 1e6

    # the drop after warmup + timed steps, before the kernel timing steps
    report = drop_report(lbm, s, p, rho_g, rho_l)
    print("per-kernel timing inside the step sequence over %d steps" % args.kernel_steps,
          file=sys.stderr, flush=True)
    kms = s.time_step_kernels(args.kernel_steps)
    s.close()
    N = NX * NY

    splash = None
    if args.splash != "none":
        print("4096 x 2048 splash: HBM point", file=sys.stderr, flush=True)
        splash = splash_hbm(torch, lbm, inputs, kernel_steps=args.kernel_steps)
        if args.splash == "full":
            splash["two_frames_10000_steps"] = splash_bench(torch, lbm, inputs)
    large = None
    if args.large != "none":
        print("16384 x 8192 splash", file=sys.stderr, flush=True)
        large = large_mesh_bench(torch, lbm, inputs)
    small = None
    if args.small != "none":
        print("64 x 64 drop: launches one by one and from graphs", file=sys.stderr, flush=True)
        small = small_mesh_bench(torch, lbm, inputs)
    copy_big_gbs = copy_bandwidth(torch, 2 << 30, reps=5)
    sweep = None if args.sweep == "none" else sweep_bench(lbm, inputs, args.sweep)
    warm = None if args.warmstart == "none" else warmstart_bench(args.warmstart)
    cpu = None if args.no_cpu_baseline else cpu_baseline()

    roofline = None
    if splash is not None:
        nodes = splash["nx"] * splash["ny"]
        dms = splash["dominant_ms"]
        ach = COLLIDE_ALG_BYTES * nodes / (dms * 1e-3) / 1e9
        roofline = {
            "kernel": splash["dominant"],
            "workload": "4096x2048 CS splash between walls (out of cache)",
            "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(splash["dominant"]),
            "traffic_unit": "bytes/launch",
            "algorithmic_bytes_per_node": COLLIDE_ALG_BYTES,
            "design_bytes_per_node": splash["kernels"][splash["dominant"]]["design_bytes_per_node"],
            "avg_ms": round(dms, 6),
            "timing": "HIP events around every launch inside the step sequence",
            "step_floor_frac": round(splash["floor_equivalent_GB_s"] / HBM_PEAK_GBS, 4),
            "device_copy_1GiB_GB_s": round(copy_big_gbs, 1),
        }
        del splash["dominant_ms"]
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "static PR drop, 1024x1024 periodic D2Q9, T/Tc=0.5, R=200, W=10, "
                        "tau=0.8, mu limit 6, k=0.1, kappa=0.004, 6th-order compact FD",
            "nx": NX, "ny": NY, "eos": "PR", "omega": 0.344, "T_r": CFG["T_r"],
            "k": CFG["k"], "kappa": CFG["kappa"], "tau": CFG["tau"], "mu_cap": CFG["mu_cap"],
            "radius": CFG["radius"], "width": CFG["width"],
        },
        "roofline": roofline,
        # 1024^2 drop: its ~240 MB working set sits largely in the 256 MB
        # last-level cache
        "kernels": {PASS_NAMES[i]: {"avg_ms": round(kms[i], 6),
                                    "design_bytes_per_node": PASS_BYTES[i],
                                    "design_GB_s": round(PASS_BYTES[i] * N / (kms[i] * 1e-3) / 1e9,
                                                         1)} for i in range(3)},
        "kernels_note": "1024x1024 drop, timed inside the step sequence; cache-resident working set",
        "collide_algorithmic_GB_s": round(COLLIDE_ALG_BYTES * N / (kms[2] * 1e-3) / 1e9, 1),
        # MLUPS x 144 B (f read and written once: the floor of any scheme)
        "floor_equivalent_GB_s": round(FLOOR_BYTES * N / (ms_per_step * 1e-3) / 1e9, 1),
        "autotune_col_width_ms": {str(k): round(v, 6) for k, v in tune.items()},
        "wall_s": round(wall, 3),
        "drop_after_run": report,
        "splash_hbm": splash,
        "small_mesh_64": small,
        "large_mesh": large,
        "sweep": sweep,
        "warm_start": warm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(strict_json(out), allow_nan=False), flush=True)


def drop_report(lbm, s, p, rho_g, rho_l):
    """The static drop after the run: steps, largest speed |v| (the spurious
    current once the drop has settled; Sec. 5.4), bulk densities inside and
    outside against the Maxwell pair, the equimolar radius and the pressure
    jump k^2 [p0(inside) - p0(outside)] times that radius (the surface
    tension, were the drop at rest; Eq. 40)."""
    import numpy as np
    r, vx, vy = s.moments()
    inside, outside = float(r[NY // 2, NX // 2]), float(r[0, 0])
    radius = float(np.sqrt(((r - outside) / (inside - outside)).sum() / np.pi))
    p_in = lbm.eos_values(p, inside)[0]
    p_out = lbm.eos_values(p, outside)[0]
    dp = p.k * p.k * (p_in - p_out)
    return {"steps": s.steps_taken, "finite": bool(np.isfinite(r).all()),
            "max_speed": float(np.hypot(vx, vy).max()),
            "rho_inside": inside, "rho_outside": outside,
            "rho_l_maxwell": rho_l, "rho_g_maxwell": rho_g,
            "rel_inside_vs_maxwell": inside / rho_l - 1, "rel_outside_vs_maxwell": outside / rho_g - 1,
            "equimolar_radius": radius, "pressure_jump": dp, "pressure_jump_x_radius": dp * radius}


if __name__ == "__main__":
    main()
