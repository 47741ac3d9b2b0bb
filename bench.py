#!/usr/bin/env python3
"""Benchmark: four-step nonequilibrium G(t,t') on the 2x7 Hubbard ladder.

Workload: half-filled open 2x7 Hubbard ladder (t=1, D = 3432 x 3432 =
11,778,624), sudden quench U: 4 -> 8; (i) ground state of H_ini by Lanczos,
(ii) forward SIL propagation to t_max = 5 (100 steps of dt = 0.05, Krylov
dim 20), (iii) backward propagation of c Phi(t_k) and c+ Phi(t_k) for every
mesh time, (iv) G^<_00(t,t') and G^>_00(t,t') on the 101 x 101 mesh.
Inputs are synthetic and seeded (start vector seed 7); everything is
resident in HBM when the timed region starts.

One timed "step" is one mesh interval of the backward sweep (steps (iii)
and (iv)) at the production block width: the block of columns
e^{iH(t_j - t_s)} c Phi(t_j) (as many as the free device memory holds) is
dotted with c Phi(t_s) (step (iv)) and moved from t_s to t_{s-1} by one
SIL step (Krylov dim 20, batched over the columns).  The ground state, the
forward mesh and the sweep's growth phase (block narrower than the
production width) run before the timed region and are timed separately;
after it the run is finished, so the line also reports the whole four-step
run (all 10,200 vector-steps) and checks the equal-time anticommutator of
the full G.

value = contour steps/s: single-column SIL steps (each Krylov dim H.v
products) completed per second in the timed intervals.
roofline: the Lanczos-form H.v class with the most time (at the production
width the strip pass of the fused two-pass step, whose algorithmic bytes
per launch are 16 B x D x columns x (3 or 4 vectors: x_k, z, x_(k-1) in,
y out); the single pass, 2 or 3 vectors, where one-column launches
dominate), divided by its launch durations measured with HIP events on the
library's stream; `traffic` scales those bytes by the committed counter
summary of that class when it matches the kernel source.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# committed rocprofv3 counter summaries of the L=14 H.v kernels, per profiled class
TRAFFIC_FILES = {
    "hv_lanczos": os.path.join(ROOT, "profiles", "hv_lanczos_ladder14_traffic.md"),
    "hv_rows_lanczos": os.path.join(ROOT, "profiles", "hv_fused_ladder14_traffic.md"),
    "hv_up_lanczos": os.path.join(ROOT, "profiles", "hv_fused_ladder14_traffic.md"),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--whole", action="store_true",
                   help="time whole four-step runs per step (kgf_greens_neq; both schedules) instead of "
                        "sweep intervals")
    p.add_argument("--no-finish", action="store_true",
                   help="stop after the timed intervals instead of finishing the four-step run")
    p.add_argument("--schedule", choices=["sweep", "plain"], default="sweep")
    p.add_argument("--batch", type=int, default=0, help="sweep block width cap (0 = from free memory)")
    p.add_argument("--reorth", type=int, default=0)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--profile-every", type=int, default=1)
    p.add_argument("--probe", action="store_true",
                   help="short run for hardware counters: one SIL step of a batch of backward-sweep "
                        "columns of the same workload, then a plain copy of one vector (calibration)")
    p.add_argument("--probe-cols", type=int, default=8)
    p.add_argument("--probe-L", type=int, choices=[14, 16], default=14,
                   help="probe: ladder size (16: the two-pass H.v of the 2x8 ladder)")
    p.add_argument("--workload", choices=["ladder14", "batch64", "ladder16", "fig1", "hub4x3", "driven", "driven4", "necpt",
                                           "two_particle", "graphs"],
                   default="ladder14",
                   help="ladder14: the four-step benchmark (default); batch64: the 64-instance uneven Anderson "
                        "batch, batched vs per instance, plus adjoint timings; ladder16: the 2x8 ladder on a "
                        "short mesh; driven: the 2x7 ladder under a periodic rung drive (commutator-free "
                        "integrator) against as many static SIL steps; hub4x3: equilibrium G of the 4x3 cluster, 24 columns batched vs one at a "
                        "time; fig1: the equilibrium spectral density of the L=10 ring (Sec. 3) for "
                        "several restart counts against the conventional Lanczos G")
    p.add_argument("--grad-instances", type=int, default=5,
                   help="batch64: instances (one per L first) whose per-instance adjoint gradient is timed")
    p.add_argument("--no-batched-adjoint", action="store_true",
                   help="batch64: skip the batched adjoint of all 64 instances")
    p.add_argument("--skip-per-instance", action="store_true",
                   help="batch64: skip the per-instance forward timing")
    p.add_argument("--nt16", type=int, default=6, help="ladder16: mesh points")
    p.add_argument("--spg16", type=int, default=1, help="ladder16: SIL steps of dt = 0.05 per mesh interval")
    p.add_argument("--adj16", type=int, default=0,
                   help="ladder16: also the adjoint gradient (all hoppings, U, fields) of a loss of G_00 on a mesh "
                        "of this many points (0: none), chains checkpointed every 10 SIL steps")
    p.add_argument("--plain-baseline", action="store_true",
                   help="batch64: also time the plain single-vector method (schedule 0) instance by instance")
    p.add_argument("--hv", default="",
                   help="H.v micro-benchmark instead of the four-step run: comma-separated ladder sizes "
                        "(14, 16); each is timed for every --hv-passes variant")
    p.add_argument("--hv-passes", default="0",
                   help="comma-separated kgf_set_option HV_PASSES values (9: the library's tuner chooses)")
    p.add_argument("--hv-strip", default="0", help="comma-separated kgf_set_option HV_STRIP values")
    p.add_argument("--hv-fuse", default="1",
                   help="comma-separated kgf_set_option HV_FUSE values (two-pass Lanczos step with the update "
                        "folded into the row pass)")
    p.add_argument("--hv-seg", default="1",
                   help="comma-separated kgf_set_option HV_SEG values (row pass with the segment hop tables)")
    p.add_argument("--hv-up-threads", default="1024",
                   help="comma-separated kgf_set_option HV_UP_THREADS values (pass-2 block size)")
    p.add_argument("--hv-reps", type=int, default=10)
    p.add_argument("--hv-cols", default="1",
                   help="comma-separated column counts of the timed SIL step (the Lanczos form); the plain "
                        "H.v is timed once per variant on one column")
    p.add_argument("--no-graphs", action="store_true",
                   help="state GRAPHS 0 explicitly (every SIL step eager, the library default); kernel traces "
                        "are taken this way")
    p.add_argument("--hv-plan", type=int, default=0,
                   help="ladder14 run and --probe: kgf_set_option HV_PASSES for every H.v of the run (0: the "
                        "library's choice by size and column count, 1: single pass, 2: two pass)")
    p.add_argument("--tune", action="store_true",
                   help="let the library time the equivalent H.v variants per sector "
                        "(kgf_set_option HV_TUNE) and keep the fastest")
    return p.parse_args()


def hv_bench(a):
    """Time H.v (y = H x) and the Lanczos-fused H.v (one SIL step, Krylov
    dim 20) on the half-filled 2xL/2 ladder's c-sector (N_up - 1, N_dn), for
    each requested kernel variant.  One JSON line per (L, variant)."""
    import torch
    import paper_1109_1205_amd as kgf
    import workloads as wl
    ctx = kgf.Context(0)
    for L in [int(v) for v in a.hv.split(",") if v]:
        q = wl.ladder14() if L == 14 else wl.ladder16()
        m = ctx.model(q.H)
        sec = ctx.sector(L, q.n_up - 1, q.n_dn)
        g = torch.Generator(device="cuda:0").manual_seed(11)
        x = torch.randn(sec.dim, dtype=torch.complex128, device="cuda:0", generator=g)
        y = torch.empty_like(x)
        variants = [(int(p_), int(s_), int(f_), int(g_), int(q_)) for p_ in a.hv_passes.split(",") if p_
                    for s_ in a.hv_strip.split(",") if s_ for f_ in a.hv_fuse.split(",") if f_
                    for g_ in a.hv_seg.split(",") if g_ for q_ in a.hv_up_threads.split(",") if q_]
        for passes, strip, fuse, seg, uthr in variants:
            # passes 9: let the library's tuner choose (HV_TUNE)
            ctx.set_option(ctx.HV_TUNE, 1 if passes == 9 else 0)
            ctx.set_option(ctx.HV_PASSES, 0 if passes == 9 else passes)
            ctx.set_option(ctx.HV_STRIP, 0 if passes == 9 else strip)
            ctx.set_option(ctx.HV_FUSE, fuse)
            ctx.set_option(ctx.HV_SEG, seg)
            ctx.set_option(ctx.HV_UP_THREADS, uthr)
            ctx.apply_h(m, sec, x, y)      # warm-up (tables, LDS opt-in)
            torch.cuda.synchronize()
            log(f"L={L} D={sec.dim} passes={passes} strip={strip} fuse={fuse} seg={seg} up_threads={uthr}: timing")
            for ci, ncols in enumerate(int(v) for v in a.hv_cols.split(",") if v):
                xs = x.clone().reshape(1, -1).repeat(ncols, 1)
                ctx.propagate(m, sec, xs, 1, q.dt, q.krylov_dim, +1)    # warm-up at this width (tuner, workspaces)
                torch.cuda.synchronize()
                ctx.profile_begin(1)
                if ci == 0:
                    for _ in range(a.hv_reps):
                        ctx.apply_h(m, sec, x, y)
                ctx.propagate(m, sec, xs, 1, q.dt, q.krylov_dim, +1)
                torch.cuda.synchronize()
                st = ctx.profile_end()
                out = {"hv_bench": L, "D": sec.dim, "passes": passes, "strip": strip, "fuse": fuse, "seg": seg,
                       "up_threads": uthr, "cols": ncols}
                step_ms = 0.0
                for k in ("hv", "hv_lanczos", "hv_rows_lanczos", "hv_up_lanczos", "lanczos_update", "combine"):
                    if k in st and st[k]["sampled"]:
                        ms = st[k]["sampled_ms"] / st[k]["sampled"]
                        gbs = st[k]["sampled_bytes"] / (st[k]["sampled_ms"] * 1e-3) / 1e9
                        out[k] = {"avg_ms": round(ms, 4), "GBps": round(gbs, 1),
                                  "frac": round(gbs / HBM_PEAK_GBPS, 4)}
                        if k != "hv":
                            step_ms += st[k]["sampled_ms"]
                out["sil_step_ms_per_column"] = round(step_ms / ncols, 4)
                print(json.dumps(out), flush=True)
                del xs
                torch.cuda.empty_cache()
        ctx.set_option(ctx.HV_PASSES, 0)
        ctx.set_option(ctx.HV_STRIP, 0)
        ctx.set_option(ctx.HV_TUNE, 0)
        ctx.set_option(ctx.HV_FUSE, 1)
        ctx.set_option(ctx.HV_SEG, 1)
        ctx.set_option(ctx.HV_UP_THREADS, 1024)
        del x, y
        torch.cuda.empty_cache()


def probe(a):
    """Launch the dominant kernel in its bench configuration a few times
    (one SIL step, Krylov dim 20, on --probe-cols c-sector columns of the
    2x7 ladder, or of the 2x8 ladder with --probe-L 16), then one plain
    vector copy y = 2x whose FETCH_SIZE/WRITE_SIZE calibrate the counters
    (16 B x D read, 16 B x D written)."""
    import torch
    import paper_1109_1205_amd as kgf
    import workloads as wl
    q = wl.ladder14() if a.probe_L == 14 else wl.ladder16()
    ctx = kgf.Context(0)
    if a.hv_plan:
        ctx.set_option(ctx.HV_PASSES, a.hv_plan)
    m = ctx.model(q.H)
    sec = ctx.sector(a.probe_L, q.n_up - 1, q.n_dn)
    log(f"probe: L={a.probe_L} D={sec.dim} cols={a.probe_cols} hv_plan={a.hv_plan}")
    g = torch.Generator(device="cuda:0").manual_seed(11)
    X = torch.randn(a.probe_cols, sec.dim, dtype=torch.complex128, device="cuda:0", generator=g)
    ctx.propagate(m, sec, X, 1, q.dt, q.krylov_dim, +1)
    y = torch.empty_like(X[0])
    torch.mul(X[0], 2.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "hv_lanczos", "L": a.probe_L, "D": sec.dim, "cols": a.probe_cols,
                      "vector_bytes": 16 * sec.dim}), flush=True)


def batch64(a):
    """The uneven batch: 64 Anderson stars (L from 8..12, U 0 -> 4), G_imp on
    50 x 50, dt = 0.05, Krylov dim 15.  Times (1) kgf_greens_neq_multi over all
    instances (each L one batch), (2) kgf_greens_neq instance by instance, and
    (3) the adjoint (kgf_greens_neq_vjp, loss sum |G - G_target|^2 with the
    target from the same instance at U = 3) for a few instances, next to the
    forward pass of the same instances."""
    import numpy as np
    import torch
    import paper_1109_1205_amd as kgf
    import workloads as wl
    qs = wl.batch_instances()
    ctx = kgf.Context(0)
    if a.tune:
        ctx.set_option(ctx.HV_TUNE, 1)
    last = [time.perf_counter()]

    def report(phase, done, total):
        now = time.perf_counter()
        if now - last[0] >= 20.0:
            last[0] = now
            log(f"  {phase} {done}/{total}")
    ctx.set_progress(report)
    Hi = [ctx.model(q.H_ini) for q in qs]
    Hf = [ctx.model(q.H) for q in qs]
    secs = [ctx.sector(q.H.L, q.n_up, q.n_dn) for q in qs]
    v0 = [torch.from_numpy(wl.start_vector(s_.dim, 7)).to("cuda:0") for s_ in secs]
    q0 = qs[0]
    kw = dict(orbitals=q0.orbitals, nt=q0.nt, steps_per_grid=q0.steps_per_grid, dt=q0.dt, krylov_dim=q0.krylov_dim)
    vsteps = len(qs) * ((q0.nt - 1) * q0.steps_per_grid + q0.steps_per_grid * q0.nt * (q0.nt - 1))
    torch.cuda.synchronize()
    log("batched: 64 instances (small-sector groups in lockstep)")
    t0 = time.perf_counter()
    outb = ctx.greens_neq_multi(Hi, Hf, secs, v0, **kw)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    log(f"batched {tb:.1f} s; group by group:")
    ctx.set_option(ctx.LOCKSTEP, 0)
    t0 = time.perf_counter()
    outg = ctx.greens_neq_multi(Hi, Hf, secs, v0, **kw)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    ctx.set_option(ctx.LOCKSTEP, 1)
    same_g = bool(np.array_equal(outg["G_lesser"], outb["G_lesser"]) and np.array_equal(outg["G_greater"],
                                                                                          outb["G_greater"]))
    log(f"group by group {tg:.1f} s (bitwise equal: {same_g}); per instance:")
    t0 = time.perf_counter()
    maxdiff = 0.0
    for i in ([] if a.skip_per_instance else range(len(qs))):
        o = ctx.greens_neq(Hi[i], Hf[i], secs[i], v0[i], schedule=1, **kw)
        sc = max(np.abs(o["G_lesser"]).max(), np.abs(o["G_greater"]).max())
        maxdiff = max(maxdiff, np.abs(o["G_lesser"] - outb["G_lesser"][i]).max() / sc,
                      np.abs(o["G_greater"] - outb["G_greater"][i]).max() / sc)
        if (i + 1) % 8 == 0:
            log(f"  {i + 1}/64")
    torch.cuda.synchronize()
    tp = None if a.skip_per_instance else time.perf_counter() - t0
    tplain = None
    if a.plain_baseline:
        log("plain single-vector schedule, instance by instance:")
        t0 = time.perf_counter()
        for i in range(len(qs)):
            ctx.greens_neq(Hi[i], Hf[i], secs[i], v0[i], schedule=0, **kw)
            if (i + 1) % 8 == 0:
                log(f"  {i + 1}/64")
        torch.cuda.synchronize()
        tplain = time.perf_counter() - t0
    # adjoint timings: the first instance of each L, then more
    order = sorted(range(len(qs)), key=lambda i: (qs[i].H.L, i))
    pick, seen = [], set()
    for i in order:
        if qs[i].H.L not in seen:
            pick.append(i)
            seen.add(qs[i].H.L)
    pick = pick[:max(1, a.grad_instances)]
    grad_rows = []
    for i in pick:
        q = qs[i]
        tgt_model = q.H.with_U([3.0] + [0.0] * (q.H.L - 1))
        tgt = ctx.greens_neq(ctx.model(q.H_ini), ctx.model(tgt_model), secs[i], v0[i], schedule=1, **kw)
        Wl = 2.0 * (outb["G_lesser"][i] - tgt["G_lesser"])
        Wg = 2.0 * (outb["G_greater"][i] - tgt["G_greater"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = ctx.greens_neq(Hi[i], Hf[i], secs[i], v0[i], schedule=0, **kw)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        t0 = time.perf_counter()
        r = ctx.greens_neq_vjp(Hi[i], Hf[i], secs[i], v0[i], q.orbitals, q.nt, q.steps_per_grid, q.dt, Wl, Wg,
                               krylov_dim=q.krylov_dim, quad_nodes=12)
        torch.cuda.synchronize()
        ta = time.perf_counter() - t0
        grad_rows.append({"instance": q.name, "D": secs[i].dim, "forward_plain_s": round(tf, 2),
                          "adjoint_s": round(ta, 2), "adjoint_over_forward": round(ta / tf, 2),
                          "grad_norm": float(np.linalg.norm(r["grad"])), "cg_iters": r["cg_iters"]})
        log(f"adjoint {q.name}: forward {tf:.1f} s, adjoint {ta:.1f} s")
    # batched adjoint of all instances (same loss, targets at U = 3)
    bat_adj = None
    if not a.no_batched_adjoint:
        log("targets for the batched adjoint (U = 3)")
        tg = ctx.greens_neq_multi(Hi, [ctx.model(q.H.with_U([3.0] + [0.0] * (q.H.L - 1))) for q in qs], secs, v0,
                                  **kw)
        Wl = [2.0 * (outb["G_lesser"][i] - tg["G_lesser"][i]) for i in range(len(qs))]
        Wg = [2.0 * (outb["G_greater"][i] - tg["G_greater"][i]) for i in range(len(qs))]
        log("batched adjoint of 64 instances")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = ctx.greens_neq_vjp_multi(Hi, Hf, secs, v0, q0.orbitals, q0.nt, q0.steps_per_grid, q0.dt, Wl, Wg,
                                      krylov_dim=q0.krylov_dim, quad_nodes=12)
        torch.cuda.synchronize()
        tba = time.perf_counter() - t0
        # per-instance adjoint time estimated from the sampled instances, per L
        per_L = {}
        for r in grad_rows:
            per_L[int(r["instance"].split("_L")[1])] = r["adjoint_s"]
        Ls = [q.H.L for q in qs]
        est = sum(per_L[L] * Ls.count(L) for L in per_L) if len(per_L) == len(set(Ls)) else None
        bat_adj = {"batched_adjoint_s": round(tba, 2),
                   "per_instance_adjoint_s_estimated": (round(est, 1) if est else None),
                   "speedup_estimated": (round(est / tba, 2) if est else None),
                   "batched_adjoint_over_batched_forward": round(tba / tb, 2),
                   "grad_norm_sum": float(sum(np.linalg.norm(r["grad"]) for r in rs))}
        log(f"batched adjoint {tba:.1f} s")
    res = {"metric": "G(t,t') contour steps/s, 64 uneven Anderson instances (batched vs per instance)",
           "value": round(vsteps / tb, 1), "unit": "vector-steps/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batch64: 64 Anderson stars, L 8..12 (seeds 4000+i), U 0->4, eps_imp -2, "
                                  "G_imp 50x50, t_k=0.2k, dt=0.05, Krylov dim 15",
                      "vector_steps": vsteps},
           "batched_s": round(tb, 2), "group_by_group_s": round(tg, 2),
           "lockstep_speedup_vs_group_by_group": round(tg / tb, 3), "lockstep_bitwise_equal": same_g,
           "per_instance_s": (round(tp, 2) if tp else None),
           "speedup": (round(tp / tb, 3) if tp else None),
           "per_instance_value": (round(vsteps / tp, 1) if tp else None),
           "max_rel_diff_batched_vs_per_instance": (maxdiff if tp else None),
           "plain_single_vector_s": (round(tplain, 2) if tplain else None),
           "speedup_vs_plain": (round(tplain / tb, 3) if tplain else None),
           "adjoint": grad_rows, "batched_adjoint": bat_adj}
    print(json.dumps(res), flush=True)


def ladder16(a):
    """The 2x8 ladder quench (D = 165,636,900) on a short mesh of --nt16
    points: restarted ground state, checkpointed forward mesh, sweeps of
    the c and c+ branches.  Reports contour steps/s and the Lanczos H.v rate."""
    import numpy as np
    import torch
    import paper_1109_1205_amd as kgf
    import workloads as wl
    q = wl.ladder16()
    ctx = kgf.Context(0)
    if a.tune:
        ctx.set_option(ctx.HV_TUNE, 1)
    last = [time.perf_counter()]

    def report(phase, done, total):
        now = time.perf_counter()
        if now - last[0] >= 20.0 or done == total:
            last[0] = now
            log(f"  {phase} {done}/{total}")
    ctx.set_progress(report)
    s = ctx.sector(16, q.n_up, q.n_dn)
    v0 = torch.from_numpy(wl.start_vector(s.dim, q.gs_seed)).to("cuda:0")
    nt = a.nt16
    ctx.profile_begin(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    spg = a.spg16
    out = ctx.greens_neq(ctx.model(q.H_ini), ctx.model(q.H), s, v0, orbitals=q.orbitals, nt=nt, steps_per_grid=spg,
                         dt=q.dt, krylov_dim=q.krylov_dim, schedule=1, gs_tol=q.gs_tol, gs_max_iter=2000)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = ctx.profile_end()
    Gl, Gg = out["G_lesser"][:, :, 0, 0], out["G_greater"][:, :, 0, 0]
    vsteps = ((nt - 1) + nt * (nt - 1)) * spg
    step = {}
    for k in ("hv_lanczos", "hv_rows_lanczos", "hv_up_lanczos", "lanczos_update"):
        if k in st and st[k]["sampled"]:
            step[k] = {"avg_ms": round(st[k]["sampled_ms"] / st[k]["sampled"], 3),
                       "GBps": round(st[k]["sampled_bytes"] / max(st[k]["sampled_ms"], 1e-9) / 1e6, 1)}
    res = {"metric": "four-step on the 2x8 ladder (L=16)", "D": s.dim, "nt": nt, "steps_per_interval": spg,
           "dt": q.dt, "t_max": round((nt - 1) * spg * q.dt, 6), "elapsed_s": round(el, 2), "vector_steps": vsteps,
           "anticommutator_err": float(np.abs(np.diag(Gg - Gl) + 1j).max()), "E0": out["E0"],
           "hermiticity_err": float(np.abs(Gl + np.conj(Gl.T)).max()),
           "n0_up": float(np.real(-1j * Gl[0, 0])), "lanczos_kernels": step,
           "kernels": {k: {"launches": v["launches"], "total_ms": round(v["sampled_ms"], 1)}
                       for k, v in sorted(st.items())}}
    print(json.dumps(res), flush=True)
    if a.adj16:
        # the adjoint of Re sum conj(W) G^< on a mesh of adj16 points (W seeded
        # by 5), chains checkpointed every 10 SIL steps
        nta = a.adj16
        rng = np.random.default_rng(5)
        W = (rng.standard_normal((nta, nta, 1, 1)) + 1j * rng.standard_normal((nta, nta, 1, 1))) / nta
        # a fresh context: the forward's sweep blocks (sized from free memory)
        # stay cached in the first one's workspaces
        ctx.close()
        torch.cuda.empty_cache()
        ctx = kgf.Context(0)
        if a.tune:
            ctx.set_option(ctx.HV_TUNE, 1)
        ctx.set_progress(report)
        s = ctx.sector(16, q.n_up, q.n_dn)
        ctx.set_option(ctx.ADJ_EVERY, 10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fw = ctx.greens_neq(ctx.model(q.H_ini), ctx.model(q.H), s, v0, orbitals=q.orbitals, nt=nta,
                            steps_per_grid=spg, dt=q.dt, krylov_dim=q.krylov_dim, schedule=0, gs_tol=q.gs_tol,
                            gs_max_iter=2000)
        torch.cuda.synchronize()
        t_fw = time.perf_counter() - t0
        ctx.close()   # again: the plain forward's blocks are sized from free memory too
        torch.cuda.empty_cache()
        ctx = kgf.Context(0)
        if a.tune:
            ctx.set_option(ctx.HV_TUNE, 1)
        ctx.set_progress(report)
        s = ctx.sector(16, q.n_up, q.n_dn)
        ctx.set_option(ctx.ADJ_EVERY, 10)
        t0 = time.perf_counter()
        g = ctx.greens_neq_vjp(ctx.model(q.H_ini), ctx.model(q.H), s, v0, q.orbitals, nta, spg, q.dt, W_lesser=W,
                               krylov_dim=q.krylov_dim, gs_tol=q.gs_tol, gs_max_iter=2000)
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
        ctx.set_option(ctx.ADJ_EVERY, 0)
        nb = len(q.H.bonds)
        print(json.dumps({"metric": "adjoint gradient on the 2x8 ladder (L=16)", "nt": nta, "steps_per_interval": spg,
                          "checkpoint_every": 10, "forward_plain_schedule_s": round(t_fw, 2),
                          "vjp_s": round(t_adj, 2), "cg_iters": g["cg_iters"],
                          "loss": float(np.real(np.sum(np.conj(W) * g["G_lesser"]))),
                          "forward_G_matches": float(np.abs(g["G_lesser"] - fw["G_lesser"]).max()),
                          "grad_hoppings_first4": [round(float(x), 10) for x in g["grad"][:4]],
                          "grad_U_site0": float(g["grad"][nb + 32])}), flush=True)


def hub4x3(a):
    """Equilibrium G_ij(t) of the half-filled 4x3 cluster (t' = -0.3, U = 8,
    D = 853,776): 12 c_i^+ vectors in (7,6) and 12 c_i vectors in (5,6), 400
    SIL steps of dt = 0.025, Krylov dim 15, all 12 x 12 dots per step.
    Timed with the columns of each sector in one block (batched) and one
    column at a time (plain); both give the same G."""
    import numpy as np
    import torch
    import paper_1109_1205_amd as kgf
    import workloads as wl
    q = wl.hub4x3()
    ctx = kgf.Context(0)
    m = ctx.model(q.H)
    s = ctx.sector(q.H.L, q.n_up, q.n_dn)
    v0 = torch.from_numpy(wl.start_vector(s.dim, 7)).to("cuda:0")
    E0, psi0, info = ctx.ground_state(m, s, v0, tol=1e-12, max_iter=400)
    log(f"hub4x3 ground state E0={E0} ({info['iters']} iterations)")
    res, G = {}, {}
    for name, batch in (("batched", 0), ("plain", 1)):
        ctx.greens_eq(m, s, psi0, E0, q.orbitals, 3, 1, q.dt_grid, krylov_dim=q.krylov_dim, batch=batch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G[name] = ctx.greens_eq(m, s, psi0, E0, q.orbitals, q.nt, q.steps_per_grid, q.dt_grid,
                                krylov_dim=q.krylov_dim, batch=batch)
        el = time.perf_counter() - t0
        vsteps = 2 * len(q.orbitals) * (q.nt - 1) * q.steps_per_grid
        res[name] = {"s": round(el, 3), "vector_steps_per_s": round(vsteps / el, 1)}
        log(f"hub4x3 {name}: {el:.2f} s")
    dG = max(float(np.abs(G["batched"][i] - G["plain"][i]).max()) for i in range(2))
    out = {"metric": "equilibrium G of the 4x3 cluster, 24 columns, batched vs plain", "D": s.dim,
           "vector_steps": 2 * len(q.orbitals) * (q.nt - 1) * q.steps_per_grid, **res,
           "batched_over_plain": round(res["plain"]["s"] / res["batched"]["s"], 2),
           "max_abs_diff_batched_plain": dG,
           "anticommutator_err": float(np.abs(np.diagonal(G["batched"][0][0] - G["batched"][1][0]) + 1j).max())}
    print(json.dumps(out), flush=True)


def driven(a):
    """Driven 2x7 ladder (7,7), D = 11,778,624: H(t) = H0 + 0.5 sin(2t) K_rung
    (K_rung: the hopping on the seven rungs), 10 steps of h = 0.05 of the
    fourth-order commutator-free integrator (two SIL steps of Krylov dim 20
    per step), timed against 20 static SIL steps of the same size."""
    import numpy as np
    import torch
    import paper_1109_1205_amd as kgf
    import workloads as wl
    q = wl.ladder14()
    ctx = kgf.Context(0)
    H0 = q.H
    nb, L = len(H0.bonds), H0.L
    th0 = np.concatenate([np.asarray(H0.t, float), np.asarray(H0.eps_up, float), np.asarray(H0.eps_dn, float),
                          np.asarray(H0.U, float)])
    kr = np.zeros(nb + 3 * L)
    for b, (i, j) in enumerate(H0.bonds):
        if j == i + 1 and i % 2 == 0:        # rung (2x, 2x+1) in the rung-major numbering
            kr[b] = 1.0
    f = lambda t: [1.0, 0.5 * np.sin(2.0 * t)]
    s = ctx.sector(L, q.n_up, q.n_dn)
    g = torch.Generator(device="cuda:0").manual_seed(3)
    x = torch.randn(1, s.dim, dtype=torch.complex128, device="cuda:0", generator=g)
    x /= torch.linalg.vector_norm(x)
    work, m0 = ctx.model(H0), ctx.model(H0)
    y = x.clone()
    ctx.propagate_driven(work, s, y, [th0, kr], f, 1, 0.05, krylov_dim=q.krylov_dim)   # warm-up (tables)
    ctx.propagate(m0, s, y, 1, 0.05, q.krylov_dim)
    torch.cuda.synchronize()
    y = x.clone()
    t0 = time.perf_counter()
    ctx.propagate_driven(work, s, y, [th0, kr], f, 10, 0.05, krylov_dim=q.krylov_dim)
    torch.cuda.synchronize()
    td = time.perf_counter() - t0
    z = x.clone()
    t0 = time.perf_counter()
    ctx.propagate(m0, s, z, 20, 0.05, q.krylov_dim)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    out = {"metric": "driven 2x7 ladder, commutator-free 4th order, 10 steps (20 SIL steps)", "D": s.dim,
           "driven_s": round(td, 3), "static_20_sil_steps_s": round(ts, 3), "overhead": round(td / ts - 1.0, 3),
           "norm_err": float(abs(torch.linalg.vector_norm(y).item() - 1.0))}
    print(json.dumps(out), flush=True)


def driven4(a):
    """Four-step G^<_00, G^>_00 of the 2x7 ladder quench (U 4 -> 8, D =
    11,778,624) with the periodic rung drive of the driven mode added to the
    final Hamiltonian: 11 mesh times 0.1 apart, one commutator-free step (two
    SIL steps of Krylov dim 20) per interval, timed against the static
    four-step with the same number of SIL steps (two of 0.05 per interval)."""
    import numpy as np
    import torch
    import paper_1109_1205_amd as kgf
    import workloads as wl
    q = wl.ladder14()
    ctx = kgf.Context(0)
    H = q.H
    nb, L = len(H.bonds), H.L
    th0 = np.concatenate([np.asarray(H.t, float), np.asarray(H.eps_up, float), np.asarray(H.eps_dn, float),
                          np.asarray(H.U, float)])
    kr = np.zeros(nb + 3 * L)
    for b, (i, j) in enumerate(H.bonds):
        if j == i + 1 and i % 2 == 0:
            kr[b] = 1.0
    f = lambda t: [1.0, 0.5 * np.sin(2.0 * t)]
    s = ctx.sector(L, q.n_up, q.n_dn)
    v0 = torch.from_numpy(wl.start_vector(s.dim, q.gs_seed)).to("cuda:0")
    m_ini, m_fin, work = ctx.model(q.H_ini), ctx.model(H), ctx.model(H)
    res, G = {}, {}

    def run(name, nt):
        if name == "driven":
            return ctx.greens_neq_driven(m_ini, work, s, v0, q.orbitals, [th0, kr], f, nt=nt, steps_per_grid=1,
                                         dt=0.1, krylov_dim=q.krylov_dim, gs_tol=q.gs_tol)
        return ctx.greens_neq(m_ini, m_fin, s, v0, orbitals=q.orbitals, nt=nt, steps_per_grid=2, dt=0.05,
                              krylov_dim=q.krylov_dim, schedule=1, gs_tol=q.gs_tol)
    for name in ("driven", "static"):
        run(name, 2)      # warm-up: hopping tables of the three sectors, workspaces
        log(f"driven4 {name}: warm-up done")
    nt = 11
    for name in ("driven", "static"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = run(name, nt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        Gl, Gg = out["G_lesser"][:, :, 0, 0], out["G_greater"][:, :, 0, 0]
        G[name] = Gl
        res[name] = {"s": round(el, 3), "anticommutator_err": float(np.abs(np.diag(Gg - Gl) + 1j).max()),
                     "E0": out["E0"]}
        log(f"driven4 {name}: {el:.2f} s")
    sil = 2 * (nt - 1) + 2 * 2 * nt * (nt - 1) // 2
    print(json.dumps({"metric": "driven four-step on the 2x7 ladder, 11 mesh times, vs static four-step "
                                "with equal SIL steps", "D": s.dim, "sil_vector_steps": sil, **res,
                      "overhead": round(res["driven"]["s"] / res["static"]["s"] - 1.0, 3),
                      "max_abs_Glesser_driven_minus_static": float(np.abs(G["driven"] - G["static"]).max())}),
          flush=True)


def necpt_bench(a):
    """Sec. 5 setting on the GPU: Anderson chain of L_c = 6 sites (U = T = V = 1,
    field h = 0.2 on the impurity for t < 0, half filling) linked at its last
    site to a 1000-site bath, t_max = 10, dt = 0.02 (nt = 501): four-step
    cluster G^<, G^> of all six sites for both spins, bath functions, and the
    CPT equation on the Keldysh contour per spin (1002 contour points, 6012
    right-hand sides).  Reports the time of each part, the kernel split of the
    contour solve and the net polarisation of the first four sites; then the
    same with the imaginary branch (beta = 15, dtau = 0.02: 751 more contour
    points), through which the connected system's initial state enters."""
    import numpy as np
    import torch
    import paper_1109_1205_amd as kgf
    import workloads as wl
    Lc, Lb, V, dt, tmax = 6, 1000, 1.0, 0.02, 10.0
    nt = int(round(tmax / dt)) + 1
    ctx = kgf.Context(0)
    H = wl.chain_siam(Lc, 1.0, 1.0)
    Hi = H.with_field(0, 0.2)
    s = ctx.sector(Lc, Lc // 2, Lc // 2)
    v0 = torch.from_numpy(wl.start_vector(s.dim, 7)).to("cuda:0")
    orbs = [(i, sp) for sp in (0, 1) for i in range(Lc)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = ctx.greens_neq(ctx.model(Hi), ctx.model(H), s, v0, orbs, nt=nt, steps_per_grid=1, dt=dt, krylov_dim=15,
                         reorth=2, gs_tol=1e-13)
    t_fs = time.perf_counter() - t0
    log(f"necpt: cluster four-step {t_fs:.2f} s")
    t0 = time.perf_counter()
    gbl, gbg = ctx.bath_chain(Lb, 1.0, nt, dt)
    torch.cuda.synchronize()
    t_bath = time.perf_counter() - t0
    dens, iso = [], []
    t_cpt = []
    ctx.profile_begin(1)
    for sp in (0, 1):
        idx = [k for k, (_, q) in enumerate(orbs) if q == sp]
        cl = np.ascontiguousarray(out["G_lesser"][:, :, idx][:, :, :, idx])
        cg = np.ascontiguousarray(out["G_greater"][:, :, idx][:, :, :, idx])
        dl, dg = torch.from_numpy(cl).to("cuda:0"), torch.from_numpy(cg).to("cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gl, gg = ctx.necpt(dl, dg, gbl, gbg, Lc - 1, V, dt)
        torch.cuda.synchronize()
        t_cpt.append(time.perf_counter() - t0)
        log(f"necpt: contour solve, spin {sp}: {t_cpt[-1]:.3f} s")
        dens.append(np.real(-1j * np.einsum("aaii->ai", gl.cpu().numpy())))
        iso.append(np.real(-1j * np.einsum("aaii->ai", cl)))
    stats = ctx.profile_end()
    m_cpt = (dens[0] - dens[1])[:, :4].sum(axis=1)
    m_iso = (iso[0] - iso[1])[:, :4].sum(axis=1)
    marks = [0, 100, 200, 300, 400, 500]
    # the same with the imaginary branch (beta = 15, dtau = 0.02): the
    # connected system's initial state enters through the CPT equation
    beta, dtau = 15.0, 0.02
    ntau = int(round(beta / dtau)) + 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outm = ctx.greens_neq(ctx.model(Hi), ctx.model(H), s, v0, orbs, nt=nt, steps_per_grid=1, dt=dt, krylov_dim=15,
                          reorth=2, gs_tol=1e-13, ntau=ntau, tau_steps_per_grid=1, dtau=dtau)
    t_fsm = time.perf_counter() - t0
    log(f"necpt: cluster four-step with the Matsubara branch ({ntau} tau points) {t_fsm:.2f} s")
    t0 = time.perf_counter()
    gb = ctx.bath_chain_contour(Lb, 1.0, nt, dt, ntau, dtau, beta)
    torch.cuda.synchronize()
    t_bathm = time.perf_counter() - t0
    # cluster functions on the contour (kgf_cluster_contour): as the ground
    # state gives them (kms 0), and completed for the finite branch (kms 1)
    densm, dens0, t_cptm = [], [], []
    for sp in (0, 1):
        idx = [k for k, (_, q) in enumerate(orbs) if q == sp]
        for kms in (1, 0):
            gcd = ctx.cluster_contour(outm, orbitals=idx, kms=bool(kms))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.necpt_contour(gcd, gb, Lc - 1, V, dt, dtau)
            torch.cuda.synchronize()
            if kms:
                t_cptm.append(time.perf_counter() - t0)
                log(f"necpt: contour solve with the Matsubara branch, spin {sp}: {t_cptm[-1]:.3f} s")
            (densm if kms else dens0).append(np.real(-1j * np.einsum("aaii->ai", res["G_lesser"].cpu().numpy())))
            del gcd, res
            torch.cuda.empty_cache()
    m_m = (densm[0] - densm[1])[:, :4].sum(axis=1)
    m1 = densm[0][:, 0] - densm[1][:, 0]
    m_sites0 = [round(float(densm[0][0, i] - densm[1][0, i]), 5) for i in range(4)]
    m_sites0_plain = [round(float(dens0[0][0, i] - dens0[1][0, i]), 5) for i in range(4)]
    m_sites0_iso = [round(float(iso[0][0, i] - iso[1][0, i]), 5) for i in range(4)]
    kern = {k: {"launches": v["launches"], "total_ms": round(v["sampled_ms"], 2)} for k, v in sorted(stats.items())}
    n, m = 2 * nt, 2 * nt * Lc
    gemm_flops = 8.0 * (n * n * n + n * n * m + m * m * n)     # 1 - P K, K X, R (K X)
    zg = stats.get("k_zgemm", {"sampled_ms": 0.0})
    print(json.dumps({"metric": "NE-CPT, L_c=6 Anderson chain + 1000-site bath, t_max=10, dt=0.02",
                      "nt": nt, "contour_points": n, "rhs": m, "cluster_four_step_s": round(t_fs, 3),
                      "bath_s": round(t_bath, 4), "contour_solve_s": [round(x, 4) for x in t_cpt],
                      "kernels": kern,
                      "zgemm_TFLOPs": (round(gemm_flops / (zg["sampled_ms"] / 2 * 1e-3) / 1e12, 2)
                                       if zg["sampled_ms"] else None),
                      "net_moment_sites_1_4": {f"t={dt * k:g}": [round(float(m_cpt[k]), 5), round(float(m_iso[k]), 5),
                                                                 round(float(m_m[k]), 5)]
                                               for k in marks},
                      "moment_columns": ["NE-CPT (Keldysh contour, disconnected initial state)", "isolated cluster",
                                         "NE-CPT with the Matsubara branch (beta = 15)"],
                      "matsubara_branch": {"beta": beta, "dtau": dtau, "ntau": ntau, "contour_points": 2 * nt + ntau,
                                           "rhs": (2 * nt + ntau) * Lc, "cluster_four_step_s": round(t_fsm, 3),
                                           "bath_s": round(t_bathm, 4),
                                           "contour_solve_s": [round(x, 4) for x in t_cptm],
                                           "impurity_moment_m1": {f"t={dt * k:g}": round(float(m1[k]), 5)
                                                                  for k in marks},
                                           "t0_moments_sites_1_4": {
                                               "cpt_completed_cluster_functions": m_sites0,
                                               "cpt_ground_state_cluster_functions": m_sites0_plain,
                                               "isolated_cluster": m_sites0_iso}}}), flush=True)


def two_particle(a):
    """Four-time function <c+_a(t1) c+_b(t2) c_c(t3) c_d(t4)> of the L = 8
    Anderson chain (U = 2, field 0.2 on the impurity for t < 0, sector (4,4),
    D = 4900) for the impurity and the far end, both spins (4 orbitals), on
    8 mesh times 0.2 apart (4 SIL steps of Krylov dim 15 per interval)."""
    import numpy as np
    import torch
    import paper_1109_1205_amd as kgf
    import workloads as wl
    ctx = kgf.Context(0)
    H = wl.chain_siam(8, 2.0, 1.0)
    Hi = H.with_field(0, 0.2)
    s = ctx.sector(8, 4, 4)
    v0 = torch.from_numpy(wl.start_vector(s.dim, 7)).to("cuda:0")
    orbs = [(0, 0), (7, 0), (0, 1), (7, 1)]
    nt, spg = 8, 4
    mi, mh = ctx.model(Hi), ctx.model(H)
    ctx.greens2_neq(mi, mh, s, v0, orbs, nt=2, steps_per_grid=1, dt=0.05)      # warm-up (tables)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = ctx.greens2_neq(mi, mh, s, v0, orbs, nt=nt, steps_per_grid=spg, dt=0.05)
    el = time.perf_counter() - t0
    nx = ny = 2
    per_class = nt * (nt - 1) * spg * ny + sum((nt - k) * nt * nx * ny for k in range(1, nt)) * spg
    vsteps = 4 * per_class + (nt - 1) * spg
    chi = out["chi"]
    print(json.dumps({"metric": "four-time function, L=8 Anderson chain, 4 orbitals, 8x8x8x8 mesh", "D": s.dim,
                      "elapsed_s": round(el, 3), "sil_vector_steps": vsteps,
                      "vector_steps_per_s": round(vsteps / el, 1), "E0": out["E0"],
                      "equal_time_antisymmetry_err": float(max(
                          np.abs(chi[k, k] + np.swapaxes(chi[k, k], -4, -3)).max() for k in range(nt)))}), flush=True)


def graphs(a):
    """Launch-bound small sectors with and without captured SIL steps
    (KGF_OPT_GRAPHS): the equilibrium G of the half-filled 8-site ring
    (D = 4,900; all 8 sites, 200 SIL steps of dt = 0.05, Krylov dim 15) and
    the four-step G of a 10-site Anderson star; both runs give bitwise the
    same G."""
    import numpy as np
    import torch
    import paper_1109_1205_amd as kgf
    import workloads as wl
    ctx = kgf.Context(0)
    q = wl.ring8()
    m = ctx.model(q.H)
    s = ctx.sector(8, 4, 4)
    v0 = torch.from_numpy(wl.start_vector(s.dim, 7)).to("cuda:0")
    E0, psi0, _ = ctx.ground_state(m, s, v0, tol=1e-12, max_iter=400)
    q10 = wl.siam10()
    s10 = ctx.sector(10, 5, 5)
    v10 = torch.from_numpy(wl.start_vector(s10.dim, 7)).to("cuda:0")
    mi10, mf10 = ctx.model(q10.H_ini), ctx.model(q10.H)
    res = {}
    for on in (0, 1, 0, 1):
        ctx.set_option(ctx.GRAPHS, on)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G = ctx.greens_eq(m, s, psi0, E0, q.orbitals, q.nt, q.steps_per_grid, q.dt_grid, krylov_dim=q.krylov_dim)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        G4 = ctx.greens_neq(mi10, mf10, s10, v10, q10.orbitals, nt=21, steps_per_grid=q10.steps_per_grid,
                            dt=q10.dt, krylov_dim=q10.krylov_dim)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res[on] = {"ring8_greens_eq_s": round(t1 - t0, 4), "siam10_four_step_nt21_s": round(t2 - t1, 4),
                   "G": G, "G4": G4["G_lesser"]}
        log(f"graphs={on}: ring8 {t1 - t0:.3f} s, siam10 {t2 - t1:.3f} s")
    same = all(np.array_equal(res[0]["G"][i], res[1]["G"][i]) for i in range(2)) and np.array_equal(
        res[0]["G4"], res[1]["G4"])
    vsteps = 2 * len(q.orbitals) * (q.nt - 1) * q.steps_per_grid
    print(json.dumps({"metric": "captured SIL steps vs eager launches, small sectors",
                      "ring8_eq_vector_steps": vsteps,
                      "eager": {k: v for k, v in res[0].items() if k.endswith("_s")},
                      "graphs": {k: v for k, v in res[1].items() if k.endswith("_s")},
                      "ring8_speedup": round(res[0]["ring8_greens_eq_s"] / res[1]["ring8_greens_eq_s"], 2),
                      "siam10_speedup": round(res[0]["siam10_four_step_nt21_s"] / res[1]["siam10_four_step_nt21_s"],
                                              2),
                      "bitwise_equal": bool(same)}), flush=True)


def fig1(a):
    """Sec. 3 on the GPU: local spectral density A(w) = -Im G_00(w) / pi of the
    half-filled L=10 Hubbard ring at U=8 (T=1), eta = 0.01, t_max = 1000, fine
    grid 0.01, Krylov dimension 100 (the paper's n), from the time-dependent Lanczos G(t) with
    f = 1000, 100 and 1 restarts and a damped transform, and the conventional
    Lanczos G^(L)(w) of the same dimension (Eq. (gapprox)); f = 1 should
    reproduce the conventional result (Eq. (res))."""
    import numpy as np
    import torch
    import paper_1109_1205_amd as kgf
    import workloads as wl
    ctx = kgf.Context(0)
    model = wl.ring(10, 1.0, 8.0)
    m = ctx.model(model)
    s = ctx.sector(10, 5, 5)
    v0 = torch.from_numpy(wl.start_vector(s.dim, 7)).to("cuda:0")
    E0, psi0, info = ctx.ground_state(m, s, v0, tol=1e-13, max_iter=600)
    tmax, dtf, eta, krylov = 1000.0, 0.01, 0.01, 100
    om = np.linspace(-6.0, 14.0, 8001)
    A, times = {}, {}
    for f in (1000, 100, 1):
        dt = tmax / f
        nfine = int(round(dt / dtf))
        t0 = time.perf_counter()
        gg = ctx.greens_eq_fine(m, s, psi0, E0, (0, 0), 1, f, nfine, dt, krylov_dim=krylov, reorth=2)
        gl = ctx.greens_eq_fine(m, s, psi0, E0, (0, 0), 0, f, nfine, dt, krylov_dim=krylov, reorth=2)
        Gw = ctx.fourier(gg - gl, dtf, eta, om)
        torch.cuda.synchronize()
        times[f] = round(time.perf_counter() - t0, 2)
        A[f] = -Gw.imag / np.pi
        log(f"f={f}: {times[f]} s")
    t0 = time.perf_counter()
    conv = ctx.greens_omega(m, s, psi0, E0, (0, 0), krylov, om, eta, reorth=2)
    times["conventional"] = round(time.perf_counter() - t0, 2)
    Ac = -(conv["G_greater"] + conv["G_lesser"]).imag / np.pi
    conv64 = ctx.greens_omega(m, s, psi0, E0, (0, 0), 64, om, eta, reorth=2)
    A["conv64"] = -(conv64["G_greater"] + conv64["G_lesser"]).imag / np.pi
    ref = A[1000]
    sc = np.abs(ref).max()
    # the bipartite ring is particle-hole symmetric about w = U/2: bins of
    # w' = w - U/2 >= 0 across the upper Hubbard band
    wp = om - 4.0
    wins = {f"{lo}<=w'<{lo + 1}": (wp >= lo) & (wp < lo + 1) for lo in range(0, 9)}
    dev = {(f"f={f}" if f != "conv64" else "conventional n=64"): {k: round(float(np.abs(A[f][w] - ref[w]).max() / sc), 6) for k, w in wins.items()}
           for f in (100, 1, "conv64")}
    res = {"metric": "Sec. 3 spectral density, L=10 ring U=8 (time-dependent vs conventional Lanczos)",
           "E0": E0, "gs_iters": info["iters"], "times_s": {str(k): v for k, v in times.items()},
           "deviation_from_f1000_rel_max": dev,
           "min_A": {f"f={f}": float(A[f].min()) for f in (1000, 100, 1)},
           "f1_vs_conventional_rel_max": float(np.abs(A[1] - Ac).max() / np.abs(Ac).max()),
           "sum_rule_f1000": float(np.trapezoid(ref, om) if hasattr(np, "trapezoid") else np.trapz(ref, om)),
           "config": {"workload": "ring10 U=8 half filling, eta=0.01, t_max=1000, fine dt=0.01, Krylov dim 100",
                      "omega": [float(om[0]), float(om[-1]), len(om)]}}
    print(json.dumps(res), flush=True)


def measured_traffic(kernel):
    """HBM bytes per algorithmic byte of a kernel class from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by the
    plain-copy calibration).  None when there is no summary for the class or
    the kernel source has changed since the counters were taken."""
    import hashlib
    if kernel not in TRAFFIC_FILES:
        return None
    src = os.path.join(ROOT, "paper_1109_1205_amd", "csrc", "hamiltonian.hip")
    cur = hashlib.sha1(open(src, "rb").read()).hexdigest()
    ratio, sha = None, None
    keys = ("traffic_bytes_per_algorithmic_byte:", f"traffic_bytes_per_algorithmic_byte.{kernel}:")
    try:
        for line in open(TRAFFIC_FILES[kernel]):
            if line.startswith(keys):
                ratio = float(line.split(":", 1)[1].strip())
            if line.startswith("kernel_source_sha1:"):
                sha = line.split(":", 1)[1].split()[0]
    except OSError:
        return None
    return ratio if sha == cur else None


def cpu_baseline(q):
    """The oracle as it stands: one SIL step (Krylov dim 20) of a c-sector
    vector of the same ladder on the host, BLAS/OpenMP pools held to one
    thread (scipy.sparse products and NumPy elementwise work are
    single-threaded anyway)."""
    import workloads as wl
    from oracle import basis, hamiltonian, propagate
    from threadpoolctl import threadpool_limits
    sec = basis.Sector(14, 6, 7)
    H = hamiltonian.Hamiltonian(q.H, sec)
    v = wl.complex_vector(sec.dim, 1)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        propagate.sil_step(H.apply, v, q.dt, q.krylov_dim, +1, reorth="none")
        dt = time.perf_counter() - t0
    return {"value": round(1.0 / dt, 5), "unit": "vector-steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"one SIL step (Krylov dim {q.krylov_dim}, dt={q.dt}, no reorthogonalisation) of a random "
                       f"D={sec.dim} c-sector vector of the 2x7 ladder with the NumPy/SciPy oracle, {dt:.1f} s on "
                       f"one thread (host os.cpu_count()={os.cpu_count()})")}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}): every workload here is a "
              "single-device run", file=sys.stderr)
        sys.exit(2)
    if a.probe:
        probe(a)
        return
    if a.hv:
        hv_bench(a)
        return
    if a.workload == "batch64":
        batch64(a)
        return
    if a.workload == "ladder16":
        ladder16(a)
        return
    if a.workload == "fig1":
        fig1(a)
        return
    if a.workload == "hub4x3":
        hub4x3(a)
        return
    if a.workload == "driven":
        driven(a)
        return
    if a.workload == "driven4":
        driven4(a)
        return
    if a.workload == "necpt":
        necpt_bench(a)
        return
    if a.workload == "two_particle":
        two_particle(a)
        return
    if a.workload == "graphs":
        graphs(a)
        return
    if a.whole:
        whole_runs(a)
        return
    stepwise(a)


HV_CLASSES = ("hv_lanczos", "hv_up_lanczos", "hv_rows_lanczos")


def roofline_of(stats):
    """roofline object of the dominant H.v kernel (the Lanczos-form H.v class
    with the most time: the single pass, or the strip or row pass of the
    fused two-pass step) from the library's HIP-event samples, plus a
    per-class kernel table."""
    def total(v):
        return v["sampled_ms"] / max(v["sampled"], 1) * v["launches"]
    dom = max(stats.items(), key=lambda kv: total(kv[1]))
    present = [k for k in HV_CLASSES if k in stats and stats[k]["sampled"]]
    kernel = max(present, key=lambda k: total(stats[k])) if present else dom[0]
    hv = stats[kernel]
    achieved = hv["sampled_bytes"] / (hv["sampled_ms"] * 1e-3) / 1e9 if hv["sampled_ms"] > 0 else 0.0
    tb = measured_traffic(kernel)
    avg_launch_bytes = hv["sampled_bytes"] / max(hv["sampled"], 1)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": (round(tb * avg_launch_bytes) if tb is not None else None),
                "kernel": kernel, "avg_launch_ms": round(hv["sampled_ms"] / max(hv["sampled"], 1), 5),
                "avg_launch_algorithmic_bytes": round(avg_launch_bytes),
                "dominant_class": dom[0]}
    kernels = {k: {"launches": v["launches"], "avg_ms": round(v["sampled_ms"] / max(v["sampled"], 1), 5),
                   "total_ms": round(v["sampled_ms"] * v["launches"] / max(v["sampled"], 1), 1),
                   "GBps": (round(v["sampled_bytes"] / (v["sampled_ms"] * 1e-3) / 1e9, 1)
                            if v["sampled_bytes"] and v["sampled_ms"] else None)}
               for k, v in sorted(stats.items())}
    return roofline, kernels


WORKLOAD_14 = ("ladder14 quench: 2x7 open Hubbard ladder t=1, half filling, D=11,778,624, U 4->8, "
               "G^<_00 and G^>_00 on 101x101, Krylov dim 20, dt=0.05")


def stepwise(a):
    """Default mode: the four-step run of the 2x7 ladder through
    kgf_neq_run_*, one timed step = one backward-sweep mesh interval at the
    production block width."""
    import numpy as np
    import torch

    import paper_1109_1205_amd as kgf
    import workloads as wl

    q = wl.ladder14()
    ctx = kgf.Context(0)
    if a.tune:
        ctx.set_option(ctx.HV_TUNE, 1)
    if a.hv_plan:
        ctx.set_option(ctx.HV_PASSES, a.hv_plan)
    if a.no_graphs:
        ctx.set_option(ctx.GRAPHS, 0)
    m_ini, m_fin = ctx.model(q.H_ini), ctx.model(q.H)
    sec = ctx.sector(14, q.n_up, q.n_dn)
    v0 = torch.from_numpy(wl.start_vector(sec.dim, q.gs_seed)).to("cuda:0")
    vec_total = (q.nt - 1) * q.steps_per_grid + 2 * q.steps_per_grid * q.nt * (q.nt - 1) // 2
    phases = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run = ctx.neq_run(m_ini, m_fin, sec, v0, q.orbitals, nt=q.nt, steps_per_grid=q.steps_per_grid, dt=q.dt,
                      krylov_dim=q.krylov_dim, reorth=a.reorth, batch=a.batch, gs_tol=q.gs_tol)
    torch.cuda.synchronize()
    phases["ground_state_and_forward_mesh_s"] = round(time.perf_counter() - t0, 3)
    log(f"ground state + forward mesh: {phases['ground_state_and_forward_mesh_s']} s (E0 = {run.E0})")
    # growth phase: advance until the next interval runs at the chunk's full width
    # with enough full-width intervals left for warm-up and timed steps
    t0 = time.perf_counter()
    info = run.advance(0)
    grow_steps = 0
    while not info["done"]:
        if (info["next_width"] == info["chunk_width"]
                and info["next_mesh_index"] >= a.warmup + a.steps):
            break
        info = run.advance(1)
        grow_steps += info["vector_steps"]
    torch.cuda.synchronize()
    phases["sweep_growth_s"] = round(time.perf_counter() - t0, 3)
    phases["sweep_growth_vector_steps"] = grow_steps
    width = info["next_width"]
    log(f"sweep growth: {phases['sweep_growth_s']} s; production block width {width} columns, "
        f"{info['next_mesh_index']} full-width intervals left in this chunk")
    for w in range(a.warmup):
        run.advance(1)
    torch.cuda.synchronize()
    log(f"warm-up: {a.warmup} interval(s)")
    ctx.profile_begin(a.profile_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timed_steps, widths = 0, []
    for k in range(a.steps):
        r = run.advance(1)
        timed_steps += r["vector_steps"]
        widths.append(r["width"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = ctx.profile_end()
    elapsed = t1 - t0
    log(f"timed: {a.steps} interval(s), {timed_steps} vector-steps in {elapsed:.3f} s")
    roofline, kernels = roofline_of(stats)
    anti, full = None, None
    if not a.no_finish:
        t0 = time.perf_counter()
        while not run.advance(8)["done"]:
            pass
        torch.cuda.synchronize()
        phases["rest_of_run_s"] = round(time.perf_counter() - t0, 3)
        out = run.result()
        Gl, Gg = out["G_lesser"][:, :, 0, 0], out["G_greater"][:, :, 0, 0]
        anti = float(np.abs(np.diag(Gg - Gl) + 1j).max())
        tot = (phases["ground_state_and_forward_mesh_s"] + phases["sweep_growth_s"] + phases["rest_of_run_s"])
        log(f"rest of the run: {phases['rest_of_run_s']} s; anticommutator error {anti:.2e}")
        full = {"vector_steps": vec_total,
                "s_excluding_warmup_and_timed": round(tot, 3),
                "s_including_warmup_and_timed_estimate": round(tot + elapsed * (1 + a.warmup / max(a.steps, 1)), 3)}
        full["vector_steps_per_s"] = round(vec_total / full["s_including_warmup_and_timed_estimate"], 2)
    run.close()
    cpu = None if a.no_cpu_baseline else cpu_baseline(q)
    res = {
        "metric": "G(t,t') contour steps/s at L=14 (four-step backward sweep, Lanczos-fused H.v GB/s in roofline)",
        "value": round(timed_steps / elapsed, 2),
        "unit": "vector-steps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(1e3 * elapsed / max(a.steps, 1), 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOAD_14, "D": sec.dim, "nt": q.nt, "krylov_dim": q.krylov_dim,
                   "step": "one backward-sweep mesh interval (dots with c Phi(t_s), one batched SIL step)",
                   "block_width": width, "vector_steps_per_step": (timed_steps // max(a.steps, 1)),
                   "interval_widths": sorted(set(widths)), "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "E0": run.E0,
        "setup": phases,
        "full_four_step_run": full,
        "anticommutator_err": anti,
        "kernels": kernels,
    }
    print(json.dumps(res), flush=True)


def whole_runs(a):
    """--whole: one step = one whole four-step run (kgf_greens_neq), either
    schedule; for the schedule comparison."""
    import numpy as np
    import torch

    import paper_1109_1205_amd as kgf
    import workloads as wl

    q = wl.ladder14()
    ctx = kgf.Context(0)
    if a.tune:
        ctx.set_option(ctx.HV_TUNE, 1)
    if a.no_graphs:
        ctx.set_option(ctx.GRAPHS, 0)
    last = [time.perf_counter()]

    def report(phase, done, total):
        now = time.perf_counter()
        if now - last[0] >= 20.0 or done == total:
            last[0] = now
            log(f"  {phase} {done}/{total}")
    ctx.set_progress(report)
    m_ini, m_fin = ctx.model(q.H_ini), ctx.model(q.H)
    sec = ctx.sector(14, q.n_up, q.n_dn)
    v0 = torch.from_numpy(wl.start_vector(sec.dim, q.gs_seed)).to("cuda:0")
    schedule = 1 if a.schedule == "sweep" else 0
    kw = dict(orbitals=q.orbitals, nt=q.nt, steps_per_grid=q.steps_per_grid, dt=q.dt,
              krylov_dim=q.krylov_dim, reorth=a.reorth, schedule=schedule, batch=a.batch, gs_tol=q.gs_tol)
    vec_steps = (q.nt - 1) * q.steps_per_grid + 2 * q.steps_per_grid * q.nt * (q.nt - 1) // 2

    for w in range(a.warmup):
        log(f"warmup {w + 1}/{a.warmup}")
        ctx.greens_neq(m_ini, m_fin, sec, v0, **kw)
    torch.cuda.synchronize()
    log(f"timed: {a.steps} step(s) of {vec_steps} vector-steps each")
    ctx.profile_begin(a.profile_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for s in range(a.steps):
        out = ctx.greens_neq(m_ini, m_fin, sec, v0, **kw)
        log(f"step {s + 1}/{a.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = ctx.profile_end()
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / a.steps

    # anticommutator on the equal-time diagonal as a cheap live sanity check
    Gl, Gg = out["G_lesser"][:, :, 0, 0], out["G_greater"][:, :, 0, 0]
    anti = float(np.abs(np.diag(Gg - Gl) + 1j).max())

    roofline, kernels = roofline_of(stats)
    cpu = None if a.no_cpu_baseline else cpu_baseline(q)
    res = {
        "metric": "G(t,t') contour steps/s at L=14 (four-step, Lanczos-fused H.v GB/s in roofline)",
        "value": round(vec_steps * a.steps / elapsed, 2),
        "unit": "vector-steps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOAD_14,
                   "D": sec.dim, "nt": q.nt, "krylov_dim": q.krylov_dim, "schedule": a.schedule,
                   "step": "one whole four-step run",
                   "vector_steps_per_step": vec_steps, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "E0": out["E0"],
        "anticommutator_err": anti,
        "kernels": kernels,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
