"""Uneven batch of Anderson instances (64 stars, L drawn from 8..12, quench
U 0 -> 4; G_imp on a 50 x 50 mesh) through kgf_greens_neq_multi, where all
instances of one L run as one multi-column batch with per-column
Hamiltonians.

* batched == per instance (kgf_greens_neq) to rounding, on a short mesh and
  on sampled instances of the full workload;
* the two L = 8 instances of the workload on the full 50 x 50 mesh against
  the oracle's four-step (bar 1e-10 relative to max|G|, the parity tolerance for G);
* every instance of the full workload: equal-time anticommutator and
  Hermiticity."""
import time

import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say, to_dev
from oracle import basis, greens

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    return k.Context(0)


def _inputs(ctx, qs):
    Hi = [ctx.model(q.H_ini) for q in qs]
    Hf = [ctx.model(q.H) for q in qs]
    secs = [ctx.sector(q.H.L, q.n_up, q.n_dn) for q in qs]
    v0 = [to_dev(wl.start_vector(s.dim, 7)) for s in secs]
    return Hi, Hf, secs, v0


def test_multi_equals_per_instance_short_mesh(ctx):
    qs = wl.batch_instances()[:10]
    say("multi vs single, L =", [q.H.L for q in qs])
    Hi, Hf, secs, v0 = _inputs(ctx, qs)
    kw = dict(orbitals=[(0, 0), (0, 1)], nt=6, steps_per_grid=2, dt=0.05, krylov_dim=15)
    out = ctx.greens_neq_multi(Hi, Hf, secs, v0, **kw)
    for i, q in enumerate(qs):
        ref = ctx.greens_neq(Hi[i], Hf[i], secs[i], v0[i], schedule=1, **kw)
        assert abs(out["E0"][i] - ref["E0"]) <= 1e-13 * abs(ref["E0"])
        assert rel_err(out["G_lesser"][i], ref["G_lesser"]) < 1e-12
        assert rel_err(out["G_greater"][i], ref["G_greater"]) < 1e-12


@pytest.mark.parametrize("batch", [0, 7])
def test_lockstep_equals_group_by_group(ctx, batch):
    """All groups (L = 8..12) advancing together, each SIL kernel one launch
    over every group's columns, equal the group-by-group batches bitwise;
    batch = 7 cuts the sweeps into several chunks of source times."""
    qs = wl.batch_instances()[:12]
    say("lockstep vs group by group, L =", sorted({q.H.L for q in qs}), "batch", batch)
    Hi, Hf, secs, v0 = _inputs(ctx, qs)
    kw = dict(orbitals=[(0, 0), (1, 1)], nt=5, steps_per_grid=2, dt=0.05, krylov_dim=12, batch=batch)
    LOCKSTEP = 9
    ctx.set_option(LOCKSTEP, 0)
    try:
        ref = ctx.greens_neq_multi(Hi, Hf, secs, v0, **kw)
    finally:
        ctx.set_option(LOCKSTEP, 1)
    got = ctx.greens_neq_multi(Hi, Hf, secs, v0, **kw)
    assert np.array_equal(got["E0"], ref["E0"])
    for key in ("G_lesser", "G_greater"):
        assert np.array_equal(got[key], ref[key]), key


def test_multi_l8_instances_full_mesh_against_oracle(ctx):
    qs = [q for q in wl.batch_instances() if q.H.L == 8][:2]
    assert len(qs) == 2
    say("L=8 instances full mesh:", [q.name for q in qs])
    Hi, Hf, secs, v0 = _inputs(ctx, qs)
    q0 = qs[0]
    out = ctx.greens_neq_multi(Hi, Hf, secs, v0, orbitals=q0.orbitals, nt=q0.nt, steps_per_grid=q0.steps_per_grid,
                               dt=q0.dt, krylov_dim=q0.krylov_dim)
    for i, q in enumerate(qs):
        say("oracle", q.name)
        o = greens.four_step(q.H_ini, q.H, q.n_up, q.n_dn, list(q.orbitals), q.nt, q.dt_grid, q.steps_per_grid,
                             q.krylov_dim, wl.start_vector(basis.Sector(q.H.L, q.n_up, q.n_dn).dim, 7),
                             gs_tol=1e-12, reorth="none")
        assert abs(out["E0"][i] - o["E0"]) <= 1e-12 * abs(o["E0"])
        assert rel_err(out["G_lesser"][i], o["G_lesser"]) < 1e-10
        assert rel_err(out["G_greater"][i], o["G_greater"]) < 1e-10


def test_full_uneven_batch(ctx):
    qs = wl.batch_instances()
    Ls = [q.H.L for q in qs]
    say("64 instances, L counts:", {L: Ls.count(L) for L in sorted(set(Ls))})
    Hi, Hf, secs, v0 = _inputs(ctx, qs)
    q0 = qs[0]
    kw = dict(orbitals=q0.orbitals, nt=q0.nt, steps_per_grid=q0.steps_per_grid, dt=q0.dt, krylov_dim=q0.krylov_dim)
    last = [time.perf_counter()]

    def report(ph, d, t):
        now = time.perf_counter()
        if d == t or now - last[0] > 20.0:
            last[0] = now
            say("  ", ph, d, t)
    ctx.set_progress(report)
    t0 = time.perf_counter()
    try:
        out = ctx.greens_neq_multi(Hi, Hf, secs, v0, **kw)
    finally:
        ctx.set_progress(None)
    say("batched forward of 64 instances: %.1f s" % (time.perf_counter() - t0))
    Gl, Gg = out["G_lesser"][:, :, :, 0, 0], out["G_greater"][:, :, :, 0, 0]
    for i in range(len(qs)):
        assert np.abs(np.diagonal(Gg[i] - Gl[i]) + 1j).max() < 1e-10, qs[i].name
        assert np.abs(Gl[i] + Gl[i].conj().T).max() < 1e-10
        assert np.abs(Gg[i] + Gg[i].conj().T).max() < 1e-10
    for L in (12, 10):
        i = Ls.index(L)
        say("per-instance check", qs[i].name)
        ref = ctx.greens_neq(Hi[i], Hf[i], secs[i], v0[i], schedule=1, **kw)
        assert rel_err(out["G_lesser"][i], ref["G_lesser"]) < 1e-12
        assert rel_err(out["G_greater"][i], ref["G_greater"]) < 1e-12


def test_batched_adjoint_equals_per_instance(ctx):
    """kgf_greens_neq_vjp_multi (two L = 8, two L = 9 and one L = 10 instance;
    same-L instances batched) against kgf_greens_neq_vjp instance by
    instance, seeded complex cotangents on G^< and G^>."""
    allq = wl.batch_instances()
    qs = [q for q in allq if q.H.L == 8][:2] + [q for q in allq if q.H.L == 9][:2] + [q for q in allq if q.H.L == 10][:1]
    say("batched adjoint:", [q.name for q in qs])
    Hi, Hf, secs, v0 = _inputs(ctx, qs)
    nt, spg, dt = 4, 2, 0.05
    rng = np.random.default_rng(5)
    Wl = [rng.standard_normal((nt, nt, 1, 1)) + 1j * rng.standard_normal((nt, nt, 1, 1)) for _ in qs]
    Wg = [rng.standard_normal((nt, nt, 1, 1)) + 1j * rng.standard_normal((nt, nt, 1, 1)) for _ in qs]
    kw = dict(krylov_dim=15, quad_nodes=8, cg_tol=1e-12)
    res = ctx.greens_neq_vjp_multi(Hi, Hf, secs, v0, [(0, 0)], nt, spg, dt, Wl, Wg, **kw)
    for i, q in enumerate(qs):
        ref = ctx.greens_neq_vjp(Hi[i], Hf[i], secs[i], v0[i], [(0, 0)], nt, spg, dt, Wl[i], Wg[i], **kw)
        assert res[i]["E0"] == ref["E0"]
        sc = max(np.abs(ref["grad"]).max(), np.abs(ref["grad_ini"]).max())
        assert np.abs(res[i]["grad"] - ref["grad"]).max() <= 1e-12 * sc, q.name
        assert np.abs(res[i]["grad_ini"] - ref["grad_ini"]).max() <= 1e-12 * sc, q.name
