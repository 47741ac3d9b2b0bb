"""Captured SIL steps (KGF_OPT_GRAPHS): a recurring batched step is replayed
from a hipGraph.  Every replay must give bitwise the eager result, also
with other eager work and synchronisations between replays, when the
model's parameters change between steps (driven propagation: the captured
step must not be reused), and inside the four-step sweep and the batched
uneven instances."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import say, to_dev, to_host

pytestmark = pytest.mark.gpu

GRAPHS = 8


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    c = k.Context(0)
    yield c
    c.set_option(GRAPHS, 0)


def _eager_then_graph(ctx, fn):
    ctx.set_option(GRAPHS, 0)
    ref = fn()
    ctx.set_option(GRAPHS, 1)
    got = fn()
    return ref, got


def test_replays_equal_eager_with_work_between(ctx):
    import torch
    q = wl.ring8()
    s = ctx.sector(8, 4, 4)
    m = ctx.model(q.H)
    X = np.stack([wl.complex_vector(s.dim, 60 + c) for c in range(3)])
    ctx.set_option(GRAPHS, 0)
    ref = [to_host(ctx.propagate(m, s, to_dev(X), n, 0.05, 15, +1)) for n in (1, 2, 3, 6)]
    ctx.set_option(GRAPHS, 1)
    buf = to_dev(X)
    other = to_dev(X[0])
    for rep in range(3):
        for n, r in zip((1, 2, 3, 6), ref):
            buf.copy_(to_dev(X))
            ctx.propagate(m, s, buf, n, 0.05, 15, +1)             # steps 2.. of a key replay a graph
            y = ctx.apply_h(m, s, other)                           # eager work between replays
            torch.cuda.synchronize()
            assert np.array_equal(to_host(buf), r), (rep, n)
            assert np.isfinite(to_host(y)).all()


def test_reorthogonalised_and_imaginary_time_steps(ctx):
    q = wl.siam10()
    s = ctx.sector(10, 5, 5)
    m = ctx.model(q.H_ini)
    X = np.stack([wl.complex_vector(s.dim, 70 + c) for c in range(2)])
    for kw in (dict(direction=-1, reorth=2), dict(direction=0, shift=-3.0, reorth=1)):
        ref, got = _eager_then_graph(ctx, lambda: to_host(ctx.propagate(m, s, to_dev(X), 4, 0.05, 12, **kw)))
        assert np.array_equal(got, ref), kw


def test_driven_steps_do_not_reuse_stale_parameters(ctx):
    H0 = wl.ring8().H
    nb, L = len(H0.bonds), H0.L
    th0 = np.concatenate([np.asarray(H0.t, float), np.asarray(H0.eps_up, float), np.asarray(H0.eps_dn, float),
                          np.asarray(H0.U, float)])
    k1 = np.zeros(nb + 3 * L)
    k1[0] = 1.0
    f = lambda t: [1.0, 0.8 * np.sin(2.0 * t)]
    s = ctx.sector(8, 4, 4)
    x = np.stack([wl.complex_vector(s.dim, 80 + c) for c in range(2)])

    def run():
        work = ctx.model(H0)
        return to_host(ctx.propagate_driven(work, s, to_dev(x), [th0, k1], f, 5, 0.05, krylov_dim=12))
    ref, got = _eager_then_graph(ctx, run)
    assert np.array_equal(got, ref)


def test_four_step_sweep_and_uneven_batch(ctx):
    H = wl.chain_siam(6, 2.0)
    Hi = H.with_field(0, 0.4)
    s = ctx.sector(6, 3, 3)
    v0 = to_dev(wl.start_vector(s.dim, 7))
    orbs = [(0, 0), (1, 1)]
    say("graphs: four-step sweep")
    ref, got = _eager_then_graph(ctx, lambda: ctx.greens_neq(ctx.model(Hi), ctx.model(H), s, v0, orbs, nt=6,
                                                             steps_per_grid=2, dt=0.1, krylov_dim=12, batch=3))
    for key in ("G_lesser", "G_greater"):
        assert np.array_equal(got[key], ref[key]), key
    say("graphs: uneven batch")
    qs = wl.batch_instances()[:6]
    secs = [ctx.sector(q.H.L, q.n_up, q.n_dn) for q in qs]
    v0s = [to_dev(wl.start_vector(sc.dim, 7)) for sc in secs]
    q0 = qs[0]

    def multi():
        return ctx.greens_neq_multi([ctx.model(q.H_ini) for q in qs], [ctx.model(q.H) for q in qs], secs, v0s,
                                    q0.orbitals, nt=4, steps_per_grid=q0.steps_per_grid, dt=q0.dt,
                                    krylov_dim=q0.krylov_dim)
    ref, got = _eager_then_graph(ctx, multi)
    for key in ("G_lesser", "G_greater"):
        assert np.array_equal(got[key], ref[key]), key
