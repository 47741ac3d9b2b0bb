"""Run-to-run reproducibility: every reduction of the path (Lanczos a_k and
b_k, norms, Gram-Schmidt dots, the step (iv) scalar products) writes one
partial per block and a one-block finaliser sums the partials in a fixed
order, so the same call on the same inputs gives bitwise the same result.
Checked for the ground state, batched SIL steps (with and without
reorthogonalisation), the four-step G on the sweep schedule with a ragged
block, the batched uneven instances and the adjoint gradient."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    return k.Context(0)


def twice(fn):
    a, b = fn(), fn()
    return a, b


def test_ground_state_and_sil_steps(ctx):
    q = wl.siam10()
    s = ctx.sector(10, 5, 5)
    m = ctx.model(q.H_ini)
    v0 = to_dev(wl.start_vector(s.dim, 7))
    say("determinism: ground state")
    (E1, p1, i1), (E2, p2, i2) = twice(lambda: ctx.ground_state(m, s, v0, tol=1e-12, max_iter=400))
    assert E1 == E2 and i1["iters"] == i2["iters"]
    assert np.array_equal(to_host(p1), to_host(p2))
    X = np.stack([wl.complex_vector(s.dim, 90 + c) for c in range(5)])
    for reorth in (0, 2):
        say("determinism: SIL steps, reorth", reorth)
        a, b = twice(lambda: to_host(ctx.propagate(m, s, to_dev(X), 3, 0.05, 15, +1, reorth=reorth)))
        assert np.array_equal(a, b), reorth


def test_four_step_and_uneven_batch(ctx):
    H = wl.chain_siam(6, 2.0)
    Hi = H.with_field(0, 0.4)
    s = ctx.sector(6, 3, 3)
    v0 = to_dev(wl.start_vector(s.dim, 7))
    orbs = [(0, 0), (2, 0), (1, 1)]
    say("determinism: four-step sweep, batch 4")
    a, b = twice(lambda: ctx.greens_neq(ctx.model(Hi), ctx.model(H), s, v0, orbs, nt=7, steps_per_grid=2, dt=0.1,
                                        krylov_dim=15, schedule=1, batch=4))
    for key in ("G_lesser", "G_greater", "E0"):
        assert np.array_equal(a[key], b[key]), key
    qs = wl.batch_instances()[:6]
    secs = [ctx.sector(q.H.L, q.n_up, q.n_dn) for q in qs]
    v0s = [to_dev(wl.start_vector(sc.dim, 7)) for sc in secs]
    q0 = qs[0]
    say("determinism: uneven batch of 6 instances")
    a, b = twice(lambda: ctx.greens_neq_multi([ctx.model(q.H_ini) for q in qs], [ctx.model(q.H) for q in qs], secs,
                                              v0s, q0.orbitals, nt=4, steps_per_grid=q0.steps_per_grid, dt=q0.dt,
                                              krylov_dim=q0.krylov_dim))
    for key in ("G_lesser", "G_greater"):
        assert np.array_equal(a[key], b[key]), key


def test_adjoint_gradient(ctx):
    H = wl.chain_siam(4, 2.0)
    Hi = H.with_field(0, 0.4)
    s = ctx.sector(4, 2, 2)
    v0 = to_dev(wl.start_vector(s.dim, 7))
    rng = np.random.default_rng(3)
    W = rng.standard_normal((4, 4, 1, 1)) + 1j * rng.standard_normal((4, 4, 1, 1))
    say("determinism: adjoint")
    a, b = twice(lambda: ctx.greens_neq_vjp(ctx.model(Hi), ctx.model(H), s, v0, [(0, 0)], 4, 2, 0.1, W_lesser=W))
    for key in ("grad", "grad_ini", "G_lesser"):
        assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), key
