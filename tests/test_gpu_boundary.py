"""Boundary behaviour of the C ABI beyond the numerics of the path:

* uniqueness of the ground state (the method assumes a nondegenerate |0>,
  Sec. 2 and Sec. 4 step (i)): the half-filled 8-site ring at U = 0 has an
  open shell (single-particle levels -2, -sqrt2 (x2), 0 (x2), ...: four
  electrons per spin leave one of the two zero levels empty), so its (4, 4)
  ground state is degenerate and a second Lanczos start must report
  KGF_EDEGENERATE; at U = 4 the bipartite ring's ground state is unique
  (Lieb) and the fidelity of the two starts is 1 to 1e-10;
* the per-step a-posteriori error estimate of a SIL step (Sec. 3, Eq.
  (udelta)), the integral of the Krylov residual over the step, bounds the
  true error of the step (measured with the oracle's dense
  eigendecomposition of H, D = 4,900) and stays within a factor 10 of it;
* the projected CG of the adjoint's ground-state term reports KGF_ENOCONV
  when held below convergence from the host (iteration limit 1);
* the per-step norm drift | ||psi after|| / ||psi before|| - 1 | of SIL
  propagation: at rounding level for the unitary real-time steps (Sec. 3),
  and for the imaginary-time direction equal to the decay of the norm that
  the oracle's dense exponential gives (so the measurement itself is
  pinned)."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import say, to_dev, to_host
from oracle import basis, hamiltonian

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    c = k.Context(0)
    yield c
    c.set_option(c.CG_MAX_ITER, 0)


def test_degenerate_ground_state_reported(ctx):
    import paper_1109_1205_amd as k
    say("uniqueness: U=0 ring (degenerate)")
    H = wl.ring(8, 1.0, 0.0)
    s = ctx.sector(8, 4, 4)
    v0 = to_dev(wl.start_vector(s.dim, 7))
    m = ctx.model(H)
    E0, psi, info = ctx.ground_state(m, s, v0, tol=1e-12, max_iter=400)       # no check: no error
    assert info["converged"] and info["fidelity2"] == -1.0
    with pytest.raises(k.KgfError) as e:
        ctx.ground_state(m, s, v0, tol=1e-12, max_iter=400, unique_check=True)
    assert e.value.code == -6
    with pytest.raises(k.KgfError) as e:
        ctx.greens_neq(m, m, s, v0, [(0, 0)], nt=2, steps_per_grid=1, dt=0.05, gs_max_iter=400,
                       gs_unique_check=True)
    assert e.value.code == -6


def test_unique_ground_state_fidelity(ctx):
    say("uniqueness: U=4 ring (unique)")
    q = wl.ring8()
    s = ctx.sector(8, 4, 4)
    E0, psi, info = ctx.ground_state(ctx.model(q.H), s, to_dev(wl.start_vector(s.dim, 7)), tol=1e-12, max_iter=400,
                                     unique_check=True, unique_seed=8)
    assert info["converged"] and 1.0 - 1e-10 <= info["fidelity2"] <= 1.0 + 1e-10


@pytest.mark.parametrize("m", [6, 8, 10])
def test_sil_error_estimate_tracks_true_error(ctx, m):
    q = wl.ring8()
    sec = basis.Sector(8, 4, 4)
    H = hamiltonian.Hamiltonian(q.H, sec)
    lam, Q = np.linalg.eigh(H.dense())
    psi = wl.complex_vector(sec.dim, 40 + m)
    dt = 0.1
    exact = Q @ (np.exp(-1j * lam * dt) * (Q.conj().T @ psi))
    say("SIL error estimate m", m)
    got, est = ctx.propagate(ctx.model(q.H), ctx.sector(8, 4, 4), to_dev(psi), 1, dt, m, -1, return_err=True)
    true = float(np.linalg.norm(to_host(got) - exact))
    assert true > 1e-11, "case must be above rounding"
    assert true * (1.0 - 1e-6) <= est <= 10.0 * true, (est, true)
    _, est0 = ctx.propagate(ctx.model(q.H), ctx.sector(8, 4, 4), to_dev(psi), 0, dt, m, -1, return_err=True)
    assert est0 == 0.0


def test_adjoint_cg_failure_reported(ctx):
    import paper_1109_1205_amd as k
    H = wl.chain_siam(4, 2.0)
    Hi = H.with_field(0, 0.4)
    s = ctx.sector(4, 2, 2)
    v0 = to_dev(wl.start_vector(s.dim, 7))
    orbs = [(0, 0)]
    rng = np.random.default_rng(3)
    W = rng.standard_normal((3, 3, 1, 1)) + 1j * rng.standard_normal((3, 3, 1, 1))
    mi, mf = ctx.model(Hi), ctx.model(H)
    ok = ctx.greens_neq_vjp(mi, mf, s, v0, orbs, 3, 1, 0.1, W_lesser=W)
    assert ok["cg_iters"] > 1
    say("adjoint CG held to one iteration")
    ctx.set_option(ctx.CG_MAX_ITER, 1)
    try:
        with pytest.raises(k.KgfError) as e:
            ctx.greens_neq_vjp(mi, mf, s, v0, orbs, 3, 1, 0.1, W_lesser=W)
        assert e.value.code == -4
    finally:
        ctx.set_option(ctx.CG_MAX_ITER, 0)


def test_norm_drift_reported(ctx):
    q = wl.ring8()
    sec = basis.Sector(8, 4, 4)
    H = hamiltonian.Hamiltonian(q.H, sec)
    X = np.stack([wl.complex_vector(sec.dim, 50 + c) for c in range(2)])
    say("norm drift: real-time steps")
    got, est, drift = ctx.propagate(ctx.model(q.H), ctx.sector(8, 4, 4), to_dev(X), 3, 0.05, 15, -1,
                                    return_err=True, return_drift=True)
    assert 0.0 <= drift < 1e-13 and est > 0.0
    _, drift0 = ctx.propagate(ctx.model(q.H), ctx.sector(8, 4, 4), to_dev(X), 0, 0.05, 15, -1, return_drift=True)
    assert drift0 == 0.0
    say("norm drift: imaginary-time step against the dense exponential")
    lam, Q = np.linalg.eigh(H.dense())
    shift, dt = float(lam[0]) + 1.0, 0.05
    ratio = []
    for c in range(2):
        y = Q @ (np.exp(-(lam - shift) * dt) * (Q.conj().T @ X[c]))
        ratio.append(abs(np.linalg.norm(y) / np.linalg.norm(X[c]) - 1.0))
    _, drift_im = ctx.propagate(ctx.model(q.H), ctx.sector(8, 4, 4), to_dev(X), 1, dt, 15, 0, shift,
                                return_drift=True)
    assert max(ratio) > 1e-3
    assert abs(drift_im - max(ratio)) <= 1e-10 * max(ratio)
