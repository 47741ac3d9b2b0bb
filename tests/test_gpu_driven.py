"""Driven Hamiltonians through the C ABI: kgf_model_set_params (parameters
replaced in place, tables kept, on-site energies recomputed) and
kgf_propagate_driven (fourth-order commutator-free integrator, each stage
one SIL step) against the oracle's same integrator with SIL stages."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say, to_dev, to_host
from oracle import basis, driven, hamiltonian
from oracle.gradients import model_with_theta, theta_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    return k.Context(0)


def test_set_params_replaces_parameters_in_place(ctx):
    A = wl.ring(8, 1.0, 4.0)
    rng = np.random.default_rng(12)
    nb, L = len(A.bonds), A.L
    thB = np.concatenate([rng.uniform(0.5, 1.5, nb), rng.uniform(-1, 1, L), rng.uniform(-1, 1, L),
                          rng.uniform(0, 3, L)])
    B = model_with_theta(A, thB)
    s = ctx.sector(8, 4, 3)
    sec = basis.Sector(8, 4, 3)
    X = np.stack([wl.complex_vector(sec.dim, 70 + c) for c in range(2)])
    m = ctx.model(A)
    ctx.apply_h(m, s, to_dev(X))                       # builds the tables with A
    say("set_params")
    m.set_params(thB[:nb], thB[nb:nb + L], thB[nb + L:nb + 2 * L], thB[nb + 2 * L:])
    got = to_host(ctx.apply_h(m, s, to_dev(X)))
    fresh = to_host(ctx.apply_h(ctx.model(B), s, to_dev(X)))
    HB = hamiltonian.Hamiltonian(B, sec)
    ref = np.stack([HB.apply(X[c]) for c in range(2)])
    assert rel_err(got, ref) < 1e-13
    assert np.array_equal(got, fresh)
    np.testing.assert_array_equal(m.theta, thB)
    with pytest.raises(ValueError):
        m.set_params(thB[:nb - 1], thB[nb:nb + L], thB[nb + L:nb + 2 * L], thB[nb + 2 * L:])


def _drive_case(name):
    if name == "ring8_hopping_and_field":
        H0 = wl.ring(8, 1.0, 4.0)
        nb, L = len(H0.bonds), H0.L
        k0 = np.zeros(nb + 3 * L)
        k0[0] = 1.0                                    # hopping on bond 0
        fld = np.zeros(nb + 3 * L)
        fld[nb + 0], fld[nb + L + 0] = -1.0, 1.0       # -h (n_up - n_dn) on site 0
        return H0, (4, 4), [theta_of(H0), k0, fld], (lambda t: [1.0, 0.8 * np.sin(2.0 * t), 0.3 * np.cos(t)]), \
            0.05, 20, 2
    H0 = wl.siam10().H                                  # star, U on the impurity only
    nb, L = len(H0.bonds), H0.L
    fld = np.zeros(nb + 3 * L)
    fld[nb + 0], fld[nb + L + 0] = -1.0, 1.0
    return H0, (5, 5), [theta_of(H0), fld], (lambda t: [1.0, 2.0 * np.exp(-t)]), 0.1, 10, 1


@pytest.mark.parametrize("name", ["ring8_hopping_and_field", "siam10_decaying_field"])
def test_propagate_driven_against_oracle(ctx, name):
    H0, (nu, nd), thetas, f, h, n, nvec = _drive_case(name)
    sec = basis.Sector(H0.L, nu, nd)
    X = np.stack([wl.complex_vector(sec.dim, 80 + c) for c in range(nvec)])
    say("driven oracle", name)
    ref = np.stack([driven.cfm4(H0, sec, thetas, f, X[c], 0.2, h, n, m=15, reorth="cgs2") for c in range(nvec)])
    say("driven GPU", name)
    work = ctx.model(H0)
    got = to_host(ctx.propagate_driven(work, ctx.sector(H0.L, nu, nd), to_dev(X), thetas, f, n, h, t0=0.2,
                                       krylov_dim=15, reorth=2))
    err = rel_err(got, ref)
    say("rel err", err)
    assert err < 1e-12
    assert np.abs(np.linalg.norm(got, axis=1) - np.linalg.norm(X, axis=1)).max() < 1e-12
    # the work model holds the last stage's parameters, on the host and on the device
    t_last = 0.2 + (n - 1) * h
    _, th2 = driven.stage_thetas(np.asarray(thetas), f, t_last, h)
    np.testing.assert_allclose(work.theta, th2, rtol=1e-13, atol=1e-14)
    v = wl.complex_vector(sec.dim, 90)
    Hl = hamiltonian.Hamiltonian(model_with_theta(H0, th2), sec)
    assert rel_err(to_host(ctx.apply_h(work, ctx.sector(H0.L, nu, nd), to_dev(v))), Hl.apply(v)) < 1e-13


def _ring8_drive():
    H = wl.ring(8, 1.0, 4.0)
    nb, L = len(H.bonds), H.L
    k0 = np.zeros(nb + 3 * L)
    k0[0] = 1.0
    fld = np.zeros(nb + 3 * L)
    fld[nb], fld[nb + L] = -1.0, 1.0
    return H.with_field(0, 0.3), H, [theta_of(H), k0, fld], (lambda t: [1.0, 0.8 * np.sin(2.0 * t), 0.3 * np.cos(t)])


@pytest.fixture(scope="module")
def driven_four_step_oracle():
    Hi, H, thetas, f = _ring8_drive()
    sec = basis.Sector(8, 4, 4)
    v0 = wl.start_vector(sec.dim, 7)
    say("driven four-step oracle")
    return driven.four_step(Hi, H, thetas, f, 4, 4, [(0, 0), (1, 0), (2, 1)], 5, 0.2, 2, 15, v0, gs_tol=1e-12)


@pytest.mark.parametrize("batch", [0, 2])
def test_greens_neq_driven_against_oracle(ctx, driven_four_step_oracle, batch):
    """Four-step G^<, G^> under a driven hopping and field on the half-filled
    8-site ring (D = 4900, nt = 5, two steps per mesh interval) against the
    oracle's plain schedule; batch = 2 splits each sweep into one mesh time
    per block."""
    Hi, H, thetas, f = _ring8_drive()
    ora = driven_four_step_oracle
    s = ctx.sector(8, 4, 4)
    v0 = to_dev(wl.start_vector(s.dim, 7))
    say("driven four-step GPU, batch", batch)
    work = ctx.model(H)
    got = ctx.greens_neq_driven(ctx.model(Hi), work, s, v0, [(0, 0), (1, 0), (2, 1)], thetas, f, nt=5,
                                steps_per_grid=2, dt=0.1, krylov_dim=15, reorth=2, batch=batch, gs_tol=1e-12)
    assert abs(got["E0"] - ora["E0"]) <= 1e-12 * abs(ora["E0"])
    for key in ("G_lesser", "G_greater"):
        e = rel_err(got[key], ora[key])
        say(key, "rel err", e)
        assert e < 1e-10, key
    # zero between orbitals of different spin
    assert not got["G_lesser"][:, :, 2, :2].any() and not got["G_greater"][:, :, :2, 2].any()
    with pytest.raises(ValueError):
        ctx.greens_neq_driven(work, work, s, v0, [(0, 0)], thetas, f, nt=2, steps_per_grid=1, dt=0.1)
