"""Adjoint (reverse mode) of the HIP path vs the CPU oracle.

* <lam| dH/dtheta |psi>: H is linear in theta = (t_b, eps_up, eps_dn, U), so
  the oracle evaluates it exactly as <lam| H(e_theta) |psi> with a one-hot
  parameter vector.
* Gradients of propagation and of the four-step G: central finite
  differences of the oracle's forward computation (bar: 1e-6 relative to
  the largest gradient component)."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say, to_dev, to_host
from oracle import basis, greens, hamiltonian, propagate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    return k.Context(0)


def theta_of(model):
    bonds, t, eu, ed, U = model.arrays()
    return np.concatenate([t, eu, ed, U])


def model_with(model, theta):
    nb, L = len(model.bonds), model.L
    return wl.Model(L=L, bonds=model.bonds, t=tuple(theta[:nb]), eps_up=tuple(theta[nb:nb + L]),
                    eps_dn=tuple(theta[nb + L:nb + 2 * L]), U=tuple(theta[nb + 2 * L:]), name=model.name)


MODELS = {
    "chain6_field": (lambda: wl.chain_siam(6, 2.0).with_field(0, 0.3), 3, 2),
    "star8": (lambda: wl.star_siam([0.3, -0.5, 1.1, 0.2, -1.4, 0.7, -0.1],
                                   [0.4, 0.2, -0.3, 0.3, 0.25, -0.35, 0.15], 3.0, -1.5), 4, 4),
    "rect3x2_tp": (lambda: wl.rect(3, 2, 1.0, -0.3, 4.0).with_field(2, 0.2), 3, 3),
}


@pytest.mark.parametrize("name", list(MODELS))
def test_dH_expect_parity(ctx, name):
    mk, nu, nd = MODELS[name]
    model = mk()
    say("dH", name)
    sec = basis.Sector(model.L, nu, nd)
    lam = np.stack([wl.complex_vector(sec.dim, 50 + p) for p in range(2)])
    psi = np.stack([wl.complex_vector(sec.dim, 60 + p) for p in range(2)])
    w = np.array([0.7 - 0.2j, -1.3 + 0.4j])
    th = theta_of(model)
    ref = np.zeros(len(th))
    for i in range(len(th)):
        e = np.zeros(len(th))
        e[i] = 1.0
        H = hamiltonian.Hamiltonian(model_with(model, e), sec)
        ref[i] = sum((w[p] * np.vdot(lam[p], H.apply(psi[p]))).real for p in range(2))
    got = ctx.dH_expect(ctx.model(model), ctx.sector(model.L, nu, nd), to_dev(lam), to_dev(psi), w)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("direction", [-1, +1])
def test_propagate_vjp_against_finite_differences(ctx, direction):
    """L = Re <chi| U^n psi0> for n SIL steps: dL/dtheta by the adjoint vs
    central differences of the oracle propagation; dL/dpsi0* vs U^+ chi / 2."""
    say("propagate vjp", direction)
    model = wl.chain_siam(6, 2.0).with_field(0, 0.3)
    nu, nd = 3, 2
    sec = basis.Sector(model.L, nu, nd)
    psi0 = wl.complex_vector(sec.dim, 3)
    chi = wl.complex_vector(sec.dim, 4)
    n, dt, m = 4, 0.1, 15

    def loss(theta):
        H = hamiltonian.Hamiltonian(model_with(model, theta), sec)
        x = propagate.propagate(H.apply, psi0, dt, n, m, direction, reorth="cgs2")
        return np.vdot(chi, x).real

    th = theta_of(model)
    h = 1e-5
    fd = np.array([(loss(th + h * np.eye(len(th))[i]) - loss(th - h * np.eye(len(th))[i])) / (2 * h)
                   for i in range(len(th))])
    lam = to_dev(0.5 * chi)
    g = ctx.propagate_vjp(ctx.model(model), ctx.sector(model.L, nu, nd), to_dev(psi0), lam, n, dt, m,
                          direction, reorth=2, quad_nodes=10)
    assert np.abs(g - fd).max() <= 1e-6 * np.abs(fd).max()
    H = hamiltonian.Hamiltonian(model, sec)
    ref = propagate.propagate(H.apply, 0.5 * chi, dt, n, m, -direction, reorth="cgs2")
    assert rel_err(to_host(lam), ref) < 1e-12


def _fd_four_step(H_ini, H, nu, nd, orbs, nt, dtg, spg, m, v0, Wl, Wg, which, h=1e-5):
    def loss(model_ini, model_fin):
        o = greens.four_step(model_ini, model_fin, nu, nd, orbs, nt, dtg, spg, m, v0, gs_tol=1e-13,
                             gs_max_iter=600, reorth="cgs2")
        return (np.sum(np.conj(Wl) * o["G_lesser"]) + np.sum(np.conj(Wg) * o["G_greater"])).real
    base = H_ini if which == "ini" else H
    th = theta_of(base)
    out = np.zeros(len(th))
    for i in range(len(th)):
        e = np.zeros(len(th))
        e[i] = h
        mp, mm = model_with(base, th + e), model_with(base, th - e)
        if which == "ini":
            out[i] = (loss(mp, H) - loss(mm, H)) / (2 * h)
        else:
            out[i] = (loss(H_ini, mp) - loss(H_ini, mm)) / (2 * h)
    return out


def test_greens_neq_vjp_against_finite_differences(ctx):
    """Four-step G^< and G^> of a small Anderson chain quench (field and
    bath-coupling change), orbitals of both spins, random complex
    cotangents: adjoint gradient w.r.t. every parameter of H and of H_ini
    vs central differences of the oracle's four-step."""
    say("four-step vjp")
    H = wl.chain_siam(5, 2.0)
    H_ini = model_with(H.with_field(0, 0.4), theta_of(H.with_field(0, 0.4)) * np.r_[[1.1, 0.9, 1.0, 1.05],
                                                                                     np.ones(15)])
    nu, nd = 3, 2
    orbs = [(0, 0), (2, 0), (1, 1)]
    nt, spg, dtg, m = 4, 2, 0.2, 14
    sec = basis.Sector(5, nu, nd)
    v0 = wl.start_vector(sec.dim, 7)
    rng = np.random.default_rng(5)
    shape = (nt, nt, len(orbs), len(orbs))
    Wl = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    Wg = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    got = ctx.greens_neq_vjp(ctx.model(H_ini), ctx.model(H), ctx.sector(5, nu, nd), to_dev(v0), orbs, nt, spg,
                             dtg / spg, Wl, Wg, krylov_dim=m, reorth=2, quad_nodes=10, cg_tol=1e-13, gs_tol=1e-13)
    fwd = greens.four_step(H_ini, H, nu, nd, orbs, nt, dtg, spg, m, v0, gs_tol=1e-13, reorth="cgs2")
    assert rel_err(got["G_lesser"], fwd["G_lesser"]) < 1e-10
    assert rel_err(got["G_greater"], fwd["G_greater"]) < 1e-10
    fd = _fd_four_step(H_ini, H, nu, nd, orbs, nt, dtg, spg, m, v0, Wl, Wg, "fin")
    say("grad H max err", np.abs(got["grad"] - fd).max(), "scale", np.abs(fd).max())
    assert np.abs(got["grad"] - fd).max() <= 1e-6 * np.abs(fd).max()
    fdi = _fd_four_step(H_ini, H, nu, nd, orbs, nt, dtg, spg, m, v0, Wl, Wg, "ini")
    say("grad H_ini max err", np.abs(got["grad_ini"] - fdi).max(), "scale", np.abs(fdi).max(), "cg", got["cg_iters"])
    assert np.abs(got["grad_ini"] - fdi).max() <= 1e-6 * np.abs(fdi).max()


def test_checkpointed_chains_are_bitwise_equal(ctx):
    """The adjoint with chain states kept as checkpoints (recomputed
    segments) returns exactly the gradient of the stored-chain adjoint."""
    say("adjoint checkpoints")
    model = wl.chain_siam(6, 2.0).with_field(0, 0.3)
    sec = basis.Sector(6, 3, 2)
    psi0 = to_dev(wl.complex_vector(sec.dim, 3))
    chi = wl.complex_vector(sec.dim, 4)
    outs = []
    for K in (0, 3, 1):
        ctx.set_option(ctx.ADJ_EVERY, K)
        try:
            lam = to_dev(0.5 * chi)
            g = ctx.propagate_vjp(ctx.model(model), ctx.sector(6, 3, 2), psi0, lam, 7, 0.1, 15, -1, reorth=2,
                                  quad_nodes=10)
            outs.append((g, to_host(lam)))
        finally:
            ctx.set_option(ctx.ADJ_EVERY, 0)
    for g, lam in outs[1:]:
        assert np.array_equal(g, outs[0][0]) and np.array_equal(lam, outs[0][1])
    H = wl.chain_siam(5, 2.0)
    Hi = H.with_field(0, 0.4)
    sec5 = basis.Sector(5, 3, 2)
    v0 = to_dev(wl.start_vector(sec5.dim, 7))
    rng = np.random.default_rng(5)
    W = rng.standard_normal((5, 5, 1, 1)) + 1j * rng.standard_normal((5, 5, 1, 1))
    res = []
    for K in (0, 2):
        ctx.set_option(ctx.ADJ_EVERY, K)
        try:
            res.append(ctx.greens_neq_vjp(ctx.model(Hi), ctx.model(H), ctx.sector(5, 3, 2), v0, [(0, 0)], 5, 3, 0.05,
                                          W, W.conj(), krylov_dim=14, quad_nodes=8))
        finally:
            ctx.set_option(ctx.ADJ_EVERY, 0)
    assert np.array_equal(res[0]["grad"], res[1]["grad"])
    assert np.array_equal(res[0]["grad_ini"], res[1]["grad_ini"])


def test_ladder16_hopping_gradient_short_mesh(ctx):
    """2x8 ladder quench (L = 16, D = 165,636,900), G^< and G^> of site 0 on a
    3-point mesh, loss Re sum conj(W) G with a seeded complex Gaussian W
    (seed 5); the 22 bond hoppings are shared by H_ini (U = 4) and H (U = 8),
    so dL/dt_b = grad[b] + grad_ini[b].  Checked against central differences
    of the GPU forward pass for two bonds (a leg and a rung), chains
    checkpointed every step."""
    import torch
    q = wl.ladder16()
    s = ctx.sector(16, 8, 8)
    say("ladder16 gradient: start vector")
    v0 = torch.from_numpy(wl.start_vector(s.dim, 7)).to("cuda:0")
    nt = 3
    rng = np.random.default_rng(5)
    Wl = rng.standard_normal((nt, nt, 1, 1)) + 1j * rng.standard_normal((nt, nt, 1, 1))
    Wg = rng.standard_normal((nt, nt, 1, 1)) + 1j * rng.standard_normal((nt, nt, 1, 1))
    kw = dict(krylov_dim=20, gs_tol=1e-13, gs_max_iter=2000)
    ctx.set_option(ctx.ADJ_EVERY, 1)
    ctx.set_progress(lambda ph, d, t: say("  ", ph, d, t) if d == t else None)
    try:
        r = ctx.greens_neq_vjp(ctx.model(q.H_ini), ctx.model(q.H), s, v0, [(0, 0)], nt, 1, q.dt, Wl, Wg,
                               quad_nodes=12, cg_tol=1e-12, **kw)
    finally:
        ctx.set_option(ctx.ADJ_EVERY, 0)
        ctx.set_progress(None)
    nb = len(q.H.bonds)
    g_t = r["grad"][:nb] + r["grad_ini"][:nb]
    say("grad norm", np.linalg.norm(g_t), "cg", r["cg_iters"])

    def loss(b, h):
        def bump(m):
            t = list(m.t)
            t[b] += h
            return wl.Model(L=m.L, bonds=m.bonds, t=tuple(t), eps_up=m.eps_up, eps_dn=m.eps_dn, U=m.U, name=m.name)
        o = ctx.greens_neq(ctx.model(bump(q.H_ini)), ctx.model(bump(q.H)), s, v0, orbitals=[(0, 0)], nt=nt,
                           steps_per_grid=1, dt=q.dt, schedule=0, **kw)
        return float((np.sum(np.conj(Wl) * o["G_lesser"]) + np.sum(np.conj(Wg) * o["G_greater"])).real)
    legs = [b for b, (i, j) in enumerate(q.H.bonds) if j - i == 2]
    rungs = [b for b, (i, j) in enumerate(q.H.bonds) if j - i == 1]
    for b in (legs[0], rungs[0]):
        h = 1e-4
        fd = (loss(b, h) - loss(b, -h)) / (2 * h)
        say("bond", q.H.bonds[b], "adjoint", g_t[b], "fd", fd)
        assert abs(g_t[b] - fd) <= 1e-6 * max(1.0, np.abs(g_t).max())


@pytest.mark.parametrize("direction", [-1, +1])
def test_propagate_vjp_against_dense_frechet_gradient(ctx, direction):
    """Adjoint of n SIL steps vs the exact gradient of exp(direction i H n dt)
    (Frechet derivative of the matrix exponential)."""
    from oracle import gradients
    model = wl.chain_siam(6, 2.0).with_field(0, 0.3)
    sec = basis.Sector(6, 3, 2)
    psi0, chi = wl.complex_vector(sec.dim, 3), wl.complex_vector(sec.dim, 4)
    n, dt, m = 5, 0.1, 15
    ref = gradients.propagation_gradient(model, sec, psi0, chi, n * dt, direction)
    lam = to_dev(0.5 * chi)
    g = ctx.propagate_vjp(ctx.model(model), ctx.sector(6, 3, 2), to_dev(psi0), lam, n, dt, m, direction, reorth=2,
                          quad_nodes=10)
    say("propagate vjp vs dense", np.abs(g - ref).max(), np.abs(ref).max())
    assert np.abs(g - ref).max() <= 1e-9 * np.abs(ref).max()


def test_greens_neq_vjp_against_dense_gradient(ctx):
    """Four-step gradient (H and H_ini, orbitals of both spins) vs the exact
    dense gradient: Frechet derivatives of every exponential and the
    sum-over-states ground-state derivative."""
    from oracle import gradients
    H = wl.chain_siam(4, 2.0)
    Hi = gradients.model_with_theta(H.with_field(0, 0.4), gradients.theta_of(H.with_field(0, 0.4)) * 1.03)
    orbs = [(0, 0), (1, 1)]
    nt, spg, dt = 3, 3, 0.1
    times = [k * spg * dt for k in range(nt)]
    rng = np.random.default_rng(3)
    shape = (nt, nt, 2, 2)
    Wl = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    Wg = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    gi_ref, g_ref, G = gradients.four_step_gradient(Hi, H, 2, 2, orbs, times, Wl, Wg)
    sec = basis.Sector(4, 2, 2)
    r = ctx.greens_neq_vjp(ctx.model(Hi), ctx.model(H), ctx.sector(4, 2, 2), to_dev(wl.start_vector(sec.dim, 7)),
                           orbs, nt, spg, dt, Wl, Wg, krylov_dim=14, reorth=2, quad_nodes=10, cg_tol=1e-13,
                           gs_tol=1e-13)
    sc = max(np.abs(g_ref).max(), np.abs(gi_ref).max())
    say("four-step vjp vs dense", np.abs(r["grad"] - g_ref).max(), np.abs(r["grad_ini"] - gi_ref).max(), sc)
    assert rel_err(r["G_lesser"], G["G_lesser"]) < 1e-10
    assert np.abs(r["grad"] - g_ref).max() <= 1e-8 * sc
    assert np.abs(r["grad_ini"] - gi_ref).max() <= 1e-8 * sc
