"""torch.autograd over the four-step G (libkgf forward + adjoint) vs central
finite differences of the oracle's four-step, including a loss written in
terms of physical Anderson parameters (bath energies, hybridisations, U)
mapped to the per-bond / per-site parameter vector with torch ops, in the
spirit of the uneven-batch gradient workload (fit of G_imp(t,t') to a
target computed at a different U)."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import say, to_dev
from oracle import basis, greens

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    from paper_1109_1205_amd import autograd as ag
    return k, ag, k.Context(0)


def star_theta(torch, eps_b, V_b, U, eps_imp, L):
    """theta = (t_b = -V_k, eps_up, eps_dn, U_i) of a star Anderson model."""
    z1 = torch.zeros(1, dtype=torch.float64)
    eps = torch.cat([eps_imp.reshape(1), eps_b])
    Uv = torch.cat([U.reshape(1), torch.zeros(L - 1, dtype=torch.float64)])
    return torch.cat([-V_b, eps, eps, Uv])


@pytest.mark.parametrize("seed", [4000, 4003])
def test_anderson_fit_gradient(env, seed):
    import torch
    k, ag, ctx = env
    rng = np.random.default_rng(seed)
    L = 5
    eb = rng.uniform(-2.0, 2.0, L - 1)
    Vb = 0.3 + 0.1 * rng.standard_normal(L - 1)
    U_fin, eps_imp = 4.0, -2.0
    nu, nd = (L + 1) // 2, L // 2
    nt, spg, dtg, m = 5, 2, 0.2, 14
    orbs = [(0, 0)]
    sec = basis.Sector(L, nu, nd)
    v0 = wl.start_vector(sec.dim, 7)
    bonds = [(0, j + 1) for j in range(L - 1)]
    # target: the same instance at U = 3 (oracle)
    tgt_model = wl.star_siam(eb, Vb, 3.0, eps_imp)
    tgt_ini = tgt_model.with_U([0.0] * L)
    tgt = greens.four_step(tgt_ini, tgt_model, nu, nd, orbs, nt, dtg, spg, m, v0, gs_tol=1e-13, reorth="cgs2")
    Tl, Tg = torch.from_numpy(tgt["G_lesser"]), torch.from_numpy(tgt["G_greater"])

    def loss_torch(eb_t, Vb_t, U_t):
        th = star_theta(torch, eb_t, Vb_t, U_t, torch.tensor(eps_imp, dtype=torch.float64), L)
        th_ini = star_theta(torch, eb_t, Vb_t, torch.zeros((), dtype=torch.float64),
                            torch.tensor(eps_imp, dtype=torch.float64), L)
        Gl, Gg = ag.greens_neq(ctx, L, bonds, bonds, th_ini, th, ctx.sector(L, nu, nd), to_dev(v0), orbs, nt, spg,
                               dtg / spg, krylov_dim=m, reorth=2, quad_nodes=10, cg_tol=1e-13, gs_tol=1e-13)
        return ((Gl - Tl).abs() ** 2).sum() + ((Gg - Tg).abs() ** 2).sum()

    def loss_oracle(eb_n, Vb_n, U_n):
        H = wl.star_siam(eb_n, Vb_n, U_n, eps_imp)
        Hi = H.with_U([0.0] * L)
        o = greens.four_step(Hi, H, nu, nd, orbs, nt, dtg, spg, m, v0, gs_tol=1e-13, reorth="cgs2")
        return float((np.abs(o["G_lesser"] - tgt["G_lesser"]) ** 2).sum()
                     + (np.abs(o["G_greater"] - tgt["G_greater"]) ** 2).sum())

    eb_t = torch.tensor(eb, requires_grad=True)
    Vb_t = torch.tensor(Vb, requires_grad=True)
    U_t = torch.tensor(U_fin, dtype=torch.float64, requires_grad=True)
    say("autograd fit", seed)
    loss = loss_torch(eb_t, Vb_t, U_t)
    loss.backward()
    assert abs(loss.item() - loss_oracle(eb, Vb, U_fin)) <= 1e-10 * max(1.0, loss.item())
    h = 1e-5
    fd_eb = [(loss_oracle(eb + h * e, Vb, U_fin) - loss_oracle(eb - h * e, Vb, U_fin)) / (2 * h) for e in np.eye(L - 1)]
    fd_Vb = [(loss_oracle(eb, Vb + h * e, U_fin) - loss_oracle(eb, Vb - h * e, U_fin)) / (2 * h) for e in np.eye(L - 1)]
    fd_U = (loss_oracle(eb, Vb, U_fin + h) - loss_oracle(eb, Vb, U_fin - h)) / (2 * h)
    got = np.concatenate([eb_t.grad.numpy(), Vb_t.grad.numpy(), [U_t.grad.item()]])
    ref = np.concatenate([fd_eb, fd_Vb, [fd_U]])
    say("max err", np.abs(got - ref).max(), "scale", np.abs(ref).max())
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max()


def test_batch_gradient_equals_single_instance_gradients(env):
    """Three Anderson instances (two of L = 5, one of L = 6) through the
    batched differentiable G: loss and theta-gradients equal the
    single-instance autograd path (itself checked against differences)."""
    import torch
    k, ag, ctx = env
    insts = []
    for seed, L in ((4001, 5), (4002, 5), (4005, 6)):
        rng = np.random.default_rng(seed)
        eb, Vb = rng.uniform(-2.0, 2.0, L - 1), 0.3 + 0.1 * rng.standard_normal(L - 1)
        insts.append((L, eb, Vb))
    nt, spg, dtg, m = 4, 2, 0.2, 14
    orbs = [(0, 0)]
    Ls, bl, thi, thf, secs, v0s, tg = [], [], [], [], [], [], []
    for L, eb, Vb in insts:
        nu, nd = (L + 1) // 2, L // 2
        bonds = [(0, j + 1) for j in range(L - 1)]
        sec = ctx.sector(L, nu, nd)
        Ls.append(L)
        bl.append(bonds)
        thi.append(star_theta(torch, torch.tensor(eb), torch.tensor(Vb), torch.zeros((), dtype=torch.float64),
                              torch.tensor(-2.0, dtype=torch.float64), L).requires_grad_(True))
        thf.append(star_theta(torch, torch.tensor(eb), torch.tensor(Vb), torch.tensor(4.0, dtype=torch.float64),
                              torch.tensor(-2.0, dtype=torch.float64), L).requires_grad_(True))
        secs.append(sec)
        v0s.append(to_dev(wl.start_vector(sec.dim, 7)))
        rng = np.random.default_rng(L)
        tg.append(torch.from_numpy(rng.standard_normal((nt, nt, 1, 1)) + 1j * rng.standard_normal((nt, nt, 1, 1))))
    say("batched autograd")
    Gl, Gg = ag.greens_neq_batch(ctx, Ls, bl, bl, thi, thf, secs, v0s, orbs, nt, spg, dtg / spg, krylov_dim=m,
                                 reorth=2, quad_nodes=10, cg_tol=1e-13, gs_tol=1e-13)
    loss = sum(((Gl[i] - tg[i]).abs() ** 2).sum() + ((Gg[i] - tg[i]).abs() ** 2).sum() for i in range(3))
    loss.backward()
    for i in range(3):
        a = thi[i].detach().clone().requires_grad_(True)
        b = thf[i].detach().clone().requires_grad_(True)
        gl, gg = ag.greens_neq(ctx, Ls[i], bl[i], bl[i], a, b, secs[i], v0s[i], orbs, nt, spg, dtg / spg,
                               krylov_dim=m, reorth=2, quad_nodes=10, cg_tol=1e-13, gs_tol=1e-13)
        li = ((gl - tg[i]).abs() ** 2).sum() + ((gg - tg[i]).abs() ** 2).sum()
        li.backward()
        scale = max(float(a.grad.abs().max()), float(b.grad.abs().max()))
        assert float((thi[i].grad - a.grad).abs().max()) <= 1e-9 * scale
        assert float((thf[i].grad - b.grad).abs().max()) <= 1e-9 * scale
