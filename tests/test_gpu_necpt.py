"""NE-CPT through the C ABI (kgf_bath_chain, kgf_necpt) against the oracle:
the bath functions of Eqs. (gb1), (gb2); the contour solve on the same
inputs (several GEMM tiles with ragged tails); the pipeline four-step ->
NE-CPT on an interacting Anderson chain; and, at the paper's sizes (1000-site
bath, dt = 0.02), the U = 0 limit in which the CPT equation is exact."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import say
from oracle import basis, greens, necpt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    return k.Context(0)


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _chain(n, t=1.0):
    h = np.zeros((n, n))
    for i in range(n - 1):
        h[i, i + 1] = h[i + 1, i] = -t
    return h


@pytest.mark.parametrize("Lb,Tb,beta", [(1000, 1.0, np.inf), (9, 0.7, np.inf), (12, 1.0, 15.0)])
def test_bath_chain_against_oracle(ctx, Lb, Tb, beta):
    nt, dt = 101, 0.02
    say("bath chain", Lb, Tb, beta)
    gl, gg = ctx.bath_chain(Lb, Tb, nt, dt, beta)
    rl, rg = necpt.bath_greens(_chain(Lb, Tb), nt, dt, beta, sites=[0])
    assert np.abs(gl.cpu().numpy() - rl[:, :, 0, 0]).max() < 1e-12
    assert np.abs(gg.cpu().numpy() - rg[:, :, 0, 0]).max() < 1e-12


def _siam_cluster(Lc, U, nt, dt):
    H = wl.chain_siam(Lc, U, 1.0)
    Hi = H.with_field(0, 0.2)
    nu = Lc // 2
    sec = basis.Sector(Lc, nu, Lc - nu)
    orbs = [(i, 0) for i in range(Lc)]
    return H, Hi, sec, orbs, greens.four_step(Hi, H, nu, Lc - nu, orbs, nt, dt, 2, 15,
                                              wl.start_vector(sec.dim, 7), gs_tol=1e-13)


@pytest.mark.parametrize("boundary", [3, 1])
def test_necpt_solve_against_oracle(ctx, boundary):
    """Same inputs on both sides: cluster G of the interacting (U = 1) Anderson
    chain from the oracle's four-step, bath of 12 sites; 82 contour points,
    328 right-hand sides."""
    nt, dt, Lb, V = 41, 0.05, 12, 0.9
    say("necpt oracle, boundary", boundary)
    *_, cl = _siam_cluster(4, 1.0, nt, dt)
    bl, bg = necpt.bath_greens(_chain(Lb), nt, dt)
    rl, rg = necpt.necpt(cl["G_lesser"], cl["G_greater"], bl, bg, boundary, V, dt)
    say("necpt GPU")
    gl, gg = ctx.necpt(_dev(cl["G_lesser"]), _dev(cl["G_greater"]), _dev(bl[:, :, 0, 0]), _dev(bg[:, :, 0, 0]),
                       boundary, V, dt)
    gl, gg = gl.cpu().numpy(), gg.cpu().numpy()
    scale = np.abs(rl).max()
    assert np.abs(gl - rl).max() < 1e-11 * scale and np.abs(gg - rg).max() < 1e-11 * scale
    assert np.abs(rl - cl["G_lesser"]).max() > 1e-2          # the coupling matters


def test_necpt_pipeline_four_step_to_cpt(ctx):
    """GPU four-step cluster G (kgf_greens_neq) -> GPU bath -> GPU NE-CPT,
    against the oracle's four-step -> bath -> CPT equation."""
    nt, dt, Lc, Lb, V = 21, 0.1, 4, 10, 1.0
    H, Hi, sec, orbs, cl = _siam_cluster(Lc, 1.0, nt, dt)
    bl, bg = necpt.bath_greens(_chain(Lb), nt, dt)
    rl, rg = necpt.necpt(cl["G_lesser"], cl["G_greater"], bl, bg, Lc - 1, V, dt)
    say("pipeline GPU")
    s = ctx.sector(Lc, sec.n_up, sec.n_dn)
    out = ctx.greens_neq(ctx.model(Hi), ctx.model(H), s, _dev(wl.start_vector(sec.dim, 7)), orbs, nt=nt,
                         steps_per_grid=2, dt=dt / 2, krylov_dim=15, reorth=2, gs_tol=1e-13)
    gbl, gbg = ctx.bath_chain(Lb, 1.0, nt, dt)
    gl, gg = ctx.necpt(_dev(out["G_lesser"]), _dev(out["G_greater"]), gbl, gbg, Lc - 1, V, dt)
    scale = np.abs(rl).max()
    say("pipeline errors", np.abs(gl.cpu().numpy() - rl).max() / scale, np.abs(gg.cpu().numpy() - rg).max() / scale)
    assert np.abs(gl.cpu().numpy() - rl).max() < 1e-10 * scale
    assert np.abs(gg.cpu().numpy() - rg).max() < 1e-10 * scale


def test_necpt_degenerate_cases(ctx):
    """V = 0 and a one-point mesh (zero quadrature weights) return G^c
    exactly; bad arguments are rejected."""
    import paper_1109_1205_amd as k
    nt, dt = 9, 0.1
    *_, cl = _siam_cluster(4, 1.0, nt, dt)
    bl, bg = necpt.bath_greens(_chain(6), nt, dt, sites=[0])
    Gl, Gg = _dev(cl["G_lesser"]), _dev(cl["G_greater"])
    b_l, b_g = _dev(bl[:, :, 0, 0]), _dev(bg[:, :, 0, 0])
    ol, og = ctx.necpt(Gl, Gg, b_l, b_g, 3, 0.0, dt)
    assert np.array_equal(ol.cpu().numpy(), cl["G_lesser"]) and np.array_equal(og.cpu().numpy(), cl["G_greater"])
    ol, og = ctx.necpt(Gl[:1, :1].contiguous(), Gg[:1, :1].contiguous(), b_l[:1, :1].contiguous(),
                       b_g[:1, :1].contiguous(), 3, 1.0, dt)
    assert np.array_equal(ol.cpu().numpy(), cl["G_lesser"][:1, :1])
    with pytest.raises(k.KgfError):
        ctx.necpt(Gl, Gg, b_l, b_g, 4, 1.0, dt)
    with pytest.raises(k.KgfError):
        ctx.necpt(Gl, Gg, b_l, b_g, 0, float("nan"), dt)
    with pytest.raises(ValueError):
        ctx.necpt(Gl, Gg, b_l[:-1], b_g, 0, 1.0, dt)


def test_necpt_u0_paper_sizes_property(ctx):
    """1000-site bath, dt = 0.02, t_max = 5, six cluster sites, U = 0: the
    CPT equation is exact there, so the GPU result equals the free-fermion G
    of the connected 1006-site chain within the scheme's second-order error
    (the same scheme evaluated on the CPU: 1.5e-4 of the coupling's effect,
    equal-time anticommutator off by 1.0e-4)."""
    Lc, Lb, V, dt, nt = 6, 1000, 1.0, 0.02, 251
    hc = _chain(Lc)
    hci = hc.copy()
    hci[0, 0] -= 0.2
    rho_c = necpt.ground_density(hci, Lc // 2)
    Gcl, Gcg = necpt.free_greens(hc, rho_c, nt, dt)
    say("necpt paper sizes GPU")
    gbl, gbg = ctx.bath_chain(Lb, 1.0, nt, dt)
    gl, gg = ctx.necpt(_dev(Gcl), _dev(Gcg), gbl, gbg, Lc - 1, V, dt)
    gl, gg = gl.cpu().numpy(), gg.cpu().numpy()
    say("exact chain")
    h = np.zeros((Lc + Lb, Lc + Lb))
    h[:Lc, :Lc], h[Lc:, Lc:] = hc, _chain(Lb)
    h[Lc - 1, Lc] = h[Lc, Lc - 1] = -V
    rho = np.zeros_like(h)
    rho[:Lc, :Lc], rho[Lc:, Lc:] = rho_c, necpt.ground_density(_chain(Lb), Lb // 2)
    e, u = np.linalg.eigh(h)
    R = u.T @ rho @ u
    M = u[:Lc][None, :, :] * np.exp(-1j * np.outer(dt * np.arange(nt), e))[:, None, :]
    El = 1j * np.einsum("aik,bjk->abij", M @ R, M.conj())
    Eg = 1j * np.einsum("aik,bjk->abij", M @ (R - np.eye(len(e))), M.conj())
    effect = np.abs(El - Gcl).max()
    err = max(np.abs(gl - El).max(), np.abs(gg - Eg).max())
    say("err / effect", err / effect)
    assert effect > 0.2 and err < 5e-4 * effect
    # equal times: G^> - G^< = -i to the same order
    d = np.einsum("aaij->aij", gg - gl)
    assert np.abs(d + 1j * np.eye(Lc)).max() < 5e-4
