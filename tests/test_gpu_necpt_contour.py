"""NE-CPT on the Keldysh-Matsubara contour through the C ABI
(kgf_bath_chain_contour, kgf_necpt_contour, and kgf_greens_neq's Matsubara
and mixed components) against the oracle (Sec. 5, Eq. (cpteq), Eqs. (gb1),
(gb2)):

* the bath functions on complex contour times, finite beta and beta -> inf;
* the contour solve on the same inputs (U = 0 cluster, thermal), every
  component, against the oracle's CPT equation with the bath written out;
* the pipeline four-step (cluster ground state, all components) -> bath ->
  contour solve on an interacting Anderson chain, against the oracle's
  pipeline; the initial (t = 0) impurity density of the connected system
  differs from the isolated cluster's, and the equal-time anticommutator
  holds to the scheme's order."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say
from oracle import basis, greens, necpt

pytestmark = pytest.mark.gpu

KEYS = ("lesser", "greater", "mixed", "mixed_left", "vert_greater", "vert_lesser")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    return k.Context(0)


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _chain(n, t=1.0, eps=None):
    h = np.zeros((n, n))
    for i in range(n - 1):
        h[i, i + 1] = h[i + 1, i] = -t
    if eps is not None:
        h += np.diag(eps)
    return h


@pytest.mark.parametrize("Lb,Tb,beta", [(12, 1.0, 3.0), (9, 0.7, np.inf), (1000, 1.0, 15.0)])
def test_bath_chain_contour_against_oracle(ctx, Lb, Tb, beta):
    nt, dt = 21, 0.1
    ntau = 31
    dtau = (3.0 if np.isinf(beta) else beta) / (ntau - 1)
    say("bath chain contour", Lb, Tb, beta)
    got = ctx.bath_chain_contour(Lb, Tb, nt, dt, ntau, dtau, beta)
    ref = necpt.bath_greens_l(_chain(Lb, Tb), nt, dt, ntau, dtau, beta, sites=[0])
    for k in KEYS:
        assert np.abs(got[k].cpu().numpy() - ref[k][..., 0, 0]).max() < 1e-12, k


def test_contour_solve_against_oracle(ctx):
    """Same inputs on both sides: thermal U = 0 cluster of 3 sites (field on
    site 0 switched off at t = 0), bath of 6 sites at beta = 3; 13 real and
    31 imaginary mesh points, 57 contour points."""
    nc, Lb, V, beta, dt, nt, ntau = 3, 6, 0.8, 3.0, 0.1, 13, 31
    dtau = beta / (ntau - 1)
    Gc = necpt.free_greens_l(_chain(nc, 1.0, [0.4, 0, 0]), _chain(nc), beta, nt, dt, ntau, dtau)
    Gb = necpt.bath_greens_l(_chain(Lb), nt, dt, ntau, dtau, beta, sites=[0])
    ref = necpt.necpt_l(Gc, Gb, 2, V, dt, dtau)
    say("contour solve (GPU)")
    got = ctx.necpt_contour({k: _dev(Gc[k]) for k in KEYS}, {k: _dev(Gb[k][..., 0, 0]) for k in KEYS}, 2, V, dt, dtau)
    for key in ("lesser", "greater", "mixed", "mixed_left"):
        e = rel_err(got["G_" + key].cpu().numpy(), ref[key])
        say(key, e)
        assert e < 1e-10, key


def test_pipeline_against_oracle(ctx):
    """Interacting Anderson chain (L_c = 4, U = 1, field 0.2 on the impurity
    switched off at t = 0), spin up; bath of 8 sites, V = 1, beta = 3: the
    GPU four-step (Matsubara and both mixed components) -> GPU bath -> GPU
    contour solve against the oracle's four-step -> bath -> CPT equation with
    the bath written out."""
    Lc, Lb, V, beta = 4, 8, 1.0, 3.0
    nt, spg, dtg = 9, 2, 0.1
    ntau, tspg = 31, 2
    dtau = beta / (ntau - 1)
    H = wl.chain_siam(Lc, 1.0, 1.0)
    Hi = H.with_field(0, 0.2)
    sec = basis.Sector(Lc, 2, 2)
    orbs = [(i, 0) for i in range(Lc)]
    v0 = wl.start_vector(sec.dim, 7)
    ora = greens.four_step(Hi, H, 2, 2, orbs, nt, dtg, spg, 15, v0, gs_tol=1e-13, reorth="none", ntau=ntau,
                           dtau_grid=dtau, tau_steps_per_grid=tspg)
    Gc_ref = necpt.cluster_fn(ora)
    Gb_ref = necpt.bath_greens_l(_chain(Lb), nt, dtg, ntau, dtau, beta, sites=[0])
    ref = necpt.necpt_l(Gc_ref, Gb_ref, Lc - 1, V, dtg, dtau)
    say("pipeline: GPU four-step with Matsubara branch")
    g4 = ctx.greens_neq(ctx.model(Hi), ctx.model(H), ctx.sector(Lc, 2, 2), _dev(v0), orbs, nt, spg, dtg / spg,
                        krylov_dim=15, reorth=0, schedule=1, ntau=ntau, tau_steps_per_grid=tspg, dtau=dtau / tspg,
                        gs_tol=1e-13)
    for key in ("G_matsubara", "G_mixed", "G_mixed_left"):
        assert rel_err(g4[key], ora[key]) < 1e-10, key
    Gc = {"lesser": g4["G_lesser"], "greater": g4["G_greater"], "mixed": g4["G_mixed"],
          "mixed_left": g4["G_mixed_left"], "vert_greater": 1j * g4["G_matsubara"][0],
          "vert_lesser": 1j * g4["G_matsubara"][1]}
    Gb = ctx.bath_chain_contour(Lb, 1.0, nt, dtg, ntau, dtau, beta)
    got = ctx.necpt_contour({k: _dev(Gc[k]) for k in KEYS}, Gb, Lc - 1, V, dtg, dtau)
    for key in ("lesser", "greater", "mixed", "mixed_left"):
        e = rel_err(got["G_" + key].cpu().numpy(), ref[key])
        say("pipeline", key, e)
        assert e < 1e-10, key
    Gl = got["G_lesser"].cpu().numpy()
    Gg = got["G_greater"].cpu().numpy()
    n_cpt = np.real(-1j * Gl[0, 0, 0, 0])
    n_iso = np.real(-1j * g4["G_lesser"][0, 0, 0, 0])
    say("impurity n_up at t = 0: connected", n_cpt, "isolated", n_iso)
    assert abs(n_cpt - n_iso) > 1e-3
    for k in range(nt):
        assert np.abs(Gg[k, k] - Gl[k, k] + 1j * np.eye(Lc)).max() < 1e-2


def test_cluster_contour_assembly_against_oracle(ctx):
    """kgf_cluster_contour on the oracle's four-step output (both spins, one
    spin selected): the plain assembly equals the oracle's cluster_fn and the
    completion for the finite imaginary branch its cluster_fn_kms, element
    by element (the same additions and conjugations on both sides)."""
    Lc, nt, spg, dtg, ntau, tspg, beta = 4, 7, 2, 0.1, 21, 2, 2.0
    dtau = beta / (ntau - 1)
    H = wl.chain_siam(Lc, 1.0, 1.0)
    Hi = H.with_field(0, 0.2)
    sec = basis.Sector(Lc, 2, 2)
    orbs = [(i, sp) for sp in (0, 1) for i in range(Lc)]
    ora = greens.four_step(Hi, H, 2, 2, orbs, nt, dtg, spg, 15, wl.start_vector(sec.dim, 7), gs_tol=1e-13,
                           reorth="none", ntau=ntau, dtau_grid=dtau, tau_steps_per_grid=tspg)
    for sp in (0, 1):
        idx = [k for k, (_, q) in enumerate(orbs) if q == sp]
        sub = {k: np.ascontiguousarray(ora[k][..., idx, :][..., idx])
               for k in ("G_lesser", "G_greater", "G_matsubara", "G_mixed", "G_mixed_left")}
        for kms, fn in ((False, necpt.cluster_fn), (True, necpt.cluster_fn_kms)):
            ref = fn(sub)
            got = ctx.cluster_contour(ora, orbitals=idx, kms=kms)
            for key in KEYS:
                assert np.abs(got[key].cpu().numpy() - ref[key]).max() <= 1e-15 * np.abs(ref[key]).max(), (sp, kms, key)


def test_pipeline_kms_moments_against_oracle(ctx):
    """The pipeline with the cluster functions completed for the finite
    imaginary branch (the reading of Sec. 5's Matsubara branch at finite beta
    for a zero-temperature cluster): GPU four-step of both spins ->
    kgf_cluster_contour (kms) -> GPU bath -> contour solve per spin, against
    the oracle's four-step -> cluster_fn_kms -> bath -> CPT equation.  The
    t = 0 local moments m_i = n_i,up - n_i,down of the connected system differ
    from the isolated cluster's: the isolated cluster's ground state has
    S_z = 0, so its net moment over the cluster vanishes (as Sec. 5 notes for
    the smallest cluster), the connected system's does not."""
    Lc, Lb, V, beta = 4, 8, 1.0, 3.0
    nt, spg, dtg = 9, 2, 0.1
    ntau, tspg = 31, 2
    dtau = beta / (ntau - 1)
    H = wl.chain_siam(Lc, 1.0, 1.0)
    Hi = H.with_field(0, 0.2)
    sec = basis.Sector(Lc, 2, 2)
    orbs = [(i, sp) for sp in (0, 1) for i in range(Lc)]
    v0 = wl.start_vector(sec.dim, 7)
    ora = greens.four_step(Hi, H, 2, 2, orbs, nt, dtg, spg, 15, v0, gs_tol=1e-13, reorth="none", ntau=ntau,
                           dtau_grid=dtau, tau_steps_per_grid=tspg)
    Gb_ref = necpt.bath_greens_l(_chain(Lb), nt, dtg, ntau, dtau, beta, sites=[0])
    say("pipeline kms: GPU four-step, both spins")
    g4 = ctx.greens_neq(ctx.model(Hi), ctx.model(H), ctx.sector(Lc, 2, 2), _dev(v0), orbs, nt, spg, dtg / spg,
                        krylov_dim=15, reorth=0, schedule=1, ntau=ntau, tau_steps_per_grid=tspg, dtau=dtau / tspg,
                        gs_tol=1e-13)
    Gb = ctx.bath_chain_contour(Lb, 1.0, nt, dtg, ntau, dtau, beta)
    n_cpt, n_iso = [], []
    for sp in (0, 1):
        idx = [k for k, (_, q) in enumerate(orbs) if q == sp]
        sub = {k: np.ascontiguousarray(ora[k][..., idx, :][..., idx])
               for k in ("G_lesser", "G_greater", "G_matsubara", "G_mixed", "G_mixed_left")}
        ref = necpt.necpt_l(necpt.cluster_fn_kms(sub), Gb_ref, Lc - 1, V, dtg, dtau)
        got = ctx.necpt_contour(ctx.cluster_contour(g4, orbitals=idx, kms=True), Gb, Lc - 1, V, dtg, dtau)
        for key in ("lesser", "greater", "mixed", "mixed_left"):
            e = rel_err(got["G_" + key].cpu().numpy(), ref[key])
            say("pipeline kms spin", sp, key, e)
            assert e < 1e-10, (sp, key)
        n_cpt.append(np.real(-1j * np.diag(got["G_lesser"][0, 0].cpu().numpy())))
        n_iso.append(np.real(-1j * np.diag(g4["G_lesser"][0, 0][idx][:, idx])))
    m_cpt, m_iso = n_cpt[0] - n_cpt[1], n_iso[0] - n_iso[1]
    say("t = 0 moments: connected", m_cpt, "isolated", m_iso)
    assert abs(m_iso.sum()) < 1e-12
    assert abs(m_cpt.sum()) > 1e-3
    assert np.abs(m_cpt - m_iso).max() > 1e-3
