"""The initial state of the NE-CPT results of Sec. 5 (Fig. 5 discussion):
Anderson chain of L_c = 6 sites (U = T = V = 1, field h = 0.2 on the
impurity), linked at its last site to a 1000-site bath, imaginary branch
beta = 15, dtau = 0.02, through the C ABI (kgf_greens_neq with the
Matsubara branch -> kgf_cluster_contour completed for the finite branch ->
kgf_bath_chain_contour -> kgf_necpt_contour per spin).  The t = 0 local
moments m_i = n_i,up - n_i,down of the connected system against the values
the paper states (tests/golden/paper_facts.json, fig5_initial_moments), and
against the isolated cluster's (whose net moment is that of its S_z = 0
ground state, so the CPT's larger net polarisation is the bath's effect)."""
import json
import os

import numpy as np
import pytest

import workloads as wl
from gpu_common import say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")


def test_fig5_initial_moments():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    spec = json.load(open(GOLDEN))["fig5_initial_moments"]
    m, cl = spec["model"], spec["claims"]
    Lc, Lb, V, beta, dtau = m["L_c"], m["L_b"], m["V"], m["beta"], m["dtau"]
    ntau = int(round(beta / dtau)) + 1
    nt, dt = 2, 0.02
    ctx = k.Context(0)
    H = wl.chain_siam(Lc, m["U"], m["T"])
    Hi = H.with_field(m["field_site"], m["field_h"])
    nu, nd = spec["sector"]
    s = ctx.sector(Lc, nu, nd)
    v0 = torch.from_numpy(wl.start_vector(s.dim, 7)).to("cuda:0")
    orbs = [(i, sp) for sp in (0, 1) for i in range(Lc)]
    say("fig5: cluster four-step with the Matsubara branch,", ntau, "tau points")
    out = ctx.greens_neq(ctx.model(Hi), ctx.model(H), s, v0, orbs, nt=nt, steps_per_grid=1, dt=dt, krylov_dim=15,
                         reorth=2, gs_tol=1e-13, ntau=ntau, tau_steps_per_grid=1, dtau=dtau)
    gb = ctx.bath_chain_contour(Lb, m["T"], nt, dt, ntau, dtau, beta)
    n_cpt, n_iso = [], []
    for sp in (0, 1):
        idx = [j for j, (_, q) in enumerate(orbs) if q == sp]
        res = ctx.necpt_contour(ctx.cluster_contour(out, orbitals=idx, kms=True), gb, Lc - 1, V, dt, dtau)
        n_cpt.append(np.real(-1j * np.diag(res["G_lesser"][0, 0].cpu().numpy())))
        n_iso.append(np.real(-1j * np.diag(out["G_lesser"][0, 0][idx][:, idx])))
    m_cpt, m_iso = n_cpt[0] - n_cpt[1], n_iso[0] - n_iso[1]
    say("t = 0 moments, connected:", m_cpt[:4], "net", m_cpt[:4].sum(), "isolated:", m_iso[:4], "net",
        m_iso[:4].sum())
    tol = cl["tolerance"]
    assert abs(m_cpt[0] - cl["impurity_moment_t0"]) < tol
    assert abs(m_cpt[:4].sum() - cl["net_moment_sites_1_4_t0"]) < tol
    assert abs(m_iso.sum()) < 1e-10                      # S_z = 0 ground state of the isolated cluster
    assert m_cpt[:4].sum() > m_iso[:4].sum() + 0.05      # the bath carries the compensating moment
