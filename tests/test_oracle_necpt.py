"""Pins of the NE-CPT oracle (Sec. 5, Eq. (cpteq), on the Keldysh contour)
against facts that do not depend on it:

* the bath functions of Eqs. (gb1), (gb2) at beta -> infinity equal the exact
  propagation of the bath's ground-state density matrix (even chain; odd
  chain with its zero level half filled);
* V = 0 returns the cluster function unchanged;
* at U = 0 the CPT equation is exact: the solution converges to the exact
  free-fermion G of the connected chain from the product initial state, at
  first order in dt (error ratio ~2 when dt halves), and the Richardson
  combination 2 G(dt/2) - G(dt) removes that order;
* the oracle's four-step cluster G at U = 0 equals the free-fermion G of the
  cluster's one-particle Hamiltonian after the field quench (the object the
  CPT equation takes as G^c, with its conventions of sign and order)."""
import numpy as np
import pytest

import workloads as wl
from oracle import basis, greens, necpt


def _chain(n, t=1.0):
    h = np.zeros((n, n))
    for i in range(n - 1):
        h[i, i + 1] = h[i + 1, i] = -t
    return h


@pytest.mark.parametrize("Lb", [10, 9])
def test_bath_formula_is_free_propagation(Lb):
    T = _chain(Lb, 0.8)
    e, u = np.linalg.eigh(T)
    rho = u[:, e < -1e-9] @ u[:, e < -1e-9].T
    z = np.abs(e) <= 1e-9
    rho = rho + 0.5 * u[:, z] @ u[:, z].T
    Gl, Gg = necpt.bath_greens(T, 7, 0.3)
    Fl, Fg = necpt.free_greens(T, rho, 7, 0.3)
    assert np.abs(Gl - Fl).max() < 1e-13 and np.abs(Gg - Fg).max() < 1e-13
    # equal times: G^> - G^< = -i
    assert np.abs(Gg[3, 3] - Gl[3, 3] + 1j * np.eye(Lb)).max() < 1e-13
    Sl, Sg = necpt.bath_greens(T, 7, 0.3, sites=[0])
    assert np.abs(Sl[:, :, 0, 0] - Gl[:, :, 0, 0]).max() < 1e-15


def _u0_system(Lc=4, Lb=10, V=1.0, field=0.1):
    hc = _chain(Lc)
    hci = hc.copy()
    hci[0, 0] -= field
    rho_c = necpt.ground_density(hci, Lc // 2)
    Tb = _chain(Lb)
    rho_b = necpt.ground_density(Tb, Lb // 2)
    h = np.zeros((Lc + Lb, Lc + Lb))
    h[:Lc, :Lc], h[Lc:, Lc:] = hc, Tb
    h[Lc - 1, Lc] = h[Lc, Lc - 1] = -V
    rho = np.zeros_like(h)
    rho[:Lc, :Lc], rho[Lc:, Lc:] = rho_c, rho_b
    return hc, rho_c, Tb, h, rho


def test_zero_coupling_returns_the_cluster_function():
    hc, rho_c, Tb, _, _ = _u0_system()
    Gcl, Gcg = necpt.free_greens(hc, rho_c, 9, 0.1)
    Gbl, Gbg = necpt.bath_greens(Tb, 9, 0.1)
    Gl, Gg = necpt.necpt(Gcl, Gcg, Gbl, Gbg, 3, 0.0, 0.1)
    assert np.abs(Gl - Gcl).max() < 1e-15 and np.abs(Gg - Gcg).max() < 1e-15


def test_u0_converges_to_the_exact_connected_chain():
    Lc, V, tmax = 4, 1.0, 2.0
    hc, rho_c, Tb, h, rho = _u0_system(Lc=Lc, V=V)
    sols, exact = [], []
    for dt in (0.1, 0.05, 0.025):
        nt = int(round(tmax / dt)) + 1
        Gcl, Gcg = necpt.free_greens(hc, rho_c, nt, dt)
        Gbl, Gbg = necpt.bath_greens(Tb, nt, dt)
        sols.append(necpt.necpt(Gcl, Gcg, Gbl, Gbg, Lc - 1, V, dt))
        El, Eg = necpt.free_greens(h, rho, nt, dt)
        exact.append((El[:, :, :Lc, :Lc], Eg[:, :, :Lc, :Lc]))
    # compare on the common coarse mesh t = 0, 0.1, ..., 2
    def coarse(G, s):
        return G[::s, ::s]
    err = []
    for k, s in enumerate((1, 2, 4)):
        err.append(max(np.abs(coarse(sols[k][q], s) - coarse(exact[k][q], s)).max() for q in (0, 1)))
    effect = np.abs(exact[0][0] - necpt.free_greens(hc, rho_c, 21, 0.1)[0]).max()
    assert effect > 0.2                      # the coupling changes G at O(1)
    assert err[0] < 0.05 * effect
    r1, r2 = err[0] / err[1], err[1] / err[2]
    assert 1.8 < r1 < 2.3 and 1.8 < r2 < 2.3, (err, r1, r2)
    rich = [max(np.abs(2 * coarse(sols[k + 1][q], 2) - coarse(sols[k][q], 1) - coarse(exact[k][q], 1)).max()
                for q in (0, 1)) for k in (0,)]
    rich2 = max(np.abs(2 * coarse(sols[2][q], 2) - coarse(sols[1][q], 1) - coarse(exact[1][q], 1)).max()
                for q in (0, 1))
    assert rich[0] < 0.3 * err[1] and rich2 < 0.3 * err[2], (rich, rich2, err)
    assert rich[0] / rich2 > 3.0, (rich, rich2)


def test_four_step_cluster_at_u0_is_free_fermions():
    """U = 0 Anderson chain, field -h (n_up - n_dn) on the impurity for t < 0:
    the oracle's many-body four-step G^<, G^> of the up spin equal the
    free-fermion functions of the one-particle Hamiltonian."""
    L = 4
    H = wl.chain_siam(L, 0.0, 1.0)
    Hi = H.with_field(0, 0.2)
    sec = basis.Sector(L, 2, 2)
    orbs = [(i, 0) for i in range(L)]
    out = greens.four_step(Hi, H, 2, 2, orbs, 6, 0.2, 2, 15, wl.start_vector(sec.dim, 7), gs_tol=1e-13)

    def one_particle(M):
        h = np.diag(np.asarray(M.eps_up, float))
        for (i, j), t in zip(M.bonds, M.t):
            h[i, j] -= t
            h[j, i] -= t
        return h
    rho = necpt.ground_density(one_particle(Hi), 2)
    Fl, Fg = necpt.free_greens(one_particle(H), rho, 6, 0.2)
    assert np.abs(out["G_lesser"] - Fl).max() < 1e-10
    assert np.abs(out["G_greater"] - Fg).max() < 1e-10
