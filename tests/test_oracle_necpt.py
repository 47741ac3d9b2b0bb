"""Pins of the NE-CPT oracle (Sec. 5, Eq. (cpteq), on the Keldysh contour)
against facts that do not depend on it:

* the bath functions of Eqs. (gb1), (gb2) at beta -> infinity equal the exact
  propagation of the bath's ground-state density matrix (even chain; odd
  chain with its zero level half filled);
* V = 0 returns the cluster function unchanged;
* at U = 0 the CPT equation is exact: the solution converges to the exact
  free-fermion G of the connected chain from the product initial state, at
  second order in dt (error ratio ~4 when dt halves); with the mean also at
  the branch ends (a plausible slip) it falls to first order (ratio ~2);
* for an interacting cluster (U = 2) the equal-time anticommutator
  G^>(t, t) - G^<(t, t) = -i, exact for the CPT equation at any U (G - G' =
  G' * V * G has no equal-time jump), is met to second order in dt;
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


def _u0_errors(Lc, V, tmax, dts, solve):
    hc, rho_c, Tb, h, rho = _u0_system(Lc=Lc, V=V)
    err, effect = [], None
    for dt in dts:
        nt = int(round(tmax / dt)) + 1
        Gcl, Gcg = necpt.free_greens(hc, rho_c, nt, dt)
        Gbl, Gbg = necpt.bath_greens(Tb, nt, dt)
        Gl, Gg = solve(Gcl, Gcg, Gbl, Gbg, Lc - 1, V, dt)
        El, Eg = necpt.free_greens(h, rho, nt, dt)
        El, Eg = El[:, :, :Lc, :Lc], Eg[:, :, :Lc, :Lc]
        err.append(max(np.abs(Gl - El).max(), np.abs(Gg - Eg).max()))
        if effect is None:
            effect = np.abs(El - Gcl).max()
    return err, effect


def _necpt_mean_at_ends(Gcl, Gcg, Gbl, Gbg, boundary, V, dt):
    """The CPT equation with the mean on the whole equal-point diagonal."""
    import scipy.linalg
    nt, nc = Gcl.shape[0], Gcl.shape[2]
    Gl, Gg, Vm = necpt.embed(Gcl, Gcg, Gbl, Gbg, boundary, V)
    n = Gl.shape[2]
    Z = necpt.to_contour(Gl, Gg).reshape(2 * nt, n, 2 * nt, n)
    for p in (0, nt - 1, nt, 2 * nt - 1):
        a = p if p < nt else 2 * nt - 1 - p
        Z[p, :, p, :] = 0.5 * (Gl[a, a] + Gg[a, a])
    Z = Z.reshape(2 * nt * n, 2 * nt * n)
    _, w = necpt.contour_points(nt, dt)
    G = scipy.linalg.solve(np.eye(Z.shape[0]) - Z @ np.kron(np.diag(w), Vm), Z)
    Hl, Hg = necpt.from_contour(G, nt, n)
    return Hl[:, :, :nc, :nc], Hg[:, :, :nc, :nc]


def test_u0_converges_to_the_exact_connected_chain():
    err, effect = _u0_errors(4, 1.0, 2.0, (0.1, 0.05, 0.025), necpt.necpt)
    assert effect > 0.2                      # the coupling changes G at O(1)
    assert err[0] < 0.01 * effect
    r1, r2 = err[0] / err[1], err[1] / err[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, (err, r1, r2)
    # the mean also at the branch ends: first order only
    bad, _ = _u0_errors(4, 1.0, 2.0, (0.1, 0.05), _necpt_mean_at_ends)
    assert 1.8 < bad[0] / bad[1] < 2.3 and bad[1] > 10 * err[1], (bad, err)


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


def test_interacting_anticommutator_converges_second_order():
    L, Lb, V, tmax = 4, 10, 1.0, 2.0
    H = wl.chain_siam(L, 2.0, 1.0)
    Hi = H.with_field(0, 0.2)
    sec = basis.Sector(L, 2, 2)
    orbs = [(i, 0) for i in range(L)]
    dev = []
    for dt in (0.1, 0.05):
        nt = int(round(tmax / dt)) + 1
        cl = greens.four_step(Hi, H, 2, 2, orbs, nt, dt, 2, 15, wl.start_vector(sec.dim, 7), gs_tol=1e-13)
        assert np.abs(np.einsum("aaij->aij", cl["G_greater"] - cl["G_lesser"]) + 1j * np.eye(L)).max() < 1e-12
        bl, bg = necpt.bath_greens(_chain(Lb), nt, dt)
        Gl, Gg = necpt.necpt(cl["G_lesser"], cl["G_greater"], bl, bg, L - 1, V, dt)
        effect = np.abs(Gl - cl["G_lesser"]).max()
        dev.append(np.abs(np.einsum("aaij->aij", Gg - Gl) + 1j * np.eye(L)).max())
        assert effect > 0.2 and dev[-1] < 0.02 * effect
    assert 3.6 < dev[0] / dev[1] < 4.4, dev
