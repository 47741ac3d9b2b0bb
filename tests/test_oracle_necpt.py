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
  CPT equation takes as G^c, with its conventions of sign and order).

On the Keldysh-Matsubara (L-shaped) contour, with the imaginary branch of
length beta through which the connected initial state enters:

* the thermal free-fermion components (overflow-free eigenbasis forms)
  equal the plain matrix-exponential definitions;
* thermal functions are antiperiodic between the contour's first point
  (t = 0) and its last (tau = beta), for the free functions and for the
  bath of Eqs. (gb1), (gb2) on complex times;
* the bath functions equal the free functions of the unquenched bath, at
  finite beta and beta -> infinity;
* at U = 0 the CPT equation on the L-shaped contour converges to the
  connected system's exact thermal functions at second order in the mesh
  step on every component, and its t = 0 densities are the connected
  system's (not the isolated cluster's);
* V = 0 returns G' on every component;
* the four-step components (G^M(+-tau), both mixed functions) at U = 0 are
  the zero-temperature free-fermion functions of the L-shaped contour."""
import numpy as np
import scipy.linalg
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


# ---- the Keldysh-Matsubara (L-shaped) contour ------------------------------

def _chain_h(L, t=1.0, eps=None):
    h = np.zeros((L, L))
    for i in range(L - 1):
        h[i, i + 1] = h[i + 1, i] = -t
    if eps is not None:
        h += np.diag(eps)
    return h


def test_free_greens_l_against_matrix_functions():
    """Components of the thermal free-fermion contour functions against the
    definitions with plain matrix exponentials and inverses (beta small
    enough that e^{beta h} is harmless)."""
    rng = np.random.default_rng(11)
    h_ini = _chain_h(4, 1.0, rng.uniform(-1, 1, 4))
    h = _chain_h(4, 1.0, rng.uniform(-1, 1, 4))
    beta, nt, dt, ntau, dtau = 2.0, 3, 0.3, 5, 0.5
    fn = necpt.free_greens_l(h_ini, h, beta, nt, dt, ntau, dtau)
    I = np.eye(4)
    f = np.linalg.inv(scipy.linalg.expm(beta * h_ini) + I)
    U = [scipy.linalg.expm(-1j * h * dt * k) for k in range(nt)]
    E = lambda x: scipy.linalg.expm(x * h_ini)
    for a in range(nt):
        for b in range(nt):
            np.testing.assert_allclose(fn["lesser"][a, b], 1j * U[a] @ f @ U[b].conj().T, atol=1e-13)
            np.testing.assert_allclose(fn["greater"][a, b], -1j * U[a] @ (I - f) @ U[b].conj().T, atol=1e-13)
        for j in range(ntau):
            tau = j * dtau
            np.testing.assert_allclose(fn["mixed"][a, j], 1j * U[a] @ f @ E(tau), atol=1e-12)
            np.testing.assert_allclose(fn["mixed_left"][j, a], -1j * E(-tau) @ (I - f) @ U[a].conj().T, atol=1e-12)
    for d in range(ntau):
        tau = d * dtau
        np.testing.assert_allclose(fn["vert_greater"][d], -1j * E(-tau) @ (I - f), atol=1e-12)
        np.testing.assert_allclose(fn["vert_lesser"][d], 1j * f @ E(tau), atol=1e-12)


def test_thermal_functions_are_antiperiodic():
    """KMS: the contour's first point (t = 0, forward) and last point
    (tau = beta) are one, up to the fermion sign: G(0, z') = -G(-i beta, z');
    checked for the free functions and for the bath of Eqs. (gb1), (gb2)."""
    h_ini = _chain_h(5, 1.0, [0.3, -0.2, 0.1, 0.0, 0.4])
    beta, nt, dt, ntau = 3.0, 4, 0.25, 31
    dtau = beta / (ntau - 1)
    for fn in (necpt.free_greens_l(h_ini, _chain_h(5), beta, nt, dt, ntau, dtau),
               necpt.bath_greens_l(h_ini, nt, dt, ntau, dtau, beta)):
        for b in range(nt):
            np.testing.assert_allclose(fn["lesser"][0, b], -fn["mixed_left"][ntau - 1, b], atol=1e-13)
        for j in range(ntau):
            np.testing.assert_allclose(fn["mixed"][0, j], -fn["vert_greater"][ntau - 1 - j], atol=1e-13)


def test_bath_l_matches_free_functions():
    """Eqs. (gb1), (gb2) on the L-shaped contour (eigenbasis of T) equal the
    free-fermion functions of the unquenched bath (matrix exponentials),
    at finite beta and at beta -> infinity."""
    T = _chain_h(7, 1.0)
    for beta in (4.0, np.inf):
        nt, dt, ntau, dtau = 5, 0.2, 21, 0.2
        a = necpt.bath_greens_l(T, nt, dt, ntau, dtau, beta, sites=[0, 1])
        b = necpt.free_greens_l(T, T, beta, nt, dt, ntau, dtau)
        for key in a:
            np.testing.assert_allclose(a[key], b[key][..., :2, :2], atol=1e-12, err_msg=key)


def _u0_quench_l(dt, beta=3.0, t_max=1.2, nb=5, V=0.7):
    """U = 0 cluster (3-site chain, field 0.4 on site 0 switched off at
    t = 0) linked at site 2 to a 5-site bath chain; everything thermal at
    beta, with the imaginary branch of length beta on the mesh dt."""
    nc = 3
    hc_ini = _chain_h(nc, 1.0, [0.4, 0.0, 0.0])
    hc = _chain_h(nc, 1.0)
    Tb = _chain_h(nb, 1.0)
    nt = int(round(t_max / dt)) + 1
    ntau = int(round(beta / dt)) + 1
    Gc = necpt.free_greens_l(hc_ini, hc, beta, nt, dt, ntau, dt)
    Gb = necpt.bath_greens_l(Tb, nt, dt, ntau, dt, beta, sites=[0])
    got = necpt.necpt_l(Gc, Gb, 2, V, dt, dt)
    # the connected system, exactly: bond -V between cluster site 2 and bath site 0
    n = nc + nb
    def full(hcl):
        h = np.zeros((n, n))
        h[:nc, :nc] = hcl
        h[nc:, nc:] = Tb
        h[2, nc] = h[nc, 2] = -V
        return h
    ref = necpt.free_greens_l(full(hc_ini), full(hc), beta, nt, dt, ntau, dt)
    return got, ref, nc


def test_lcontour_cpt_exact_at_u0_second_order():
    """At U = 0 the CPT equation on the L-shaped contour is exact: the
    discretised solution converges to the connected system's functions
    (prepared in its own thermal state by the imaginary branch) at second
    order in the mesh step, the t = 0 densities included."""
    errs = []
    for dt in (0.2, 0.1):
        got, ref, nc = _u0_quench_l(dt)
        e = max(np.abs(got[k] - ref[k][..., :nc, :nc]).max() for k in ref)
        errs.append(e)
    assert errs[1] < 5e-3, errs
    ratio = errs[0] / errs[1]
    assert 3.3 < ratio < 4.8, (errs, ratio)
    # initial densities: the connected equilibrium, not the isolated cluster's
    got, ref, nc = _u0_quench_l(0.1)
    n_got = np.real(-1j * np.diag(got["lesser"][0, 0]))
    n_ref = np.real(-1j * np.diag(ref["lesser"][0, 0][:nc, :nc]))
    hc_ini = _chain_h(nc, 1.0, [0.4, 0.0, 0.0])
    n_iso = np.real(np.diag(necpt.free_greens_l(hc_ini, hc_ini, 3.0, 1, 0.1, 2, 0.1)["lesser"][0, 0] * -1j))
    assert np.abs(n_got - n_ref).max() < 1e-4
    assert np.abs(n_ref - n_iso).max() > 3e-3


def test_lcontour_reduces_to_keldysh_without_imaginary_branch_coupling():
    """V = 0: the solution is G' itself on every component."""
    got, _, nc = _u0_quench_l(0.2, V=0.0)
    hc_ini = _chain_h(nc, 1.0, [0.4, 0.0, 0.0])
    nt, ntau = got["lesser"].shape[0], got["vert_greater"].shape[0]
    Gc = necpt.free_greens_l(hc_ini, _chain_h(nc), 3.0, nt, 0.2, ntau, 0.2)
    for key in got:
        np.testing.assert_allclose(got[key], Gc[key], atol=1e-12, err_msg=key)


def test_four_step_cluster_components_at_u0_are_free_fermions():
    """The contour components the L-shaped CPT takes from the four-step
    (G^<, G^>, G^M(+-tau), both mixed functions) equal, at U = 0, the
    zero-temperature free-fermion functions of the one-particle Hamiltonian
    (H_ini on the imaginary branch, H on the real ones): the conventions of
    sign, order and branch of cluster_fn."""
    L = 4
    H = wl.chain_siam(L, 0.0, 1.0)
    Hi = H.with_field(0, 0.2)
    sec = basis.Sector(L, 2, 2)
    orbs = [(i, 0) for i in range(L)]
    nt, dtg, ntau, dtau = 5, 0.2, 6, 0.3
    out = greens.four_step(Hi, H, 2, 2, orbs, nt, dtg, 2, 15, wl.start_vector(sec.dim, 7), gs_tol=1e-13,
                           ntau=ntau, dtau_grid=dtau, tau_steps_per_grid=3)

    def one_particle(M):
        h = np.diag(np.asarray(M.eps_up, float))
        for (i, j), t in zip(M.bonds, M.t):
            h[i, j] -= t
            h[j, i] -= t
        return h
    e = np.linalg.eigvalsh(one_particle(Hi))
    assert (e < 0).sum() == 2 and np.abs(e).min() > 0.1          # two occupied levels, no zero level
    ref = necpt.free_greens_l(one_particle(Hi), one_particle(H), np.inf, nt, dtg, ntau, dtau)
    got = necpt.cluster_fn(out)
    for key in ref:
        assert np.abs(got[key] - ref[key]).max() < 1e-10, key


def test_kms_completed_ground_state_functions_are_thermal():
    """The cluster's zero-temperature components completed for an imaginary
    branch of length beta (cluster_fn_kms) equal the thermal functions at
    beta up to terms e^{-beta Delta}: at U = 0 (free fermions: the four-step
    replaced by the exact zero-temperature components) the difference falls
    from 1e-3 at beta = 15 to below 1e-5 at beta = 30; and the CPT equation
    fed with them reproduces the connected system's thermal densities."""
    nc, nb, V, dt, nt = 6, 12, 1.0, 0.1, 2
    eps = np.zeros(nc)
    eps[0] = -0.2
    hc_ini, hc, Tb = _chain_h(nc, 1.0, eps), _chain_h(nc), _chain_h(nb)
    for beta, bound in ((15.0, 2e-3), (30.0, 1e-5)):
        dtau = 0.1
        ntau = int(round(beta / dtau)) + 1
        t0 = necpt.free_greens_l(hc_ini, hc, np.inf, nt, dt, ntau, dtau)
        GM = np.stack([-1j * t0["vert_greater"], -1j * t0["vert_lesser"]])
        fake = {"G_lesser": t0["lesser"], "G_greater": t0["greater"], "G_mixed": t0["mixed"],
                "G_mixed_left": t0["mixed_left"], "G_matsubara": GM}
        got = necpt.cluster_fn_kms(fake)
        ref = necpt.free_greens_l(hc_ini, hc, beta, nt, dt, ntau, dtau)
        err = max(np.abs(got[k] - ref[k]).max() for k in ref)
        assert err < bound, (beta, err)
        plain = necpt.cluster_fn(fake)
        assert max(np.abs(plain[k] - ref[k]).max() for k in ("vert_greater", "mixed")) > 0.1   # the completion matters
    # the connected densities through the CPT equation (beta = 30)
    Gb = necpt.bath_greens_l(Tb, nt, dt, ntau, dtau, beta, sites=[0])
    res = necpt.necpt_l(got, Gb, nc - 1, V, dt, dtau)
    h = np.zeros((nc + nb, nc + nb))
    h[:nc, :nc], h[nc:, nc:] = hc_ini, Tb
    h[nc - 1, nc] = h[nc, nc - 1] = -V
    hf = h.copy()
    hf[:nc, :nc] = hc
    ex = necpt.free_greens_l(h, hf, beta, nt, dt, 2, dtau)
    n_got = np.real(-1j * np.diag(res["lesser"][0, 0]))
    n_ex = np.real(-1j * np.diag(ex["lesser"][0, 0]))[:nc]
    assert np.abs(n_got - n_ex).max() < 2e-4
