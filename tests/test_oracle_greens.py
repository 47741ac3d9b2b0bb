"""Pins of the oracle's Green's functions (CPU only).

References: the exact definitions evaluated by full diagonalisation in
each sector, the U = 0 single-particle closed form, the anticommutator,
Hermiticity, particle-number sum rule, time-translation invariance in
equilibrium, particle-hole symmetry, and the facts the paper states for
its worked examples (tests/golden/paper_facts.json)."""
import json
import os

import numpy as np
import pytest

import workloads as wl
from oracle import basis, exact, greens, hamiltonian, lanczos

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")


def _dense(model, sec):
    return exact.DenseSector(hamiltonian.Hamiltonian(model, sec).dense())


def _exact_four_step(H_ini, H, nu, nd, orbitals, times, taus=()):
    """Definitions of Sec. 4 evaluated with full diagonalisation."""
    L = H.L
    sec = basis.Sector(L, nu, nd)
    E0, psi0 = _dense(H_ini, sec).ground()
    Dfin = {}

    def D(model, s, cache):
        key = (id(model), s.n_up, s.n_dn)
        if key not in cache:
            cache[key] = _dense(model, s)
        return cache[key]

    no, nt = len(orbitals), len(times)
    Gl = np.zeros((nt, nt, no, no), complex)
    Gg = np.zeros((nt, nt, no, no), complex)
    phis = [D(H, sec, Dfin).apply_exp(psi0, t) for t in times]
    Psi, Chi = {}, {}
    for a, (site, spin) in enumerate(orbitals):
        for k, t in enumerate(times):
            w, tgt = hamiltonian.apply_ladder(sec, site, spin, False, phis[k])
            Psi[a, k] = (D(H, tgt, Dfin).apply_exp(w, -t), spin)
            w, tgt = hamiltonian.apply_ladder(sec, site, spin, True, phis[k])
            Chi[a, k] = (D(H, tgt, Dfin).apply_exp(w, -t), spin)
    for a in range(no):
        for b in range(no):
            for k in range(nt):
                for kp in range(nt):
                    if Psi[a, k][1] == Psi[b, kp][1]:
                        Gl[k, kp, a, b] = 1j * np.vdot(Psi[b, kp][0], Psi[a, k][0])
                        Gg[k, kp, a, b] = -1j * np.vdot(Chi[a, k][0], Chi[b, kp][0])
    out = {"G_lesser": Gl, "G_greater": Gg, "E0": E0}
    if len(taus):
        cache = {}
        GM = np.zeros((2, len(taus), no, no), complex)
        Gmix = np.zeros((nt, len(taus), no, no), complex)
        Gmixl = np.zeros((len(taus), nt, no, no), complex)
        for a, (sa, spa) in enumerate(orbitals):
            for b, (sb, spb) in enumerate(orbitals):
                if spa != spb:
                    continue
                ca_d, tp = hamiltonian.apply_ladder(sec, sa, spa, True, psi0)
                cb_d, _ = hamiltonian.apply_ladder(sec, sb, spb, True, psi0)
                ca, th = hamiltonian.apply_ladder(sec, sa, spa, False, psi0)
                cb, _ = hamiltonian.apply_ladder(sec, sb, spb, False, psi0)
                Dp, Dh = D(H_ini, tp, cache), D(H_ini, th, cache)
                for j, tau in enumerate(taus):
                    GM[0, j, a, b] = -np.exp(E0 * tau) * np.vdot(ca_d, Dp.apply_exp(cb_d, -1j * tau))
                    GM[1, j, a, b] = np.exp(E0 * tau) * np.vdot(cb, Dh.apply_exp(ca, -1j * tau))
                    phi_b = np.exp(E0 * tau) * Dh.apply_exp(cb, -1j * tau)
                    phi_a = np.exp(E0 * tau) * Dp.apply_exp(ca_d, -1j * tau)
                    for k in range(nt):
                        Gmix[k, j, a, b] = 1j * np.vdot(phi_b, Psi[a, k][0])
                        # -i <0| c_a e^{-(H_ini-E0) tau} e^{iHt} c+_b e^{-iHt} |0>
                        Gmixl[j, k, a, b] = -1j * np.vdot(phi_a, Chi[b, k][0])
        out["G_matsubara"] = GM
        out["G_mixed"] = Gmix
        out["G_mixed_left"] = Gmixl
    return out


def test_equilibrium_against_full_diagonalisation():
    model = wl.ring(6, 1.0, 4.0)
    sec = basis.Sector(6, 3, 3)
    H = hamiltonian.Hamiltonian(model, sec)
    gs = lanczos.ground_state(H.apply, wl.start_vector(H.dim, 7), tol=1e-13)
    orbs = [(i, 0) for i in range(6)]
    nt, dtg = 21, 0.1
    Gg, Gl = greens.equilibrium(model, 3, 3, orbs, nt, dtg, 2, 15, gs.psi, gs.E0)
    E0, psi0 = _dense(model, sec).ground()
    Dp = _dense(model, sec.shifted(0, +1))
    Dh = _dense(model, sec.shifted(0, -1))
    x = [hamiltonian.apply_ladder(sec, s, sp, True, psi0)[0] for s, sp in orbs]
    y = [hamiltonian.apply_ladder(sec, s, sp, False, psi0)[0] for s, sp in orbs]
    for k in range(nt):
        t = k * dtg
        xt = [Dp.apply_exp(v, t) for v in x]
        yt = [Dh.apply_exp(v, -t) for v in y]
        for i in range(len(orbs)):
            for j in range(len(orbs)):
                ref = -1j * np.exp(1j * E0 * t) * np.vdot(x[i], xt[j])
                assert abs(Gg[k, i, j] - ref) < 1e-11
                ref = 1j * np.exp(-1j * E0 * t) * np.vdot(y[j], yt[i])
                assert abs(Gl[k, i, j] - ref) < 1e-11


@pytest.fixture(scope="module")
def quench_small():
    H = wl.chain_siam(5, 2.0)
    H_ini = H.with_field(0, 0.4)
    orbs = [(0, 0), (1, 0), (0, 1)]
    nt, dtg, spg = 8, 0.25, 3
    ntau, dtau, tspg = 5, 0.3, 2
    sec = basis.Sector(5, 3, 2)
    v0 = wl.start_vector(sec.dim, 7)
    ora = greens.four_step(H_ini, H, 3, 2, orbs, nt, dtg, spg, 15, v0, gs_tol=1e-13,
                           ntau=ntau, dtau_grid=dtau, tau_steps_per_grid=tspg)
    ref = _exact_four_step(H_ini, H, 3, 2, orbs, np.arange(nt) * dtg, np.arange(ntau) * dtau)
    return ora, ref, orbs


def test_four_step_against_full_diagonalisation(quench_small):
    ora, ref, _ = quench_small
    assert abs(ora["E0"] - ref["E0"]) < 1e-12 * abs(ref["E0"])
    for key in ("G_lesser", "G_greater", "G_matsubara", "G_mixed", "G_mixed_left"):
        err = np.abs(ora[key] - ref[key]).max()
        assert err < 1e-11, (key, err)


def test_anticommutator_and_hermiticity(quench_small):
    ora, _, orbs = quench_small
    Gl, Gg = ora["G_lesser"], ora["G_greater"]
    nt, no = Gl.shape[0], Gl.shape[2]
    for k in range(nt):
        for a in range(no):
            for b in range(no):
                want = -1j if a == b else 0.0
                assert abs(Gg[k, k, a, b] - Gl[k, k, a, b] - want) < 1e-12
    # G^<_{ab}(t,t')^* = -G^<_{ba}(t',t), same for G^>
    np.testing.assert_allclose(Gl.conj(), -Gl.transpose(1, 0, 3, 2), atol=1e-13)
    np.testing.assert_allclose(Gg.conj(), -Gg.transpose(1, 0, 3, 2), atol=1e-13)


def test_particle_number_sum_rule():
    """n_{i sigma}(t) = -i G^<_{ii sigma}(t,t) (Sec. 5) summed over sites is
    N_sigma at every t; sum_i m_i = N_up - N_dn."""
    H = wl.ring(5, 1.0, 3.0, periodic=False)
    H_ini = H.with_field(2, 0.5)
    orbs = [(i, s) for s in (0, 1) for i in range(5)]
    sec = basis.Sector(5, 3, 2)
    o = greens.four_step(H_ini, H, 3, 2, orbs, 5, 0.4, 4, 15, wl.start_vector(sec.dim, 7))
    for k in range(5):
        n = (-1j * np.array([o["G_lesser"][k, k, a, a] for a in range(10)])).real
        assert abs(n[:5].sum() - 3) < 1e-12 and abs(n[5:].sum() - 2) < 1e-12


def test_equilibrium_time_translation_invariance():
    H = wl.star_siam([0.5, -0.4, 1.2, -1.1], [0.3, 0.4, 0.25, 0.35], 2.0, -1.0)
    sec = basis.Sector(5, 3, 2)
    o = greens.four_step(H, H, 3, 2, [(0, 0)], 6, 0.3, 2, 15, wl.start_vector(sec.dim, 7))
    Gl = o["G_lesser"][:, :, 0, 0]
    for d in range(-5, 6):
        diag = np.array([Gl[k, k - d] for k in range(6) if 0 <= k - d < 6])
        assert np.abs(diag - diag[0]).max() < 1e-11


def test_noninteracting_quench_closed_form():
    """U = 0: quench of bath energies and a field on a star, against the
    single-particle exponential (Eqs. (gb1), (gb2) at beta -> infinity)."""
    H = wl.star_siam([0.5, -0.4, 1.2, -1.1, 0.2], [0.3, 0.4, 0.25, 0.35, 0.5], 0.0, 0.1)
    H_ini = wl.star_siam([0.1, -0.9, 0.8, -0.3, 0.6], [0.3, 0.4, 0.25, 0.35, 0.5], 0.0, 0.1).with_field(0, 0.3)
    orbs = [(i, 0) for i in range(6)]
    sec = basis.Sector(6, 3, 3)
    nt, dtg = 6, 0.4
    o = greens.four_step(H_ini, H, 3, 3, orbs, nt, dtg, 4, 15, wl.start_vector(sec.dim, 7), gs_tol=1e-13)
    Gl, Gg = exact.free_greens(H_ini, H, 0, 3, np.arange(nt) * dtg)
    assert np.abs(o["G_lesser"] - Gl).max() < 1e-11
    assert np.abs(o["G_greater"] - Gg).max() < 1e-11


def test_particle_hole_symmetry_half_filled_ring():
    """Bipartite ring at half filling, no field: G^>_ii(t) =
    e^{-iUt} conj(G^<_ii(t)) (chemical potential U/2 shifts the phase)."""
    U = 3.0
    model = wl.ring(6, 1.0, U)
    sec = basis.Sector(6, 3, 3)
    H = hamiltonian.Hamiltonian(model, sec)
    gs = lanczos.ground_state(H.apply, wl.start_vector(H.dim, 7), tol=1e-13)
    nt, dtg = 11, 0.2
    Gg, Gl = greens.equilibrium(model, 3, 3, [(0, 0)], nt, dtg, 2, 15, gs.psi, gs.E0)
    t = np.arange(nt) * dtg
    np.testing.assert_allclose(Gg[:, 0, 0], np.exp(-1j * U * t) * Gl[:, 0, 0].conj(), atol=1e-11)


def _paper_model(spec):
    m = spec["model"]
    assert m["geometry"] == "chain_siam"
    H = wl.chain_siam(m["L"], m["U"], m["T"])
    return H, H.with_field(m["field_site"], m["field_h"])


def test_paper_fig2_equal_time_anticommutator():
    spec = json.load(open(GOLDEN))["fig2_siam_chain"]
    H, H_ini = _paper_model(spec)
    nu, nd = spec["sector"]
    sec = basis.Sector(H.L, nu, nd)
    o = greens.four_step(H_ini, H, nu, nd, [(0, 0)], 1, 0.1, 1, 15, wl.start_vector(sec.dim, 7),
                         gs_tol=1e-13)
    gl, gg = o["G_lesser"][0, 0, 0, 0], o["G_greater"][0, 0, 0, 0]
    c = spec["claims"]
    assert abs((gl.imag - gg.imag) - c["im_Gless_minus_im_Ggtr_at_00"]) < 1e-12
    assert abs(gl.real - c["re_Gless_at_00"]) < 1e-12 and abs(gg.real - c["re_Ggtr_at_00"]) < 1e-12
    # Im G^<(0,0) = <n_{1 up}>, from the ground-state vector directly
    bu = hamiltonian.occupation_bits(sec.up, H.L)[:, 0]
    n_imp = float(np.sum(np.abs(o["psi0"].reshape(sec.d_up, sec.d_dn)) ** 2 * bu[:, None]))
    assert abs(gl.imag - n_imp) < 1e-12


@pytest.mark.parametrize("key", ["fig4_moments", "lc4_isolated_cluster"])
def test_paper_total_polarisation(key):
    spec = json.load(open(GOLDEN))[key]
    H, H_ini = _paper_model(spec)
    nu, nd = spec["sector"]
    L = H.L
    sec = basis.Sector(L, nu, nd)
    orbs = [(i, s) for s in (0, 1) for i in range(L)]
    o = greens.four_step(H_ini, H, nu, nd, orbs, 1, 0.1, 1, 15, wl.start_vector(sec.dim, 7), gs_tol=1e-13)
    n = (-1j * np.array([o["G_lesser"][0, 0, a, a] for a in range(2 * L)])).real
    m = n[:L] - n[L:]
    c = spec["claims"]
    assert abs(m.sum() - c["sum_moments_t0"]) < 1e-12
    if c.get("impurity_moment_positive"):
        assert m[0] > 0.05
    k = c.get("moments_alternate_near_impurity", 0)
    for i in range(k - 1):
        assert m[i] * m[i + 1] < 0


def _moments(sec, L, psi):
    """m_i = <n_i,up> - <n_i,dn> of a sector vector (row-major D_up x D_dn)."""
    p = np.abs(psi.reshape(sec.d_up, sec.d_dn)) ** 2
    bu = hamiltonian.occupation_bits(sec.up, L)
    bd = hamiltonian.occupation_bits(sec.dn, L)
    return (p.sum(1)[:, None] * bu).sum(0) - (p.sum(0)[:, None] * bd).sum(0)


def test_paper_fig4_dynamics():
    """The time dependence the paper states for the isolated L_c = 8 cluster
    after the field is switched off, with the oracle's SIL propagation
    (which equals -i G^<_ii(t,t) of the four-step; tested elsewhere)."""
    from oracle import lanczos, propagate
    spec = json.load(open(GOLDEN))["fig4_dynamics"]
    H, H_ini = _paper_model(spec)
    nu, nd = spec["sector"]
    L = H.L
    sec = basis.Sector(L, nu, nd)
    Hi, Hf = hamiltonian.Hamiltonian(H_ini, sec), hamiltonian.Hamiltonian(H, sec)
    gs = lanczos.ground_state(Hi.apply, wl.start_vector(sec.dim, 7), tol=1e-13, max_iter=400)
    psi = gs.psi.astype(complex)
    ms = [_moments(sec, L, psi)]
    for _ in range(110):   # t = 0.1 k, k <= 110
        psi = propagate.propagate(Hf.apply, psi, 0.1, 1, 15, -1, 0.0, "cgs2")
        ms.append(_moments(sec, L, psi))
    ms = np.array(ms)
    t = 0.1 * np.arange(len(ms))
    c = spec["claims"]
    assert np.abs(ms.sum(1)).max() < 1e-12
    assert ms[t <= c["impurity_half_decay_before"] + 1e-9, 0].min() < 0.5 * ms[0, 0]
    win = (t >= 1.0) & (t <= 11.0 + 1e-9)
    k = np.argmax(np.where(win, ms[:, 0], -np.inf))
    assert c["revival_window"][0] <= t[k] <= c["revival_window"][1] and ms[k, 0] > 0.5 * ms[0, 0]
    e = c["edge_maximum"]
    assert np.argmax(ms[int(round(e["t"] / 0.1))]) + 1 == e["site"]
    # one Krylov space over the whole interval (Eq. (udelta) with dt = t)
    sk = c["single_krylov_space"]
    dev = []
    for n in sk["dims"]:
        d = 0.0
        for kk in range(5, 101, 5):
            p = propagate.sil_step(Hf.apply, gs.psi.astype(complex), 0.1 * kk, n, -1, 0.0, "cgs2")
            d = max(d, float(np.abs(_moments(sec, L, p) - ms[kk]).max()))
        dev.append(d)
    assert all(dev[i + 1] < dev[i] for i in range(len(dev) - 1)) and dev[-1] < sk["converged_tol"]
