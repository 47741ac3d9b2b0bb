"""Pins of the driven-Hamiltonian oracle (fourth-order commutator-free
exponential integrator, the method the paper's outlook proposes for driven
systems, Sec. 6) against facts that do not depend on it:

* a constant drive is propagated exactly (the two stages add up to exp(-iHh));
* a drive that commutes with the rest (the number of up electrons, a
  constant in a sector) enters through the integral of f, which the two
  Gauss nodes give exactly for a cubic f;
* a non-commuting drive converges with order four (halving h divides the
  error by ~16);
* the Krylov (SIL) form agrees with the exact exponentials, and the norm is
  conserved."""
import numpy as np
import pytest
import scipy.linalg

import workloads as wl
from oracle import basis, driven, hamiltonian
from oracle.gradients import model_with_theta, theta_of


def _ring(L=6, U=2.0):
    return wl.ring(L, 1.0, U, periodic=True)


def _zero_theta(model):
    return np.zeros(len(theta_of(model)))


def _one_bond_theta(model, b=0):
    th = _zero_theta(model)
    th[b] = 1.0
    return th


def test_constant_drive_is_exact():
    H0 = _ring()
    sec = basis.Sector(H0.L, 3, 3)
    th0, th1 = theta_of(H0), _one_bond_theta(H0, 2)
    psi = wl.complex_vector(sec.dim, 3)
    h, n = 0.3, 5
    got = driven.cfm4(H0, sec, [th0, th1], lambda t: [1.0, 0.7], psi, 0.0, h, n)
    Hd = hamiltonian.Hamiltonian(model_with_theta(H0, th0 + 0.7 * th1), sec).dense()
    ref = scipy.linalg.expm(-1j * h * n * Hd) @ psi
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_commuting_cubic_drive_is_integrated_exactly():
    H0 = _ring()
    sec = basis.Sector(H0.L, 3, 3)
    L, nb = H0.L, len(H0.bonds)
    thN = _zero_theta(H0)
    thN[nb:nb + L] = 1.0             # eps_up = 1 on every site: N_up, = 3 in this sector
    f = lambda t: [1.0, 1.0 + 0.5 * t - 0.3 * t ** 2 + 0.1 * t ** 3]
    F = lambda T: T + 0.25 * T ** 2 - 0.1 * T ** 3 + 0.025 * T ** 4
    psi = wl.complex_vector(sec.dim, 4)
    h, n = 0.4, 6
    got = driven.cfm4(H0, sec, [theta_of(H0), thN], f, psi, 0.0, h, n)
    T = h * n
    ref = scipy.linalg.expm(-1j * T * hamiltonian.Hamiltonian(H0, sec).dense()) @ psi * np.exp(-1j * 3 * F(T))
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_fourth_order_convergence():
    """Error ratio ~17 when h halves (with the two stages' weights swapped
    the scheme drops to second order: ratio ~4)."""
    H0 = _ring(4)
    sec = basis.Sector(H0.L, 2, 2)
    ths = [theta_of(H0), _one_bond_theta(H0, 0)]
    f = lambda t: [1.0, 0.8 * np.sin(2.0 * t)]
    psi = wl.complex_vector(sec.dim, 5)
    T = 1.6
    ref = driven.cfm4(H0, sec, ths, f, psi, 0.0, T / 128, 128)
    err = []
    for n in (8, 16):
        got = driven.cfm4(H0, sec, ths, f, psi, 0.0, T / n, n)
        err.append(np.abs(got - ref).max())
    ratio = err[0] / err[1]
    assert 12.0 < ratio < 20.0, (err, ratio)


@pytest.mark.parametrize("reorth", ["cgs2", "none"])
def test_krylov_stages_match_exact_and_conserve_norm(reorth):
    H0 = _ring()
    sec = basis.Sector(H0.L, 3, 3)
    ths = [theta_of(H0), _one_bond_theta(H0, 0), _one_bond_theta(H0, 3)]
    f = lambda t: [1.0, 0.8 * np.sin(2.0 * t), 0.5 * np.cos(t)]
    psi = wl.complex_vector(sec.dim, 6)
    exact = driven.cfm4(H0, sec, ths, f, psi, 0.1, 0.05, 10)
    kry = driven.cfm4(H0, sec, ths, f, psi, 0.1, 0.05, 10, m=15, reorth=reorth)
    assert np.abs(kry - exact).max() < 1e-12 * np.abs(exact).max()
    assert abs(np.linalg.norm(kry) - np.linalg.norm(psi)) < 1e-12 * np.linalg.norm(psi)


def _chain_siam_pair(L=4, U=1.0, h=0.2):
    H = wl.chain_siam(L, U, 1.0)
    return H, H.with_field(0, h)


def test_driven_four_step_with_constant_drive_is_the_static_four_step():
    """A constant drive: the driven four-step equals the static one (Sec. 4)
    with H = sum_j f_j H_j."""
    from oracle import greens
    H, H_ini = _chain_siam_pair()
    L, nb = H.L, len(H.bonds)
    k0 = np.zeros(nb + 3 * L)
    k0[1] = 1.0
    f = lambda t: [1.0, 0.4]
    orbs = [(0, 0), (1, 0), (0, 1)]
    sec = basis.Sector(L, 2, 2)
    v0 = wl.start_vector(sec.dim, 7)
    got = driven.four_step(H_ini, H, [theta_of(H), k0], f, 2, 2, orbs, 5, 0.2, 2, 15, v0, gs_tol=1e-13)
    Hs = model_with_theta(H, theta_of(H) + 0.4 * k0)
    ref = greens.four_step(H_ini, Hs, 2, 2, orbs, 5, 0.2, 2, 15, v0, gs_tol=1e-13)
    for key in ("G_lesser", "G_greater"):
        assert np.abs(got[key] - ref[key]).max() < 1e-11 * np.abs(ref[key]).max()


def test_driven_four_step_commuting_drive_is_a_phase():
    """H(t) = H + f(t) N_up with N_up constant on a sector: for up-spin
    orbitals G^<(t,t') and G^>(t,t') pick up exp(-i (F(t) - F(t'))), F = the
    integral of f (cubic f: integrated exactly); down-spin ones are unchanged."""
    from oracle import greens
    H, H_ini = _chain_siam_pair()
    L, nb = H.L, len(H.bonds)
    thN = np.zeros(nb + 3 * L)
    thN[nb:nb + L] = 1.0
    f = lambda t: [1.0, 0.5 + t - 0.4 * t ** 2 + 0.2 * t ** 3]
    F = lambda t: 0.5 * t + 0.5 * t ** 2 - 0.4 / 3 * t ** 3 + 0.05 * t ** 4
    orbs = [(0, 0), (2, 0), (1, 1)]
    sec = basis.Sector(L, 2, 2)
    v0 = wl.start_vector(sec.dim, 7)
    nt, dtg, spg = 5, 0.25, 2
    got = driven.four_step(H_ini, H, [theta_of(H), thN], f, 2, 2, orbs, nt, dtg, spg, 15, v0, gs_tol=1e-13)
    ref = greens.four_step(H_ini, H, 2, 2, orbs, nt, dtg, spg, 15, v0, gs_tol=1e-13)
    t = dtg * np.arange(nt)
    ph = np.exp(-1j * (F(t)[:, None] - F(t)[None, :]))
    for key in ("G_lesser", "G_greater"):
        r = ref[key].copy()
        for a, (_, sa) in enumerate(orbs):
            for b, (_, sb) in enumerate(orbs):
                if sa == 0 and sb == 0:
                    r[:, :, a, b] *= ph
        assert np.abs(got[key] - r).max() < 1e-11 * np.abs(r).max()
