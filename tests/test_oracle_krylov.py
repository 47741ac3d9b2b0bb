"""Pins of the oracle's Lanczos recursion, ground state and SIL step.

References: the paper's literal unnormalised recursion (retyped from its
definition, then compared coefficient by coefficient), the exact moment
identity of the Krylov tridiagonal matrix, dense diagonalisation / matrix
exponentials, ARPACK, the continued-fraction form of the conventional
Lanczos Green's function, Hellmann-Feynman."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as wl
from oracle import basis, exact, hamiltonian, lanczos, propagate


def _ham(model, nu, nd):
    return hamiltonian.Hamiltonian(model, basis.Sector(model.L, nu, nd))


def test_normalised_recursion_equals_paper_unnormalised_form():
    """Eq. (recursion) with unnormalised |i_k>, a_k = <i_k|H|i_k>/<i_k|i_k>,
    b_k^2 = <i_k|i_k>/<i_{k-1}|i_{k-1}>, gives the same (a_k, b_k^2)."""
    H = _ham(wl.ring(6, 1.0, 4.0), 3, 3)
    v0 = wl.complex_vector(H.dim, 3, normalise=False)
    n = 8
    K = lanczos.lanczos(H.apply, v0, n, reorth="none")
    prev, cur = np.zeros_like(v0), v0.copy()
    b2 = 0.0
    for k in range(n):
        Hi = H.apply(cur)
        ak = (np.vdot(cur, Hi) / np.vdot(cur, cur)).real
        assert abs(ak - K.a[k]) < 1e-12 * max(1, abs(ak))
        if k > 0:
            assert abs(b2 - K.b[k] ** 2) < 1e-11 * b2
        nxt = Hi - ak * cur - b2 * prev
        b2 = (np.vdot(nxt, nxt) / np.vdot(cur, cur)).real
        prev, cur = cur, nxt


def test_tmatrix_is_projection_and_basis_orthonormal():
    """Eq. (tmatrix): T = V^+ H V, with V^+ V = 1."""
    H = _ham(wl.star_siam([0.3, -0.5, 1.1, 0.2, -1.4], [0.4, 0.2, -0.3, 0.3, 0.25], 3.0, -1.5), 3, 3)
    v0 = wl.complex_vector(H.dim, 5)
    K = lanczos.lanczos(H.apply, v0, 20, reorth="cgs2")
    V = np.stack(K.V, axis=1)
    np.testing.assert_allclose(V.conj().T @ V, np.eye(K.n), atol=1e-13)
    HV = np.stack([H.apply(v) for v in K.V], axis=1)
    np.testing.assert_allclose(V.conj().T @ HV, K.T(), atol=1e-12)


@pytest.mark.parametrize("m", [4, 7, 10])
def test_moments_exact_through_2m_minus_1(m):
    """e_1^T T^r e_1 beta0^2 = <i0|H^r|i0> for r <= 2m-1 (Gauss quadrature
    property behind the moment statement of Sec. 2; the paper's 'first n'
    is a lower bound) and not for r = 2m."""
    H = _ham(wl.ring(6, 1.0, 4.0), 3, 3)
    Hd = H.dense()
    x = wl.complex_vector(H.dim, 9, normalise=False)
    K = lanczos.lanczos(H.apply, x, m, reorth="cgs2")
    T = K.T()
    e = np.zeros(m); e[0] = 1.0
    Tr, Hr = e.copy(), x.copy()
    for r in range(0, 2 * m + 1):
        lhs = K.beta0 ** 2 * Tr[0]
        rhs = np.vdot(x, Hr).real
        scale = max(1.0, abs(rhs))
        if r <= 2 * m - 1:
            assert abs(lhs - rhs) < 1e-13 * scale, r
        else:
            assert abs(lhs - rhs) > 1e-10 * scale
        Tr = T @ Tr
        Hr = Hd @ Hr


@pytest.mark.parametrize("case", ["ring6", "siam_field", "rect_tp"])
def test_ground_state_against_dense(case):
    if case == "ring6":
        model, nu, nd = wl.ring(6, 1.0, 4.0), 3, 3
    elif case == "siam_field":
        model, nu, nd = wl.chain_siam(6, 1.0).with_field(0, 0.2), 3, 3
    else:
        model, nu, nd = wl.rect(3, 2, 1.0, -0.3, 8.0), 3, 3
    H = _ham(model, nu, nd)
    w, U = np.linalg.eigh(H.dense())
    gs = lanczos.ground_state(H.apply, wl.start_vector(H.dim, 7), tol=1e-12, max_iter=300)
    assert gs.converged
    assert abs(gs.E0 - w[0]) < 1e-12 * abs(w[0])
    assert abs(abs(np.vdot(U[:, 0], gs.psi)) - 1) < 1e-12
    r = np.linalg.norm(H.apply(gs.psi) - gs.E0 * gs.psi)
    assert r < 1e-10


def test_ground_state_ring8_against_arpack_and_two_starts():
    H = _ham(wl.ring(8, 1.0, 4.0), 4, 4)
    ev, evec = spla.eigsh(H.sparse(), k=2, which="SA", tol=1e-14)
    gs7 = lanczos.ground_state(H.apply, wl.start_vector(H.dim, 7), tol=1e-12)
    gs8 = lanczos.ground_state(H.apply, wl.start_vector(H.dim, 8), tol=1e-12)
    assert abs(gs7.E0 - ev[0]) < 1e-12 * abs(ev[0])
    assert lanczos.fidelity(gs7.psi, gs8.psi) > 1 - 1e-10
    assert ev[1] - ev[0] > 1e-3        # nondegenerate (gap)


def test_hellmann_feynman_double_occupancy():
    """dE0/dU = <0| sum_i n_up n_dn |0> (central finite difference)."""
    def e0(U):
        H = _ham(wl.ring(6, 1.0, U), 3, 3)
        return lanczos.ground_state(H.apply, wl.start_vector(H.dim, 7), tol=1e-13).E0
    U, h = 4.0, 1e-4
    fd = (e0(U + h) - e0(U - h)) / (2 * h)
    H = _ham(wl.ring(6, 1.0, U), 3, 3)
    gs = lanczos.ground_state(H.apply, wl.start_vector(H.dim, 7), tol=1e-13)
    sec = H.sector
    bu = hamiltonian.occupation_bits(sec.up, 6)
    bd = hamiltonian.occupation_bits(sec.dn, 6)
    dbl = (bu @ bd.T).reshape(-1)
    ref = float(np.sum(np.abs(gs.psi) ** 2 * dbl))
    assert abs(fd - ref) < 1e-7


@pytest.mark.parametrize("direction", [-1, +1, 0])
def test_sil_step_against_dense_exponential(direction):
    H = _ham(wl.chain_siam(6, 2.0).with_field(0, 0.3), 3, 2)
    D = exact.DenseSector(H.dense())
    psi = wl.complex_vector(H.dim, 4)
    dt, shift = 0.05, -1.7
    got = propagate.sil_step(H.apply, psi, dt, 15, direction, shift=shift)
    if direction == 0:
        ref = np.exp(shift * dt) * D.apply_exp(psi, -1j * dt)
    else:
        ref = D.apply_exp(psi, -direction * dt)
    assert np.linalg.norm(got - ref) < 1e-13


def test_sil_many_steps_norm_and_exactness():
    H = _ham(wl.ring(6, 1.0, 4.0), 3, 3)
    D = exact.DenseSector(H.dense())
    psi = wl.complex_vector(H.dim, 5)
    out = propagate.propagate(H.apply, psi, 0.05, 200, 15, -1)
    assert abs(np.linalg.norm(out) - 1) < 1e-12
    assert np.linalg.norm(out - D.apply_exp(psi, 10.0)) < 1e-11


def test_sil_convergence_in_krylov_dim():
    H = _ham(wl.ring(6, 1.0, 4.0), 3, 3)
    D = exact.DenseSector(H.dense())
    psi = wl.complex_vector(H.dim, 6)
    ref = D.apply_exp(psi, 0.2)
    errs = [np.linalg.norm(propagate.sil_step(H.apply, psi, 0.2, m, -1) - ref) for m in (4, 6, 8, 10, 20)]
    assert all(errs[i + 1] < errs[i] for i in range(4))
    assert errs[-1] < 1e-13


def test_sil_breakdown_is_exact():
    """Krylov dimension above the sector dimension: the recursion stops at
    an invariant subspace and the step is exact (b_k -> 0)."""
    H = _ham(wl.ring(3, 1.0, 2.0, periodic=False), 1, 2)    # dim 9
    D = exact.DenseSector(H.dense())
    psi = wl.complex_vector(H.dim, 1)
    K = lanczos.lanczos(H.apply, psi, 15)
    assert K.breakdown and K.n <= H.dim
    got = propagate.sil_step(H.apply, psi, 1.3, 15, -1)
    assert np.linalg.norm(got - D.apply_exp(psi, 1.3)) < 1e-12


def test_single_krylov_space_equals_conventional_lanczos():
    """f = 1 (Eq. (res)): the time-dependent Lanczos G(t) from one Krylov
    space is the Fourier transform of the n-pole G^(L)(omega) of
    Eq. (gapprox); checked through the continued fraction of T."""
    H = _ham(wl.ring(6, 1.0, 4.0), 3, 3)
    gs = lanczos.ground_state(H.apply, wl.start_vector(H.dim, 7), tol=1e-12)
    sec = H.sector
    x, tgt = hamiltonian.apply_ladder(sec, 0, 0, True, gs.psi)
    Ht = hamiltonian.Hamiltonian(H.model, tgt)
    n = 12
    K = lanczos.lanczos(Ht.apply, x, n)
    eta = 0.3
    lam, Q = propagate.tridiag_eig(K)
    w = K.beta0 ** 2 * Q[0, :] ** 2
    # time domain: <x| V c(t)> from the SIL machinery equals Eq. (res)
    for t in (0.0, 0.7, 3.1, 25.0):
        state = propagate.combine(K, propagate.krylov_coefficients(K, t, -1))
        assert abs(np.vdot(x, state) - np.sum(w * np.exp(-1j * lam * t))) < 1e-12
    # frequency domain: the pole sum is the continued fraction of T
    for omega in (-2.0, 0.5, 3.0, 7.5):
        z = omega + 1j * eta + gs.E0
        g = 0.0
        for k in reversed(range(K.n)):
            g = 1.0 / (z - K.a[k] - (K.b[k + 1] ** 2) * g) if k + 1 < K.n else 1.0 / (z - K.a[k])
        g_cf = K.beta0 ** 2 * g
        g_poles = np.sum(w / (z - lam))
        assert abs(g_cf - g_poles) < 1e-12 * abs(g_cf)
