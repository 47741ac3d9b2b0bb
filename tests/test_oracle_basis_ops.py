"""Pins of the oracle's basis and operators (CPU only).

Each check compares against something other than the oracle itself:
binomial counts, the combinatorial-number-system closed form of the
position of a mask, Jordan-Wigner matrices in the full Fock space (no
shared sign logic), textbook closed forms (two-site Hubbard dimer, U = 0
spectra)."""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as wl
from oracle import basis, exact, hamiltonian


@pytest.mark.parametrize("L", range(1, 13))
def test_sector_counts_and_order(L):
    for N in range(L + 1):
        s = basis.spin_states(L, N)
        assert len(s) == math.comb(L, N)
        assert np.all(np.diff(s) > 0)
        # position = sum_k C(p_k, k) over set bits p_1 < p_2 < ... (colex rank)
        for r, m in enumerate(s):
            bits = [p for p in range(L) if (int(m) >> p) & 1]
            assert sum(math.comb(p, k + 1) for k, p in enumerate(bits)) == r


def _models_small():
    yield wl.ring(4, 1.0, 3.0)
    yield wl.ring(3, 0.7, 2.0, periodic=False).with_field(0, 0.4)
    yield wl.star_siam([0.3, -0.5, 1.1], [0.4, 0.2, -0.3], 2.5, -1.25)
    yield wl.rect(2, 2, 1.0, -0.3, 4.0).with_field(1, 0.2)


@pytest.mark.parametrize("mi", range(4))
def test_sector_hamiltonian_matches_jordan_wigner(mi):
    model = list(_models_small())[mi]
    L = model.L
    cs = exact.jw_annihilators(L)
    Hf = exact.jw_hamiltonian(model, cs)
    for nu, nd in itertools.product(range(L + 1), repeat=2):
        sec = basis.Sector(L, nu, nd)
        P = exact.sector_projector(sec)
        ref = (P.T @ Hf @ P).toarray()
        got = hamiltonian.Hamiltonian(model, sec).dense()
        np.testing.assert_allclose(got, ref, atol=1e-14, rtol=0)
        # the Fock-space H does not couple the sector to the rest
        leak = Hf @ P - P @ (P.T @ Hf @ P)
        assert (abs(leak).max() if leak.nnz else 0.0) < 1e-14


@pytest.mark.parametrize("L", [3, 4])
def test_ladder_operators_match_jordan_wigner(L):
    cs = exact.jw_annihilators(L)
    rng = np.random.default_rng(11)
    for nu, nd in itertools.product(range(L + 1), repeat=2):
        sec = basis.Sector(L, nu, nd)
        P = exact.sector_projector(sec)
        for site in range(L):
            for spin in (0, 1):
                for dagger in (False, True):
                    M, tgt = hamiltonian.ladder_operator(sec, site, spin, dagger)
                    if tgt.dim == 0:
                        continue
                    Pt = exact.sector_projector(tgt)
                    c = cs[exact.mode(site, spin, L)]
                    op = c.T if dagger else c
                    ref = (Pt.T @ op @ P).toarray()
                    np.testing.assert_array_equal(M.toarray(), ref)
                    v = rng.standard_normal(sec.dim) + 1j * rng.standard_normal(sec.dim)
                    w, _ = hamiltonian.apply_ladder(sec, site, spin, dagger, v)
                    np.testing.assert_allclose(w, ref @ v, atol=1e-15)


def test_hermitian_and_apply_consistency():
    model = wl.rect(4, 3, 1.0, -0.3, 8.0)
    sec = basis.Sector(model.L, 3, 2)
    H = hamiltonian.Hamiltonian(model, sec)
    x = wl.complex_vector(sec.dim, 1)
    y = wl.complex_vector(sec.dim, 2)
    lhs = np.vdot(x, H.apply(y))
    rhs = np.vdot(H.apply(x), y)
    assert abs(lhs - rhs) < 1e-12
    np.testing.assert_allclose(H.apply(y), H.sparse() @ y, atol=1e-13)


def test_apply_rows_matches_assembled_matrix():
    """Row-sampled H.v equals the same rows of the Kronecker-assembled
    sparse matrix times the vector (non-square sector, site-dependent U)."""
    model = wl.siam10().H_ini
    sec = basis.Sector(model.L, 4, 6)
    H = hamiltonian.Hamiltonian(model, sec)
    y = wl.complex_vector(sec.dim, 3)
    full = (H.sparse() @ y).reshape(sec.d_up, sec.d_dn)
    rows = [0, 1, sec.d_up // 2, sec.d_up - 1]
    np.testing.assert_allclose(H.apply_rows(y, rows), full[rows], atol=1e-13)


@pytest.mark.parametrize("U", [0.0, 1.0, 4.0, 8.0])
def test_dimer_closed_form(U):
    t = 1.3
    model = wl.dimer(t, U)
    H = hamiltonian.Hamiltonian(model, basis.Sector(2, 1, 1)).dense()
    E0 = np.linalg.eigvalsh(H)[0]
    assert abs(E0 - (U / 2 - math.sqrt(U * U / 4 + 4 * t * t))) < 1e-13


def test_noninteracting_spectrum_is_sum_of_levels():
    model = wl.star_siam([0.3, -0.5, 1.1, 0.05], [0.4, 0.2, -0.3, 0.25], 0.0, -0.2).with_field(0, 0.3)
    L = model.L
    hu = exact.single_particle_h(model, 0)
    hd = exact.single_particle_h(model, 1)
    eu, ed = np.linalg.eigvalsh(hu), np.linalg.eigvalsh(hd)
    for nu, nd in [(2, 3), (3, 2), (1, 4)]:
        H = hamiltonian.Hamiltonian(model, basis.Sector(L, nu, nd)).dense()
        ev = np.sort(np.linalg.eigvalsh(H))
        ref = sorted(sum(eu[list(a)]) + sum(ed[list(b)])
                     for a in itertools.combinations(range(L), nu)
                     for b in itertools.combinations(range(L), nd))
        np.testing.assert_allclose(ev, ref, atol=1e-12)


def test_atomic_limit_is_diagonal():
    model = wl.ring(6, 0.0, 3.0).with_field(2, 0.5)
    sec = basis.Sector(6, 3, 2)
    H = hamiltonian.Hamiltonian(model, sec)
    assert H.T_up.count_nonzero() == 0 and H.T_dn.count_nonzero() == 0
    # energy = U * doubly occupied + field term, counted by hand
    for iu, u in enumerate(sec.up):
        for idn, d in enumerate(sec.dn):
            dbl = bin(int(u) & int(d)).count("1")
            f = -0.5 * ((int(u) >> 2) & 1) + 0.5 * ((int(d) >> 2) & 1)
            assert abs(H.diag[iu, idn] - (3.0 * dbl + f)) < 1e-15


def test_ring8_ground_energy_against_arpack():
    """The half-filled L=8 ring (dim 4,900): a library eigensolver on the
    oracle's sparse H and on an independently assembled Fock-space H agree."""
    model = wl.ring(8, 1.0, 4.0)
    sec = basis.Sector(8, 4, 4)
    H = hamiltonian.Hamiltonian(model, sec)
    e_sector = spla.eigsh(H.sparse(), k=1, which="SA", tol=1e-14)[0][0]
    # the same sector assembled from the JW Fock-space operators
    L = 8
    cs = exact.jw_annihilators(L)
    Hf = exact.jw_hamiltonian(model, cs)
    P = exact.sector_projector(sec)
    e_jw = spla.eigsh((P.T @ Hf @ P).tocsr(), k=1, which="SA", tol=1e-14)[0][0]
    assert abs(e_sector - e_jw) < 1e-12
