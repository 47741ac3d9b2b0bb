"""Second-quantised operators restricted to one sector.

Test infrastructure (see the package docstring).

The Hamiltonians are the Hubbard model of Sec. 3 and the Anderson model of
Sec. 4 (Eq. of the SIAM chain, with the local field of Eq. (hfi)), written
with site-resolved parameters:

    H = - sum_b t_b sum_sigma (c^+_{i sigma} c_{j sigma} + c^+_{j sigma} c_{i sigma})
        + sum_{i sigma} eps_{i sigma} n_{i sigma} + sum_i U_i n_{i up} n_{i dn}

Fermionic signs follow from the definition of the operators on the
ordered product state
    |s_up, s_dn> = prod_{i in s_up, ascending} c^+_{i up}
                   prod_{j in s_dn, ascending} c^+_{j dn} |vac>,
i.e. the modes are ordered (0 up, ..., L-1 up, 0 dn, ..., L-1 dn).  An
annihilator/creator on mode p picks up (-1)^(number of occupied modes
before p).  Every sign below is obtained by applying the operators one at a
time with that rule (no closed-form shortcut), and the result is pinned in
the tests against Jordan-Wigner matrices in the full Fock space.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .basis import Sector, popcount


def _occupied_before(up: int, dn: int, L: int, site: int, spin: int) -> int:
    """Number of occupied modes preceding mode (site, spin) in the ordering
    (0 up .. L-1 up, 0 dn .. L-1 dn)."""
    below = (1 << site) - 1
    if spin == 0:
        return popcount(up & below)
    return popcount(up) + popcount(dn & below)


def annihilate(up: int, dn: int, L: int, site: int, spin: int):
    """c_{site,spin}|up,dn>  ->  (sign, up', dn') or None if empty."""
    mask = up if spin == 0 else dn
    if not (mask >> site) & 1:
        return None
    sign = -1 if _occupied_before(up, dn, L, site, spin) % 2 else 1
    if spin == 0:
        return sign, up ^ (1 << site), dn
    return sign, up, dn ^ (1 << site)


def create(up: int, dn: int, L: int, site: int, spin: int):
    """c^+_{site,spin}|up,dn>  ->  (sign, up', dn') or None if occupied."""
    mask = up if spin == 0 else dn
    if (mask >> site) & 1:
        return None
    sign = -1 if _occupied_before(up, dn, L, site, spin) % 2 else 1
    if spin == 0:
        return sign, up | (1 << site), dn
    return sign, up, dn | (1 << site)


def hop(up: int, dn: int, L: int, i: int, j: int, spin: int):
    """c^+_{i spin} c_{j spin} |up,dn> -> (sign, up', dn') or None."""
    r = annihilate(up, dn, L, j, spin)
    if r is None:
        return None
    s1, u1, d1 = r
    r = create(u1, d1, L, i, spin)
    if r is None:
        return None
    s2, u2, d2 = r
    return s1 * s2, u2, d2


def hopping_matrix(L: int, states: np.ndarray, bonds, t, spin: int) -> sp.csr_matrix:
    """Single-species hopping matrix T_sigma with entries
    <s|H_hop|s'> for masks of one spin, the other species empty.

    For a same-species hop the other species contributes the factor
    (-1)^(2 N_other) = 1, so this matrix acts on either index of the
    D_up x D_dn state matrix."""
    rank = {int(s): r for r, s in enumerate(states)}
    rows, cols, vals = [], [], []
    for col, s in enumerate(states):
        s = int(s)
        for b, (i, j) in enumerate(bonds):
            for (a, c) in ((i, j), (j, i)):
                if spin == 0:
                    r = hop(s, 0, L, a, c, 0)
                    if r is None:
                        continue
                    sign, s2, _ = r
                else:
                    r = hop(0, s, L, a, c, 1)
                    if r is None:
                        continue
                    sign, _, s2 = r
                rows.append(rank[s2])
                cols.append(col)
                vals.append(-float(t[b]) * sign)
    D = len(states)
    return sp.csr_matrix((vals, (rows, cols)), shape=(D, D))


def occupation_bits(states: np.ndarray, L: int) -> np.ndarray:
    """[D, L] 0/1 matrix of site occupations."""
    return ((states[:, None] >> np.arange(L)[None, :]) & 1).astype(np.float64)


class Hamiltonian:
    """H restricted to one sector, applied to flat complex vectors of length
    D_up*D_dn (up-major), as T_up V + V T_dn^T + d o V."""

    def __init__(self, model, sector: Sector):
        bonds, t, eps_up, eps_dn, U = model.arrays()
        self.model = model
        self.sector = sector
        L = sector.L
        assert model.L == L
        self.T_up = hopping_matrix(L, sector.up, bonds, t, 0)
        self.T_dn = hopping_matrix(L, sector.dn, bonds, t, 1)
        bu = occupation_bits(sector.up, L)
        bd = occupation_bits(sector.dn, L)
        e_up = bu @ eps_up
        e_dn = bd @ eps_dn
        self.diag = e_up[:, None] + e_dn[None, :] + (bu * U[None, :]) @ bd.T

    @property
    def dim(self) -> int:
        return self.sector.dim

    def apply(self, v: np.ndarray) -> np.ndarray:
        V = np.asarray(v).reshape(self.sector.d_up, self.sector.d_dn)
        W = self.T_up @ V + (self.T_dn @ V.T).T + self.diag * V
        return W.reshape(-1)

    def apply_rows(self, v: np.ndarray, rows) -> np.ndarray:
        """Rows u (up-spin indices) of H.v viewed as the D_up x D_dn matrix,
        from the same three terms as apply(): for checking a product at
        sizes where the full one is too slow."""
        V = np.asarray(v).reshape(self.sector.d_up, self.sector.d_dn)
        rows = np.asarray(rows, dtype=np.int64)
        return self.T_up[rows] @ V + V[rows] @ self.T_dn.T + self.diag[rows] * V[rows]

    def sparse(self) -> sp.csr_matrix:
        Iu = sp.identity(self.sector.d_up, format="csr")
        Id = sp.identity(self.sector.d_dn, format="csr")
        H = sp.kron(self.T_up, Id) + sp.kron(Iu, self.T_dn) + sp.diags(self.diag.reshape(-1))
        return H.tocsr()

    def dense(self) -> np.ndarray:
        return self.sparse().toarray()


def ladder_operator(sector: Sector, site: int, spin: int, dagger: bool):
    """Sparse matrix of c_{site,spin} (dagger=False) or c^+_{site,spin}
    from `sector` to the neighbouring sector; returns (matrix, target)."""
    L = sector.L
    target = sector.shifted(spin, +1 if dagger else -1)
    rows, cols, vals = [], [], []
    if target.dim == 0:
        return sp.csr_matrix((0, sector.dim)), target
    for iu, up in enumerate(sector.up):
        for idn, dn in enumerate(sector.dn):
            f = create if dagger else annihilate
            r = f(int(up), int(dn), L, site, spin)
            if r is None:
                continue
            sign, u2, d2 = r
            rows.append(target.rank_up[u2] * target.d_dn + target.rank_dn[d2])
            cols.append(iu * sector.d_dn + idn)
            vals.append(float(sign))
    M = sp.csr_matrix((vals, (rows, cols)), shape=(target.dim, sector.dim))
    return M, target


def apply_ladder(sector: Sector, site: int, spin: int, dagger: bool, v: np.ndarray):
    """c_alpha v or c^+_alpha v for a flat sector vector (vectorised form of
    ladder_operator, used on large sectors).  Returns (w, target sector)."""
    L = sector.L
    target = sector.shifted(spin, +1 if dagger else -1)
    V = np.asarray(v).reshape(sector.d_up, sector.d_dn)
    W = np.zeros((target.d_up, target.d_dn), dtype=np.complex128)
    if target.dim == 0:
        return W.reshape(-1), target
    below = (1 << site) - 1
    if spin == 0:
        src = sector.up
        occ = (src >> site) & 1
        keep = occ == (0 if dagger else 1)
        new = src ^ (1 << site)
        par = np.array([popcount(int(s) & below) for s in src]) % 2
        sign = np.where(par == 1, -1.0, 1.0)
        idx = np.searchsorted(target.up, new[keep])
        W[idx, :] = sign[keep][:, None] * V[keep, :]
    else:
        src = sector.dn
        occ = (src >> site) & 1
        keep = occ == (0 if dagger else 1)
        new = src ^ (1 << site)
        par = (np.array([popcount(int(s) & below) for s in src]) + sector.n_up) % 2
        sign = np.where(par == 1, -1.0, 1.0)
        idx = np.searchsorted(target.dn, new[keep])
        W[:, idx] = sign[keep][None, :] * V[:, keep]
    return W.reshape(-1), target
