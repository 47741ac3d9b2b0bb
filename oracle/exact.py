"""Dense references used to pin the Krylov oracle.

Test infrastructure (see the package docstring).

* Jordan-Wigner construction of c_p in the full 4^L Fock space (modes
  ordered 0 up .. L-1 up, 0 dn .. L-1 dn, mode 0 the leftmost Kronecker
  factor).  It shares no sign logic with `hamiltonian`.
* Full diagonalisation inside a sector, the comparison method of Sec. 4
  (all eigenstates), giving exp(-iHt) and the Green's functions by
  eigen-decomposition.
* The U = 0 closed form: with a quadratic H the operators evolve with the
  single-particle matrix h (the bath Green's function of Eqs. (gb1), (gb2)
  at beta -> infinity is this form), so
      G^<_{ij}(t,t') = +i [e^{-iht} rho e^{+iht'}]_{ij},
      G^>_{ij}(t,t') = -i [e^{-iht} (1-rho) e^{+iht'}]_{ij},
  with rho_{kl} = <c^+_l c_k> of the ground state of h_ini.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np
import scipy.sparse as sp

from .basis import Sector


# ----------------------------------------------------------------------------
# Jordan-Wigner Fock space
# ----------------------------------------------------------------------------
def jw_annihilators(L: int):
    """List of 2L sparse matrices c_p acting on the 4^L Fock space."""
    n = 2 * L
    a = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))   # |1> -> |0>
    Z = sp.csr_matrix(np.diag([1.0, -1.0]))
    I = sp.identity(2, format="csr")
    ops = []
    for p in range(n):
        m = sp.identity(1, format="csr")
        for q in range(n):
            f = Z if q < p else (a if q == p else I)
            m = sp.kron(m, f, format="csr")
        ops.append(m)
    return ops


def mode(site: int, spin: int, L: int) -> int:
    return site + (L if spin else 0)


def fock_index(up: int, dn: int, L: int) -> int:
    """Kronecker-basis index of the product state |up, dn> (mode 0 leftmost)."""
    idx = 0
    n = 2 * L
    for p in range(n):
        occ = (up >> p) & 1 if p < L else (dn >> (p - L)) & 1
        if occ:
            idx |= 1 << (n - 1 - p)
    return idx


def jw_hamiltonian(model, cs=None):
    bonds, t, eps_up, eps_dn, U = model.arrays()
    L = model.L
    cs = jw_annihilators(L) if cs is None else cs
    dim = 4 ** L
    H = sp.csr_matrix((dim, dim))
    for b, (i, j) in enumerate(bonds):
        for s in (0, 1):
            ci, cj = cs[mode(i, s, L)], cs[mode(j, s, L)]
            H = H - t[b] * (ci.T @ cj + cj.T @ ci)
    for i in range(L):
        nu = cs[mode(i, 0, L)].T @ cs[mode(i, 0, L)]
        nd = cs[mode(i, 1, L)].T @ cs[mode(i, 1, L)]
        H = H + eps_up[i] * nu + eps_dn[i] * nd + U[i] * (nu @ nd)
    return H.tocsr()


def sector_projector(sector: Sector) -> sp.csr_matrix:
    """Columns = Fock vectors of the sector basis in its own order."""
    L = sector.L
    rows = [fock_index(int(u), int(d), L) for u in sector.up for d in sector.dn]
    cols = np.arange(len(rows))
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(4 ** L, len(rows)))


# ----------------------------------------------------------------------------
# full diagonalisation in a sector
# ----------------------------------------------------------------------------
class DenseSector:
    """All eigenpairs of H in one sector (Sec. 4 full-diagonalisation)."""

    def __init__(self, Hdense: np.ndarray):
        self.H = Hdense
        self.w, self.U = np.linalg.eigh(Hdense)

    def expm(self, t: complex) -> np.ndarray:
        """exp(-i H t) for real t; exp(-H tau) via t = -i tau."""
        return (self.U * np.exp(-1j * self.w * t)) @ self.U.conj().T

    def apply_exp(self, v: np.ndarray, t: complex) -> np.ndarray:
        return self.U @ (np.exp(-1j * self.w * t) * (self.U.conj().T @ v))

    def ground(self):
        return self.w[0], self.U[:, 0]


def single_particle_h(model, spin: int) -> np.ndarray:
    bonds, t, eps_up, eps_dn, U = model.arrays()
    L = model.L
    h = np.diag(eps_up if spin == 0 else eps_dn).astype(np.float64)
    for b, (i, j) in enumerate(bonds):
        h[i, j] -= t[b]
        h[j, i] -= t[b]
    return h


def free_density(model, spin: int, N: int) -> np.ndarray:
    """rho_{kl} = <c^+_l c_k> in the N-particle ground state of h."""
    h = single_particle_h(model, spin)
    w, phi = np.linalg.eigh(h)
    occ = phi[:, :N]
    return occ @ occ.conj().T


def free_greens(H_ini_model, H_model, spin: int, N: int, times: Sequence[float]):
    """U = 0 closed form of G^<_{ij}(t,t') and G^>_{ij}(t,t') for all
    site pairs: arrays [nt, nt, L, L]."""
    rho = free_density(H_ini_model, spin, N)   # rho[k,l] = <c+_l c_k>
    h = single_particle_h(H_model, spin)
    w, phi = np.linalg.eigh(h)
    Ls = H_model.L
    ev = [(phi * np.exp(-1j * w * t)) @ phi.conj().T for t in times]
    nt = len(times)
    Gl = np.zeros((nt, nt, Ls, Ls), dtype=np.complex128)
    Gg = np.zeros((nt, nt, Ls, Ls), dtype=np.complex128)
    one = np.eye(Ls)
    for a in range(nt):
        for b in range(nt):
            Gl[a, b] = 1j * ev[a] @ rho @ ev[b].conj().T
            Gg[a, b] = -1j * ev[a] @ (one - rho) @ ev[b].conj().T
    return Gl, Gg
