"""Occupation-number basis of one (N_up, N_dn) sector.

Test infrastructure (see the package docstring).

The paper works in the occupation-number basis |n_1, n_2, ...> (Sec. 2,
discussion after Eq. (tmatrix)) and uses conservation of the particle
number and of S_z to restrict H to one sector (Sec. 4, comparison with full
diagonalisation).  It does not fix an ordering; the reading used here:

* one spin species: an L-bit mask, bit i = occupation of site i; the masks
  with N set bits are listed in ascending numeric order;
* the sector basis is the product up x dn with composite index
  i_up * D_dn + i_dn (up-major), i.e. a state vector is a D_up x D_dn
  row-major matrix.

The enumeration below is brute force over all 2^L masks (independent of
any combinatorial ranking formula).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict

import numpy as np


def popcount(x: int) -> int:
    return bin(int(x)).count("1")


def spin_states(L: int, N: int) -> np.ndarray:
    """All L-bit masks with N bits set, ascending (brute-force scan)."""
    if N < 0 or N > L:
        return np.zeros(0, dtype=np.int64)
    return np.array([m for m in range(1 << L) if popcount(m) == N], dtype=np.int64)


def rank_table(states: np.ndarray) -> Dict[int, int]:
    """mask -> position in the ascending list (dictionary lookup)."""
    return {int(s): r for r, s in enumerate(states)}


@dataclass
class Sector:
    L: int
    n_up: int
    n_dn: int

    def __post_init__(self):
        self.up = spin_states(self.L, self.n_up)
        self.dn = spin_states(self.L, self.n_dn)
        self.rank_up = rank_table(self.up)
        self.rank_dn = rank_table(self.dn)

    @property
    def d_up(self) -> int:
        return len(self.up)

    @property
    def d_dn(self) -> int:
        return len(self.dn)

    @property
    def dim(self) -> int:
        return self.d_up * self.d_dn

    def states(self, spin: int) -> np.ndarray:
        return self.up if spin == 0 else self.dn

    def shifted(self, spin: int, delta: int) -> "Sector":
        """The sector reached by adding `delta` particles of `spin`."""
        if spin == 0:
            return Sector(self.L, self.n_up + delta, self.n_dn)
        return Sector(self.L, self.n_up, self.n_dn + delta)
