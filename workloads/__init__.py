"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only *describes* problems: lattice geometries (bond lists),
model parameters drawn from seeded generators, sector fillings, time grids
and random start vectors.  It contains none of the method's arithmetic
(no basis, no Hamiltonian action, no Krylov step), so that the CPU oracle
and the GPU library can both consume it without sharing any computation.

Model convention (the Hubbard / Anderson Hamiltonians of the paper, Sec. 3
and Sec. 4, with site-resolved parameters):

    H = - sum_b t_b sum_sigma (c^+_{i_b sigma} c_{j_b sigma} + h.c.)
        + sum_{i sigma} eps_{i sigma} n_{i sigma}
        + sum_i U_i n_{i up} n_{i dn}

Each undirected bond appears once in ``bonds``; both hopping directions are
part of H.  The local field of Eq. (hfi), H_field = -h (n_{1 up} - n_{1 dn}),
is folded into eps_up / eps_dn of the initial-state Hamiltonian.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Model", "Quench", "ring", "chain_siam", "star_siam", "rect", "ladder",
    "start_vector", "complex_vector", "ring8", "siam10", "hub4x3",
    "batch_instances", "ladder14", "ladder16", "dimer",
]


@dataclass(frozen=True)
class Model:
    """Site-resolved parameters of one cluster Hamiltonian (see module doc)."""
    L: int
    bonds: Tuple[Tuple[int, int], ...]
    t: Tuple[float, ...]
    eps_up: Tuple[float, ...]
    eps_dn: Tuple[float, ...]
    U: Tuple[float, ...]
    name: str = ""

    def bond_array(self) -> np.ndarray:
        return np.asarray(self.bonds, dtype=np.int32).reshape(-1, 2)

    def arrays(self):
        """(bonds int32 [nb,2], t, eps_up, eps_dn, U) as float64 numpy arrays."""
        return (self.bond_array(), np.asarray(self.t, dtype=np.float64),
                np.asarray(self.eps_up, dtype=np.float64),
                np.asarray(self.eps_dn, dtype=np.float64),
                np.asarray(self.U, dtype=np.float64))

    def with_field(self, site: int, h: float) -> "Model":
        """Add H_field = -h (n_{site up} - n_{site dn}) (Eq. hfi, t<0 part)."""
        eu = list(self.eps_up)
        ed = list(self.eps_dn)
        eu[site] -= h
        ed[site] += h
        return replace(self, eps_up=tuple(eu), eps_dn=tuple(ed))

    def with_U(self, U) -> "Model":
        if np.isscalar(U):
            U = [float(U)] * self.L
        return replace(self, U=tuple(float(x) for x in U))


@dataclass(frozen=True)
class Quench:
    """A sudden switch H_ini -> H at t=0 plus the sector and contour grid."""
    H_ini: Model
    H: Model
    n_up: int
    n_dn: int
    nt: int                 # real-time grid points t_k = k * dt_grid, k=0..nt-1
    dt_grid: float
    steps_per_grid: int     # SIL steps per grid interval
    krylov_dim: int
    orbitals: Tuple[Tuple[int, int], ...] = ((0, 0),)   # (site, spin 0=up 1=dn)
    ntau: int = 0           # Matsubara grid tau_j = j * dtau_grid, j=0..ntau-1
    dtau_grid: float = 0.0
    tau_steps_per_grid: int = 1
    gs_tol: float = 1e-12
    gs_seed: int = 7
    name: str = ""

    @property
    def dt(self) -> float:
        return self.dt_grid / self.steps_per_grid


def _uniform(L, x):
    return tuple([float(x)] * L)


def _model(L, bonds, t, eps_up=None, eps_dn=None, U=0.0, name=""):
    bonds = tuple((int(i), int(j)) for i, j in bonds)
    if np.isscalar(t):
        t = [float(t)] * len(bonds)
    eps_up = _uniform(L, 0.0) if eps_up is None else tuple(float(x) for x in eps_up)
    eps_dn = eps_up if eps_dn is None else tuple(float(x) for x in eps_dn)
    Uv = _uniform(L, U) if np.isscalar(U) else tuple(float(x) for x in U)
    return Model(L=L, bonds=bonds, t=tuple(float(x) for x in t),
                 eps_up=eps_up, eps_dn=eps_dn, U=Uv, name=name)


# ----------------------------------------------------------------------------
# geometries
# ----------------------------------------------------------------------------
def ring(L: int, t: float = 1.0, U: float = 0.0, periodic: bool = True) -> Model:
    """1D Hubbard ring (Sec. 3 example geometry): bonds (i, i+1 mod L)."""
    nb = L if periodic else L - 1
    bonds = [(i, (i + 1) % L) for i in range(nb)]
    return _model(L, bonds, t, U=U, name=f"ring{L}")


def chain_siam(L: int, U: float, t: float = 1.0) -> Model:
    """Anderson impurity at site 0 of an open chain (Sec. 4 example):
    eps_imp = -U/2 on the impurity, U only on the impurity."""
    bonds = [(i, i + 1) for i in range(L - 1)]
    eps = [0.0] * L
    eps[0] = -U / 2.0
    Uv = [0.0] * L
    Uv[0] = U
    return _model(L, bonds, t, eps, eps, Uv, name=f"siam_chain{L}")


def star_siam(eps_bath, V_bath, U: float, eps_imp: float) -> Model:
    """Impurity site 0 hybridised with bath sites 1..L-1 (star geometry).

    The hybridisation term +V_k (c^+_0 c_k + h.c.) is written as a bond with
    t_b = -V_k in the convention H = -sum t_b (...)."""
    nb = len(eps_bath)
    L = nb + 1
    bonds = [(0, k + 1) for k in range(nb)]
    t = [-float(v) for v in V_bath]
    eps = [float(eps_imp)] + [float(e) for e in eps_bath]
    Uv = [float(U)] + [0.0] * nb
    return _model(L, bonds, t, eps, eps, Uv, name=f"siam_star{L}")


def rect(Lx: int, Ly: int, t: float = 1.0, tp: float = 0.0, U: float = 0.0) -> Model:
    """Open Lx x Ly cluster, site index i = x + Lx*y; nearest-neighbour
    bonds with amplitude t and both plaquette diagonals with amplitude tp."""
    def idx(x, y):
        return x + Lx * y
    bonds, ts = [], []
    for y in range(Ly):
        for x in range(Lx):
            if x + 1 < Lx:
                bonds.append((idx(x, y), idx(x + 1, y))); ts.append(t)
            if y + 1 < Ly:
                bonds.append((idx(x, y), idx(x, y + 1))); ts.append(t)
    if tp != 0.0:
        for y in range(Ly - 1):
            for x in range(Lx - 1):
                bonds.append((idx(x, y), idx(x + 1, y + 1))); ts.append(tp)
                bonds.append((idx(x + 1, y), idx(x, y + 1))); ts.append(tp)
    return _model(Lx * Ly, bonds, ts, U=U, name=f"rect{Lx}x{Ly}")


def ladder(Lx: int, t: float = 1.0, U: float = 0.0) -> Model:
    """Open two-leg ladder with Lx rungs, rung-major numbering i = 2x + y:
    rungs (2x, 2x+1), legs (2x+y, 2x+2+y)."""
    bonds = []
    for x in range(Lx):
        bonds.append((2 * x, 2 * x + 1))
        if x + 1 < Lx:
            bonds.append((2 * x, 2 * x + 2))
            bonds.append((2 * x + 1, 2 * x + 3))
    return _model(2 * Lx, bonds, t, U=U, name=f"ladder2x{Lx}")


def dimer(t: float = 1.0, U: float = 0.0) -> Model:
    return _model(2, [(0, 1)], t, U=U, name="dimer")


# ----------------------------------------------------------------------------
# seeded vectors
# ----------------------------------------------------------------------------
def start_vector(dim: int, seed: int) -> np.ndarray:
    """Lanczos start vector: real standard-normal entries from
    numpy default_rng(seed), normalised (complex128)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(dim)
    v /= np.linalg.norm(v)
    return v.astype(np.complex128)


def complex_vector(dim: int, seed: int, normalise: bool = True) -> np.ndarray:
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
    if normalise:
        v /= np.linalg.norm(v)
    return v


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
def ring8() -> Quench:
    """Plain equilibrium case: half-filled L=8 Hubbard ring, t=1, U=4
    (dim 4,900); G_ii(t) for all sites, 200 SIL steps of dt=0.05, m=15."""
    H = ring(8, 1.0, 4.0)
    orbs = tuple((i, 0) for i in range(8))
    return Quench(H_ini=H, H=H, n_up=4, n_dn=4, nt=201, dt_grid=0.05,
                  steps_per_grid=1, krylov_dim=15, orbitals=orbs, name="ring8")


def siam10(seed: int = 2) -> Quench:
    """Anderson impurity quench: impurity + 9 bath sites in a star, U=6,
    eps_imp=-U/2, bath energies uniform in [-2,2], hybridisations
    0.3+0.1 N(0,1) (drawn in that order from default_rng(seed)); field h=2
    on the impurity in H_ini, switched off at t=0.  Real-time grid
    t_k = 0.1 k (k<100) with 2 SIL steps per interval; Matsubara grid
    tau_j = 0.15 j (j<=100) with 3 imaginary-time steps per interval."""
    rng = np.random.default_rng(seed)
    eps_b = rng.uniform(-2.0, 2.0, 9)
    V_b = 0.3 + 0.1 * rng.standard_normal(9)
    U = 6.0
    H = star_siam(eps_b, V_b, U, -U / 2.0)
    H_ini = H.with_field(0, 2.0)
    return Quench(H_ini=H_ini, H=H, n_up=5, n_dn=5, nt=100, dt_grid=0.1,
                  steps_per_grid=2, krylov_dim=15, orbitals=((0, 0),),
                  ntau=101, dtau_grid=0.15, tau_steps_per_grid=3,
                  name="siam10")


def hub4x3() -> Quench:
    """Half-filled open 4x3 Hubbard cluster, t=1, t'=-0.3, U=8 (dim
    853,776); equilibrium, 400 SIL steps of dt=0.025 for all 12 spin-up
    c_i / c_i^+ components."""
    H = rect(4, 3, 1.0, -0.3, 8.0)
    orbs = tuple((i, 0) for i in range(12))
    return Quench(H_ini=H, H=H, n_up=6, n_dn=6, nt=401, dt_grid=0.025,
                  steps_per_grid=1, krylov_dim=15, orbitals=orbs, name="hub4x3")


def batch_instances(n: int = 64, U_final: float = 4.0, base_seed: int = 4000):
    """Uneven batch of Anderson star instances, instance i seeded with
    base_seed+i: L uniform in 8..12, then bath energies uniform in [-2,2]
    and hybridisations 0.3+0.1 N(0,1) (L-1 each).  Quench U: 0 -> U_final
    with eps_imp = -U_final/2 fixed; 50x50 grid t_k = 0.2 k, dt = 0.05."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(base_seed + i)
        L = int(rng.integers(8, 13))
        eps_b = rng.uniform(-2.0, 2.0, L - 1)
        V_b = 0.3 + 0.1 * rng.standard_normal(L - 1)
        H = star_siam(eps_b, V_b, U_final, -U_final / 2.0)
        H_ini = H.with_U([0.0] * L)
        out.append(Quench(H_ini=H_ini, H=H, n_up=(L + 1) // 2, n_dn=L // 2,
                          nt=50, dt_grid=0.2, steps_per_grid=4, krylov_dim=15,
                          orbitals=((0, 0),), name=f"batch{i}_L{L}"))
    return out


def ladder14() -> Quench:
    """2x7 open Hubbard ladder, t=1, half filling (dim 11,778,624), quench
    U: 4 -> 8 at t=0; Krylov dim 20, dt = 0.05, 100 steps: G_00(t,t') on a
    101 x 101 grid."""
    H_ini = ladder(7, 1.0, 4.0)
    H = ladder(7, 1.0, 8.0)
    return Quench(H_ini=H_ini, H=H, n_up=7, n_dn=7, nt=101, dt_grid=0.05,
                  steps_per_grid=1, krylov_dim=20, orbitals=((0, 0),),
                  name="ladder14")


def ladder16() -> Quench:
    """2x8 open Hubbard ladder, t=1, half filling (dim 165,636,900), quench
    U: 4 -> 8; Krylov dim 20, 100 steps of dt = 0.05."""
    H_ini = ladder(8, 1.0, 4.0)
    H = ladder(8, 1.0, 8.0)
    return Quench(H_ini=H_ini, H=H, n_up=8, n_dn=8, nt=101, dt_grid=0.05,
                  steps_per_grid=1, krylov_dim=20, orbitals=((0, 0),),
                  name="ladder16")
