"""Equilibrium and nonequilibrium single-particle Green's functions.

Test infrastructure (see the package docstring).

Equilibrium (Sec. 3, Eqs. (psit), (psigreen), eta = 0):
    G^>_{ij}(t) = -i e^{+i E0 t} <c^+_i 0| e^{-iHt} |c^+_j 0>
    G^<_{ij}(t) = +i e^{-i E0 t} <c_j 0| e^{+iHt} |c_i 0>
(the lesser form is Eq. (glesser) at t' = 0 with |0> an eigenstate).

Nonequilibrium, four-step procedure (Sec. 4):
  (i)   |0> = ground state of H_ini (Lanczos);
  (ii)  Phi(t_k) = e^{-iH t_k}|0> on the time mesh;
  (iii) Psi_a(t_k) = e^{+iH t_k} c_a Phi(t_k)  for every mesh time
        (and chi_a(t_k) = e^{+iH t_k} c^+_a Phi(t_k) for G^>);
  (iv)  G^<_{aa'}(t,t') = i <Psi_a'(t')|Psi_a(t)>,
        G^>_{aa'}(t,t') = -i <chi_a(t)|chi_a'(t')>.
The greater form is the one the text says is obtained "likewise"; it follows
from Eq. (gnon) with z later than z'.  The Matsubara component is the
equilibrium G of H_ini; at zero temperature (ground-state projection) the
reading used is
    G^M_{aa'}(+tau) = -<0| c_a e^{-(H_ini - E0) tau} c^+_a' |0>,
    G^M_{aa'}(-tau) = +<0| c^+_a' e^{-(H_ini - E0) tau} c_a |0>,  tau >= 0,
and the mixed component
    G^|_{aa'}(t, tau') = i <phi_a'(tau')|Psi_a(t)>,
    phi_a'(tau') = e^{-(H_ini - E0) tau'} c_a' |0>.
All propagations are restarted short-iterative-Lanczos steps (Sec. 3).
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

from .basis import Sector
from .hamiltonian import Hamiltonian, apply_ladder
from .lanczos import ground_state, vdot
from .propagate import sil_step


class _HamCache:
    """Hamiltonians per sector for one model."""

    def __init__(self, model):
        self.model = model
        self._c: Dict[Tuple[int, int], Hamiltonian] = {}

    def __call__(self, sec: Sector) -> Hamiltonian:
        key = (sec.n_up, sec.n_dn)
        if key not in self._c:
            self._c[key] = Hamiltonian(self.model, Sector(sec.L, sec.n_up, sec.n_dn))
        return self._c[key]


def equilibrium(model, n_up: int, n_dn: int, orbitals: Sequence[Tuple[int, int]],
                nt: int, dt_grid: float, steps_per_grid: int, m: int,
                psi0: np.ndarray, E0: float, reorth: str = "cgs2"):
    """G^>[k, i, j] and G^<[k, i, j] at t_k = k*dt_grid, k = 0..nt-1."""
    sec = Sector(model.L, n_up, n_dn)
    hams = _HamCache(model)
    no = len(orbitals)
    Gg = np.zeros((nt, no, no), dtype=np.complex128)
    Gl = np.zeros((nt, no, no), dtype=np.complex128)
    dt = dt_grid / steps_per_grid
    tk = np.arange(nt) * dt_grid
    for dagger, direction, G, pref in ((True, -1, Gg, -1j), (False, +1, Gl, +1j)):
        init = []
        for (site, spin) in orbitals:
            w, tgt = apply_ladder(sec, site, spin, dagger, psi0)
            init.append((w, tgt, spin))
        for j in range(no):
            wj, tgt, sj = init[j]
            if tgt.dim == 0:
                continue
            H = hams(tgt)
            state = wj.copy()
            for k in range(nt):
                if k > 0:
                    for _ in range(steps_per_grid):
                        state = sil_step(H.apply, state, dt, m, direction, reorth=reorth)
                for i in range(no):
                    wi, _, si = init[i]
                    if si != sj:
                        continue
                    ov = vdot(wi, state)
                    if dagger:   # G^>_{ij}(t) = -i e^{iE0 t} <c+_i 0|e^{-iHt}|c+_j 0>
                        G[k, i, j] = pref * np.exp(1j * E0 * tk[k]) * ov
                    else:        # G^<_{ji}(t) = i e^{-iE0 t} <c_i 0|e^{iHt}|c_j 0>
                        G[k, j, i] = pref * np.exp(-1j * E0 * tk[k]) * ov
    return Gg, Gl


def forward_states(H: Hamiltonian, psi0: np.ndarray, nt: int, steps_per_grid: int,
                   dt: float, m: int, reorth: str = "cgs2") -> List[np.ndarray]:
    """Step (ii): Phi(t_k) = e^{-iH t_k}|0> on the mesh."""
    phis = [psi0.copy()]
    state = psi0.copy()
    for _ in range(1, nt):
        for _ in range(steps_per_grid):
            state = sil_step(H.apply, state, dt, m, -1, reorth=reorth)
        phis.append(state.copy())
    return phis


def back_propagated(H: Hamiltonian, src: np.ndarray, k: int, steps_per_grid: int,
                    dt: float, m: int, reorth: str = "cgs2") -> np.ndarray:
    """Step (iii) for one mesh time: e^{+iH t_k} applied to c_a Phi(t_k)."""
    state = src.copy()
    for _ in range(k * steps_per_grid):
        state = sil_step(H.apply, state, dt, m, +1, reorth=reorth)
    return state


def imaginary_time_states(H: Hamiltonian, src: np.ndarray, ntau: int,
                          tau_steps_per_grid: int, dtau: float, E0: float, m: int,
                          reorth: str = "cgs2") -> List[np.ndarray]:
    """e^{-(H - E0) tau_j} src on the Matsubara mesh."""
    out = [src.copy()]
    state = src.copy()
    for _ in range(1, ntau):
        for _ in range(tau_steps_per_grid):
            state = sil_step(H.apply, state, dtau, m, 0, shift=E0, reorth=reorth)
        out.append(state.copy())
    return out


def four_step(H_ini_model, H_model, n_up: int, n_dn: int,
              orbitals: Sequence[Tuple[int, int]], nt: int, dt_grid: float,
              steps_per_grid: int, m: int, v0: np.ndarray, gs_tol: float = 1e-12,
              gs_max_iter: int = 400, reorth: str = "cgs2", ntau: int = 0,
              dtau_grid: float = 0.0, tau_steps_per_grid: int = 1,
              times: Sequence[int] = None, gs=None) -> Dict[str, np.ndarray]:
    """The four-step procedure of Sec. 4, literally: every mesh time gets
    its own backward propagation in step (iii).

    Returns G_lesser[k, k', a, a'] = G^<_{aa'}(t_k, t_k') and
    G_greater[k, k', a, a'] (both nt x nt x n_orb x n_orb), optionally
    G_matsubara[2, ntau, a, a'] (+tau and -tau parts) and
    G_mixed[k, j, a, a'] = G^|_{aa'}(t_k, tau_j) = G^<_{aa'}(t_k, -i tau_j) and
    G_mixed_left[j, k, a, a'] = G^|_{aa'}(tau_j, t_k) = G^>_{aa'}(-i tau_j, t_k)
    (the contour functions with one argument on the imaginary branch).
    `times` restricts step (iii)/(iv) to a subset of mesh indices (entries
    outside the subset are left at zero); the forward sweep (ii) still runs
    to the largest requested time."""
    sec = Sector(H_model.L, n_up, n_dn)
    ham_ini = _HamCache(H_ini_model)
    ham = _HamCache(H_model)
    dt = dt_grid / steps_per_grid
    if gs is None:
        gs = ground_state(ham_ini(sec).apply, v0, tol=gs_tol, max_iter=gs_max_iter, reorth=reorth)
    psi0, E0 = gs.psi, gs.E0
    idx = list(range(nt)) if times is None else sorted(set(int(t) for t in times))
    kmax = max(idx)
    phis = forward_states(ham(sec), psi0, kmax + 1, steps_per_grid, dt, m, reorth)
    no = len(orbitals)
    Gl = np.zeros((nt, nt, no, no), dtype=np.complex128)
    Gg = np.zeros((nt, nt, no, no), dtype=np.complex128)
    psi_l: Dict[Tuple[int, int], Tuple[np.ndarray, int]] = {}
    psi_g: Dict[Tuple[int, int], Tuple[np.ndarray, int]] = {}
    for a, (site, spin) in enumerate(orbitals):
        for k in idx:
            w, tgt = apply_ladder(sec, site, spin, False, phis[k])
            if tgt.dim:
                psi_l[(a, k)] = (back_propagated(ham(tgt), w, k, steps_per_grid, dt, m, reorth), spin)
            w, tgt = apply_ladder(sec, site, spin, True, phis[k])
            if tgt.dim:
                psi_g[(a, k)] = (back_propagated(ham(tgt), w, k, steps_per_grid, dt, m, reorth), spin)
    for a in range(no):
        for b in range(no):
            for k in idx:
                for kp in idx:
                    if (a, k) in psi_l and (b, kp) in psi_l:
                        x, sa = psi_l[(a, k)]
                        y, sb = psi_l[(b, kp)]
                        if sa == sb:
                            Gl[k, kp, a, b] = 1j * vdot(y, x)
                    if (a, k) in psi_g and (b, kp) in psi_g:
                        x, sa = psi_g[(a, k)]
                        y, sb = psi_g[(b, kp)]
                        if sa == sb:
                            Gg[k, kp, a, b] = -1j * vdot(x, y)
    out = {"G_lesser": Gl, "G_greater": Gg, "E0": E0, "psi0": psi0, "gs": gs}
    if ntau > 0:
        dtau = dtau_grid / tau_steps_per_grid
        GM = np.zeros((2, ntau, no, no), dtype=np.complex128)
        Gmix = np.zeros((nt, ntau, no, no), dtype=np.complex128)
        Gmixl = np.zeros((ntau, nt, no, no), dtype=np.complex128)
        part, hole = {}, {}
        for a, (site, spin) in enumerate(orbitals):
            w, tgt = apply_ladder(sec, site, spin, True, psi0)
            if tgt.dim:
                part[a] = (imaginary_time_states(ham_ini(tgt), w, ntau, tau_steps_per_grid,
                                                 dtau, E0, m, reorth), w, spin)
            w, tgt = apply_ladder(sec, site, spin, False, psi0)
            if tgt.dim:
                hole[a] = (imaginary_time_states(ham_ini(tgt), w, ntau, tau_steps_per_grid,
                                                 dtau, E0, m, reorth), w, spin)
        for a in range(no):
            for b in range(no):
                if b in part and a in part and part[a][2] == part[b][2]:
                    # -<c_a 0| e^{-(H-E0)tau} |c+_b 0>
                    for j in range(ntau):
                        GM[0, j, a, b] = -vdot(part[a][1], part[b][0][j])
                if a in hole and b in hole and hole[a][2] == hole[b][2]:
                    for j in range(ntau):
                        GM[1, j, a, b] = vdot(hole[b][1], hole[a][0][j])
                for j in range(ntau):
                    for k in idx:
                        # G^<(t_k, -i tau_j) = i <e^{-(H_ini-E0) tau_j} c_b 0 | Psi_a(t_k)>
                        if (a, k) in psi_l and b in hole and psi_l[(a, k)][1] == hole[b][2]:
                            Gmix[k, j, a, b] = 1j * vdot(hole[b][0][j], psi_l[(a, k)][0])
                        # G^>(-i tau_j, t_k) = -i <e^{-(H_ini-E0) tau_j} c+_a 0 | chi_b(t_k)>
                        if (b, k) in psi_g and a in part and psi_g[(b, k)][1] == part[a][2]:
                            Gmixl[j, k, a, b] = -1j * vdot(part[a][0][j], psi_g[(b, k)][0])
        out["G_matsubara"] = GM
        out["G_mixed"] = Gmix
        out["G_mixed_left"] = Gmixl
    return out
