"""Driven Hamiltonians (test infrastructure only; the product path never
imports this module).

H(t) = sum_j f_j(t) H_j, with H_j the Hamiltonian of parameter vector
theta_j = (t_b, eps_up, eps_dn, U) on one bond list (H is linear in theta),
propagated by the fourth-order commutator-free exponential integrator with
two exponentials per step, the class of method the paper's outlook (Sec. 6)
proposes for driven systems (its reference [AF11]).  On a step [t, t + h]
with Gauss-Legendre nodes t_1,2 = t + (1/2 -+ sqrt(3)/6) h:

    U(t + h, t) = exp(-i h B_2) exp(-i h B_1),
    B_1 = a_2 H(t_1) + a_1 H(t_2),   B_2 = a_1 H(t_1) + a_2 H(t_2),
    a_1,2 = 1/4 -+ sqrt(3)/6.

Each exponential is taken either exactly (dense matrix exponential) or by
the oracle's short-iterative-Lanczos step of dimension m (Eqs. (newstate),
(udelta)), the form the GPU path evaluates.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import propagate
from .gradients import model_with_theta, theta_of
from .hamiltonian import Hamiltonian

C1, C2 = 0.5 - np.sqrt(3.0) / 6.0, 0.5 + np.sqrt(3.0) / 6.0
A1, A2 = 0.25 - np.sqrt(3.0) / 6.0, 0.25 + np.sqrt(3.0) / 6.0


def stage_thetas(thetas: np.ndarray, f, t: float, h: float):
    """Parameter vectors of B_1 and B_2 for the step starting at t."""
    f1 = np.asarray(f(t + C1 * h), dtype=np.float64).reshape(-1)
    f2 = np.asarray(f(t + C2 * h), dtype=np.float64).reshape(-1)
    return (A2 * f1 + A1 * f2) @ thetas, (A1 * f1 + A2 * f2) @ thetas


def cfm4(template, sector, thetas, f, psi, t0: float, h: float, nsteps: int, m: int | None = None,
         reorth: str = "cgs2") -> np.ndarray:
    """psi(t0) -> psi(t0 + nsteps h).  m = None: exact exponentials of each
    stage; else SIL steps of Krylov dimension m."""
    th = np.asarray(thetas, dtype=np.float64).reshape(-1, len(theta_of(template)))
    out = np.asarray(psi, dtype=np.complex128).copy()
    for n in range(nsteps):
        for theta in stage_thetas(th, f, t0 + n * h, h):
            H = Hamiltonian(model_with_theta(template, theta), sector)
            if m is None:
                out = scipy.linalg.expm(-1j * h * H.dense()) @ out
            else:
                out = propagate.sil_step(H.apply, out, h, m, -1, 0.0, reorth)
    return out


def four_step(H_ini, template, thetas, f, n_up: int, n_dn: int, orbitals, nt: int, dt_grid: float,
              steps_per_grid: int, m: int, v0: np.ndarray, gs_tol: float = 1e-12, gs_max_iter: int = 400,
              reorth: str = "cgs2"):
    """The four-step procedure of Sec. 4 with a driven final Hamiltonian:
    (i) |0> = ground state of H_ini; (ii) Phi(t_k) = U(t_k, 0)|0> with the
    integrator above, t_k = k dt_grid (driven steps of h = dt_grid /
    steps_per_grid from t = 0); (iii) Psi_a(t_k) = U(t_k, 0)^+ c_a Phi(t_k)
    and chi_a(t_k) = U(t_k, 0)^+ c_a^+ Phi(t_k), where U^+ applies the
    adjoint stage exponentials exp(+i h B) in reverse order; (iv)
    G^<_ab(t, t') = i <Psi_b(t')|Psi_a(t)>, G^>_ab(t, t') = -i <chi_a(t)|chi_b(t')>.
    Returns G_lesser, G_greater [nt, nt, n_orb, n_orb] and E0."""
    from .basis import Sector
    from .hamiltonian import apply_ladder
    from .lanczos import ground_state

    sec = Sector(template.L, n_up, n_dn)
    th = np.asarray(thetas, dtype=np.float64).reshape(-1, len(theta_of(template)))
    h = dt_grid / steps_per_grid
    nsteps = (nt - 1) * steps_per_grid
    stages = [stage_thetas(th, f, n * h, h) for n in range(nsteps)]
    cache = {}

    def ham(n, s, sector):
        key = (n, s, sector.n_up, sector.n_dn)
        if key not in cache:
            cache[key] = Hamiltonian(model_with_theta(template, stages[n][s]), sector)
        return cache[key]

    gs = ground_state(Hamiltonian(H_ini, sec).apply, v0, tol=gs_tol, max_iter=gs_max_iter, reorth=reorth)
    phis = [np.asarray(gs.psi, dtype=np.complex128)]
    for k in range(1, nt):
        psi = phis[-1]
        for n in range((k - 1) * steps_per_grid, k * steps_per_grid):
            for s in (0, 1):
                psi = propagate.sil_step(ham(n, s, sec).apply, psi, h, m, -1, 0.0, reorth)
        phis.append(psi)
    no = len(orbitals)
    Gl = np.zeros((nt, nt, no, no), dtype=np.complex128)
    Gg = np.zeros((nt, nt, no, no), dtype=np.complex128)
    for dagger, G in ((0, Gl), (1, Gg)):
        P = {}
        for a, (site, spin) in enumerate(orbitals):
            for k in range(nt):
                v, tgt = apply_ladder(sec, site, spin, bool(dagger), phis[k])
                if tgt.dim == 0:
                    P[(k, a)] = (v, spin)
                    continue
                for n in range(k * steps_per_grid - 1, -1, -1):
                    for s in (1, 0):
                        v = propagate.sil_step(ham(n, s, tgt).apply, v, h, m, +1, 0.0, reorth)
                P[(k, a)] = (v, spin)
        for j in range(nt):
            for s_ in range(nt):
                for a in range(no):
                    for b in range(no):
                        va, sa = P[(j, a)]
                        vb, sb = P[(s_, b)]
                        if sa != sb:
                            continue
                        G[j, s_, a, b] = 1j * np.vdot(vb, va) if dagger == 0 else -1j * np.vdot(va, vb)
    return {"G_lesser": Gl, "G_greater": Gg, "E0": gs.E0}
