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
