"""Short-iterative-Lanczos (time-dependent Lanczos) propagation, Sec. 3.

Test infrastructure (see the package docstring).

For a short step dt the state exp(-iH dt)|Psi(t)> lies, to numerical
accuracy, in the Krylov space K_n(t) built from |i_0> = |Psi(t)>
(Eq. (newstate)); inside that space the propagator is
U exp(-i D dt) U^+ with D = Q^+ T Q and U = V Q (Eq. (udelta)).  Applied to
|Psi(t)> = beta0 v_0 this is
    Psi(t+dt) = beta0 * V Q exp(-i Lambda dt) Q^T e_1,
and restarting from the new state repeats the step (Sec. 3, restarts f).
The same Krylov space also gives the state at any intermediate time
s < dt (fine-grid evaluation, Sec. 3 after Fig. 1 and Sec. 4 step (iii)).

direction = -1 : exp(-i H dt)      (forward real time)
direction = +1 : exp(+i H dt)      (backward real time, step (iii))
direction =  0 : exp(-(H - shift) dt)  (imaginary time, Matsubara branch)
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal

from .lanczos import Krylov, lanczos


def tridiag_eig(K: Krylov):
    """Eq. (tdiag) for the Krylov tridiagonal T: eigenvalues and the
    orthogonal eigenvector matrix Q."""
    n = K.n
    if n == 1:
        return np.array([K.a[0]]), np.ones((1, 1))
    return eigh_tridiagonal(K.a, K.b[1:n])


def phase(lam: np.ndarray, s: float, direction: int, shift: float = 0.0) -> np.ndarray:
    if direction == -1:
        return np.exp(-1j * lam * s)
    if direction == +1:
        return np.exp(+1j * lam * s)
    if direction == 0:
        return np.exp(-(lam - shift) * s).astype(np.complex128)
    raise ValueError("direction must be -1, +1 or 0")


def krylov_coefficients(K: Krylov, s: float, direction: int, shift: float = 0.0) -> np.ndarray:
    """c = beta0 * Q f(Lambda, s) Q^T e_1, the coordinates of the propagated
    state in the Lanczos basis (Eq. (udelta) applied to beta0 v_0)."""
    lam, Q = tridiag_eig(K)
    return K.beta0 * (Q @ (phase(lam, s, direction, shift) * Q[0, :]))


def combine(K: Krylov, c: np.ndarray) -> np.ndarray:
    out = np.zeros_like(K.V[0])
    for k in range(len(c)):
        out = out + c[k] * K.V[k]
    return out


def sil_step(apply_h, psi: np.ndarray, dt: float, m: int, direction: int = -1,
             shift: float = 0.0, reorth: str = "cgs2",
             breakdown_tol: float = 1e-13) -> np.ndarray:
    """One restart of the time-dependent Lanczos method: psi -> f(H) psi."""
    if not np.any(psi):
        return np.zeros_like(psi)
    K = lanczos(apply_h, psi, m, reorth=reorth, breakdown_tol=breakdown_tol)
    return combine(K, krylov_coefficients(K, dt, direction, shift))


def sil_fine(apply_h, psi: np.ndarray, nodes, m: int, direction: int = -1,
             shift: float = 0.0, reorth: str = "cgs2") -> list:
    """States at several times s in one Krylov space (no restart)."""
    K = lanczos(apply_h, psi, m, reorth=reorth)
    return [combine(K, krylov_coefficients(K, s, direction, shift)) for s in nodes]


def propagate(apply_h, psi: np.ndarray, dt: float, nsteps: int, m: int,
              direction: int = -1, shift: float = 0.0, reorth: str = "cgs2") -> np.ndarray:
    for _ in range(nsteps):
        psi = sil_step(apply_h, psi, dt, m, direction, shift, reorth)
    return psi
