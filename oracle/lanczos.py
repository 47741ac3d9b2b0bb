"""Lanczos recursion and ground state (Sec. 2).

Test infrastructure (see the package docstring).

Eq. (recursion) builds the Krylov space K_n(|i_0>) of Eq. (kspace) with
    |i_{k+1}> = H|i_k> - a_k |i_k> - b_k^2 |i_{k-1}>,
    a_k = <i_k|H|i_k>/<i_k|i_k>,  b_k^2 = <i_k|i_k>/<i_{k-1}|i_{k-1}>,
followed by normalisation; in the normalised basis H is the tridiagonal
T = V^+ H V of Eq. (tmatrix) with diagonal a_0..a_{n-1} and off-diagonal
b_1..b_{n-1} (the positive square roots).  This module runs the same
recursion directly on the normalised vectors v_k = |i_k>/||i_k||, which
gives the identical coefficients (a_k, b_k).  The paper adds Gram-Schmidt
reorthogonalisation of each new vector against the stored basis (Sec. 3,
Fig. 1 discussion; Sec. 4, Fig. 4 caption); the variant is not named, the
reading here is classical Gram-Schmidt applied twice ("cgs2"), with "none"
and a single pass ("cgs") available as well.

Eigenpairs of T (Eq. tdiag) come from scipy's symmetric tridiagonal
eigensolver; the Ritz vector is Eq. (eigen).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
from scipy.linalg import eigh_tridiagonal


def vdot(x, y) -> complex:
    return complex(np.vdot(x, y))


def _reorthogonalise(w: np.ndarray, basis: List[np.ndarray], passes: int) -> np.ndarray:
    for _ in range(passes):
        if not basis:
            break
        B = np.stack(basis, axis=1)
        h = B.conj().T @ w
        w = w - B @ h
    return w


REORTH_PASSES = {"none": 0, "cgs": 1, "cgs2": 2}


@dataclass
class Krylov:
    """Result of n Lanczos steps from a start vector."""
    V: List[np.ndarray]          # orthonormal basis v_0..v_{n-1}
    a: np.ndarray                # diagonal of T
    b: np.ndarray                # b[k] couples v_{k-1}, v_k (b[0] = 0); len n+1
    beta0: float                 # norm of the start vector
    breakdown: bool = False

    @property
    def n(self) -> int:
        return len(self.a)

    def T(self) -> np.ndarray:
        n = self.n
        return np.diag(self.a) + np.diag(self.b[1:n], 1) + np.diag(self.b[1:n], -1)


def lanczos(apply_h: Callable, v0: np.ndarray, n: int, reorth: str = "cgs2",
            breakdown_tol: float = 1e-13) -> Krylov:
    """n steps of Eq. (recursion) from |i_0> = v0 (normalised internally).

    Stops early when the new off-diagonal element b_{k+1} falls below
    breakdown_tol * max(|a_j|, b_j) (the Krylov space is invariant: the
    truncated T is then exact for every function of H applied to v0)."""
    passes = REORTH_PASSES[reorth]
    beta0 = float(np.linalg.norm(v0))
    v = v0 / beta0
    V = [v]
    a, b = [], [0.0]
    scale = 0.0
    breakdown = False
    for k in range(n):
        w = apply_h(V[k])
        ak = vdot(V[k], w).real
        a.append(ak)
        w = w - ak * V[k]
        if k > 0:
            w = w - b[k] * V[k - 1]
        w = _reorthogonalise(w, V, passes)
        bk1 = float(np.linalg.norm(w))
        scale = max(scale, abs(ak), b[k])
        if k == n - 1:
            b.append(bk1)
            break
        if bk1 <= breakdown_tol * scale:
            b.append(0.0)
            breakdown = True
            break
        b.append(bk1)
        V.append(w / bk1)
    return Krylov(V=V, a=np.array(a), b=np.array(b), beta0=beta0, breakdown=breakdown)


@dataclass
class GroundState:
    E0: float
    psi: np.ndarray
    iters: int
    residual: float
    converged: bool
    history: List[float] = field(default_factory=list)


def ground_state(apply_h: Callable, v0: np.ndarray, tol: float = 1e-12,
                 max_iter: int = 300, reorth: str = "cgs2",
                 check_every: int = 1) -> GroundState:
    """Step (i) of the four-step procedure (Sec. 4) / the first Lanczos run
    of Sec. 2: Lanczos from an arbitrary start vector with finite overlap,
    T_k diagonalised (Eq. tdiag), lowest Ritz value E0 and Ritz vector
    |0> = sum_j y_j v_j (Eq. eigen).

    The paper runs a fixed n (about 100 to 200); the reading here stops
    when the Ritz residual ||H|0> - E0|0>|| = b_{k+1}|y_{k}| falls below
    tol * max(1, |E0|), or at max_iter."""
    passes = REORTH_PASSES[reorth]
    v = v0 / np.linalg.norm(v0)
    V = [v]
    a, b = [], [0.0]
    hist = []
    converged = False
    theta, y, res = None, None, np.inf
    k = 0
    for k in range(max_iter):
        w = apply_h(V[k])
        ak = vdot(V[k], w).real
        a.append(ak)
        w = w - ak * V[k]
        if k > 0:
            w = w - b[k] * V[k - 1]
        w = _reorthogonalise(w, V, passes)
        bk1 = float(np.linalg.norm(w))
        last = (k == max_iter - 1)
        if (k + 1) % check_every == 0 or last or bk1 == 0.0:
            if k == 0:
                theta, Y = np.array([a[0]]), np.ones((1, 1))
            else:
                theta, Y = eigh_tridiagonal(np.array(a), np.array(b[1:k + 1]))
            y = Y[:, 0]
            res = bk1 * abs(y[-1])
            hist.append(float(theta[0]))
            if res <= tol * max(1.0, abs(theta[0])):
                converged = True
                break
        if bk1 == 0.0:
            converged = True
            break
        b.append(bk1)
        V.append(w / bk1)
    n = len(a)
    if theta is None or len(y) != n:
        if n == 1:
            theta, Y = np.array([a[0]]), np.ones((1, 1))
        else:
            theta, Y = eigh_tridiagonal(np.array(a), np.array(b[1:n]))
        y = Y[:, 0]
    psi = np.zeros_like(V[0])
    for j in range(n):
        psi = psi + y[j] * V[j]
    psi = psi / np.linalg.norm(psi)
    return GroundState(E0=float(theta[0]), psi=psi, iters=n, residual=float(res),
                       converged=converged, history=hist)


def fidelity(psi_a: np.ndarray, psi_b: np.ndarray) -> float:
    """|<a|b>|^2 of two normalised states (two-start uniqueness check of
    the nondegenerate-ground-state assumption of Eq. (gomega))."""
    return abs(vdot(psi_a, psi_b)) ** 2
