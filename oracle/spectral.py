"""Equilibrium spectra of Secs. 2 and 3.

Test infrastructure (see the package docstring).

* lanczos_greens_omega: the conventional Lanczos Green's function of
  Eq. (gapprox): a second Lanczos run from |i0> = c+_a|0> (c_a|0> for the
  hole part), the Ritz pairs of its tridiagonal matrix (Eq. (eigen)) and the
  pole sum over them.
* greens_time_fine: the time-dependent Lanczos G(t) of Eqs. (psit) and
  (psigreen) with a restart every dt and the states inside a step taken from
  that step's Krylov space (Eq. (udelta) at the intermediate times).
* fourier: the damped transform int_0^T dt e^{i omega t - eta t} G(t) by the
  trapezoid rule on the time grid.
"""
from __future__ import annotations

import numpy as np

from .basis import Sector
from .hamiltonian import Hamiltonian, apply_ladder
from .lanczos import lanczos, vdot
from .propagate import combine, krylov_coefficients, tridiag_eig


def lanczos_greens_omega(model, sector: Sector, psi0, E0: float, orbital, n: int, omegas, eta: float,
                         reorth: str = "cgs2"):
    """G^(L)(omega) of Eq. (gapprox): particle part sum_m w_m / (omega + i eta
    - E_m + E0) from |i0> = c+|0>, hole part sum_m w_m / (omega + i eta + E_m
    - E0) from |i0> = c|0>, with w_m = <i0|i0> |Q_0m|^2."""
    site, spin = orbital
    z = np.asarray(omegas, dtype=np.float64) + 1j * eta
    out = {}
    for greater in (True, False):
        i0, tgt = apply_ladder(sector, site, spin, greater, psi0)
        key = "G_greater" if greater else "G_lesser"
        if tgt.dim == 0 or not np.any(i0):
            out[key] = np.zeros(len(z), dtype=np.complex128)
            continue
        K = lanczos(Hamiltonian(model, tgt).apply, i0, n, reorth=reorth)
        lam, Q = tridiag_eig(K)
        w = K.beta0 ** 2 * Q[0, :] ** 2
        if greater:
            out[key] = (w[None, :] / (z[:, None] - lam[None, :] + E0)).sum(axis=1)
        else:
            out[key] = (w[None, :] / (z[:, None] + lam[None, :] - E0)).sum(axis=1)
    return out


def greens_time_fine(model, sector: Sector, psi0, E0: float, orbital, dagger: bool, nsteps: int, nfine: int,
                     dt: float, m: int, reorth: str = "none"):
    """G^>(t) = -i e^{iE0 t} <c+0|e^{-iHt}|c+0> (dagger) or G^<(t) = +i
    e^{-iE0 t} <c0|e^{iHt}|c0> on t_j = j dt / nfine, j = 0..nsteps*nfine."""
    site, spin = orbital
    i0, tgt = apply_ladder(sector, site, spin, dagger, psi0)
    if tgt.dim == 0:
        return np.zeros(nsteps * nfine + 1, dtype=np.complex128)
    H = Hamiltonian(model, tgt)
    direction = -1 if dagger else +1
    pf = -1.0 if dagger else 1.0
    out = [pf * 1j * vdot(i0, i0)]
    psi = i0
    for k in range(nsteps):
        K = lanczos(H.apply, psi, m, reorth=reorth)
        for q in range(1, nfine + 1):
            s = dt if q == nfine else q * dt / nfine
            phi = combine(K, krylov_coefficients(K, s, direction))
            t = k * dt + s
            out.append(pf * 1j * vdot(i0, phi) * np.exp(-1j * direction * E0 * t))
        psi = phi
    return np.array(out)


def fourier(G, dt: float, eta: float, omegas):
    """sum_k w_k e^{(i omega - eta) t_k} G_k, t_k = k dt, trapezoid weights."""
    G = np.asarray(G, dtype=np.complex128)
    t = dt * np.arange(len(G))
    w = np.full(len(G), dt)
    w[0] = w[-1] = 0.5 * dt
    E = np.exp((1j * np.asarray(omegas)[:, None] - eta) * t[None, :])
    return E @ (w * G)
