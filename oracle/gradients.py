"""Exact (dense) gradients: the reference for the adjoint.

Test infrastructure (see the package docstring).

The paper has no derivatives; these are the textbook ones.  H is linear in
the parameters theta = (t_b, eps_up_i, eps_dn_i, U_i), so dH/dtheta_p is H
evaluated at the one-hot parameter vector e_p.  The derivative of a matrix
exponential exp(A) in the direction E is its Frechet derivative
(scipy.linalg.expm_frechet, the Al-Mohy--Higham algorithm).  The derivative
of a nondegenerate ground state is, by first-order perturbation theory,
d|0> = - sum_{n != 0} |n><n| dH |0> / (E_n - E_0) (full diagonalisation),
the component along |0> being a phase that no Green's function sees.

Everything here is dense and meant for sectors of a few hundred states.
"""
from __future__ import annotations

from dataclasses import replace
from typing import Dict, Sequence, Tuple

import numpy as np
import scipy.linalg as sla

from .basis import Sector
from .hamiltonian import Hamiltonian, ladder_operator


def theta_of(model) -> np.ndarray:
    """(t_b, eps_up, eps_dn, U) of a model as one vector."""
    _, t, eu, ed, U = model.arrays()
    return np.concatenate([t, eu, ed, U])


def model_with_theta(model, theta) -> object:
    nb, L = len(model.bonds), model.L
    th = np.asarray(theta, dtype=np.float64)
    return replace(model, t=tuple(th[:nb]), eps_up=tuple(th[nb:nb + L]), eps_dn=tuple(th[nb + L:nb + 2 * L]),
                   U=tuple(th[nb + 2 * L:]))


def dH_matrices(model, sector: Sector):
    """Dense dH/dtheta_p for every parameter p (H at one-hot theta)."""
    n = len(theta_of(model))
    out = []
    for p in range(n):
        e = np.zeros(n)
        e[p] = 1.0
        out.append(Hamiltonian(model_with_theta(model, e), sector).dense())
    return out


def propagation_gradient(model, sector: Sector, psi0, chi, t: float, direction: int) -> np.ndarray:
    """dL/dtheta for L = Re <chi| exp(direction i H t) |psi0>."""
    H = Hamiltonian(model, sector).dense()
    A = direction * 1j * t * H
    g = []
    for dH in dH_matrices(model, sector):
        dU = sla.expm_frechet(A, direction * 1j * t * dH, compute_expm=False)
        g.append(np.vdot(chi, dU @ psi0).real)
    return np.array(g)


def propagation_exact(model, sector: Sector, psi0, t: float, direction: int) -> np.ndarray:
    H = Hamiltonian(model, sector).dense()
    return sla.expm(direction * 1j * t * H) @ psi0


def _ground(H0: np.ndarray):
    w, V = np.linalg.eigh(H0)
    return w, V


def four_step_exact(H_ini_model, H_model, n_up: int, n_dn: int, orbitals: Sequence[Tuple[int, int]],
                    times: Sequence[float]) -> Dict[str, np.ndarray]:
    """The four-step G^< and G^> with exact exponentials (dense)."""
    return _four_step(H_ini_model, H_model, n_up, n_dn, orbitals, times, None, None)[0]


def four_step_gradient(H_ini_model, H_model, n_up: int, n_dn: int, orbitals: Sequence[Tuple[int, int]],
                       times: Sequence[float], W_lesser, W_greater):
    """Exact dL/dtheta_ini and dL/dtheta for L = Re sum conj(W^<) G^< + Re sum
    conj(W^>) G^> (W: [nt][nt][n_orb][n_orb]).  Returns (grad_ini, grad, G)."""
    G, gi, g = _four_step(H_ini_model, H_model, n_up, n_dn, orbitals, times, W_lesser, W_greater)
    return gi, g, G


def _four_step(H_ini_model, H_model, n_up, n_dn, orbitals, times, Wl, Wg):
    L = H_model.L
    sec = Sector(L, n_up, n_dn)
    nt, no = len(times), len(orbitals)
    w, V = _ground(Hamiltonian(H_ini_model, sec).dense())
    assert w[1] - w[0] > 1e-8, "degenerate ground state"
    psi0 = V[:, 0]
    Hf = Hamiltonian(H_model, sec).dense()
    # operators and target-sector Hamiltonians: (c_a, H_T) for lesser, (c+_a, H_T) for greater
    ops = {}
    for a, (site, spin) in enumerate(orbitals):
        for dag in (False, True):
            M, tgt = ladder_operator(sec, site, spin, dag)
            HT = Hamiltonian(H_model, tgt).dense() if tgt.dim else np.zeros((0, 0))
            ops[(a, dag)] = (M.toarray(), HT, tgt)

    def states(phi0, dH_N=None, dH_T=None, dphi0=None):
        """Psi[a][dag][j] and, when derivatives are given, their first-order changes."""
        Psi, dPsi = {}, {}
        for j, t in enumerate(times):
            UN = sla.expm(-1j * t * Hf)
            phi = UN @ phi0
            dphi = None
            if dH_N is not None:
                dphi = sla.expm_frechet(-1j * t * Hf, -1j * t * dH_N, compute_expm=False) @ phi0
            if dphi0 is not None:
                dphi = UN @ dphi0 if dphi is None else dphi + UN @ dphi0
            for (a, dag), (M, HT, tgt) in ops.items():
                if tgt.dim == 0:
                    continue
                UT = sla.expm(1j * t * HT)
                x = M @ phi
                Psi[(a, dag, j)] = UT @ x
                if dphi is not None or dH_T is not None:
                    d = np.zeros(tgt.dim, dtype=np.complex128)
                    if dH_T is not None:
                        d += sla.expm_frechet(1j * t * HT, 1j * t * dH_T[(a, dag)], compute_expm=False) @ x
                    if dphi is not None:
                        d += UT @ (M @ dphi)
                    dPsi[(a, dag, j)] = d
        return Psi, dPsi

    def green(Psi, dPsi=None):
        Gl = np.zeros((nt, nt, no, no), dtype=np.complex128)
        Gg = np.zeros_like(Gl)
        for j in range(nt):
            for s in range(nt):
                for a in range(no):
                    for b in range(no):
                        if orbitals[a][1] != orbitals[b][1]:
                            continue
                        if (a, False, j) in Psi:
                            pa, pb = Psi[(a, False, j)], Psi[(b, False, s)]
                            v = np.vdot(pb, pa)
                            if dPsi is not None:
                                v = np.vdot(dPsi[(b, False, s)], pa) + np.vdot(pb, dPsi[(a, False, j)])
                            Gl[j, s, a, b] = 1j * v
                        if (a, True, j) in Psi:
                            pa, pb = Psi[(a, True, j)], Psi[(b, True, s)]
                            v = np.vdot(pa, pb)
                            if dPsi is not None:
                                v = np.vdot(dPsi[(a, True, j)], pb) + np.vdot(pa, dPsi[(b, True, s)])
                            Gg[j, s, a, b] = -1j * v
        return Gl, Gg

    Psi, _ = states(psi0)
    Gl, Gg = green(Psi)
    G = {"G_lesser": Gl, "G_greater": Gg, "E0": w[0]}
    if Wl is None and Wg is None:
        return G, None, None
    Wl = np.zeros_like(Gl) if Wl is None else np.asarray(Wl).reshape(Gl.shape)
    Wg = np.zeros_like(Gg) if Wg is None else np.asarray(Wg).reshape(Gg.shape)

    def loss_derivative(dGl, dGg):
        return float((np.sum(np.conj(Wl) * dGl) + np.sum(np.conj(Wg) * dGg)).real)

    # parameters of H (in every sector)
    dHN = dH_matrices(H_model, sec)
    dHT = {key: dH_matrices(H_model, tgt) if tgt.dim else None for key, (M, HT, tgt) in ops.items()}
    grad = np.zeros(len(dHN))
    for p in range(len(dHN)):
        dT = {key: (v[p] if v is not None else None) for key, v in dHT.items()}
        _, dPsi = states(psi0, dH_N=dHN[p], dH_T=dT)
        grad[p] = loss_derivative(*green(Psi, dPsi))
    # parameters of H_ini (through the ground state)
    dHI = dH_matrices(H_ini_model, sec)
    grad_ini = np.zeros(len(dHI))
    for p in range(len(dHI)):
        coef = (V[:, 1:].conj().T @ (dHI[p] @ psi0)) / (w[1:] - w[0])
        dpsi0 = -V[:, 1:] @ coef
        _, dPsi = states(psi0, dphi0=dpsi0)
        grad_ini[p] = loss_derivative(*green(Psi, dPsi))
    return G, grad_ini, grad
