"""Nonequilibrium cluster-perturbation theory (Sec. 5, Eq. (cpteq)) on the
Keldysh contour (test infrastructure only; the product path never imports
this module).

The CPT equation G = (G'^-1 - V)^-1, with G' the Green's function of the
disconnected system (the correlated cluster and the uncorrelated bath) and V
the inter-cluster hopping, is a contour integral equation

    G(z, z') = G'(z, z') + int_C dz'' G'(z, z'') V G(z'', z').

Reading taken here (the paper leaves the discretisation to its reference):
the initial state is the ground state of the disconnected system (cluster
ground state times bath ground state, the bath's Eqs. (gb1), (gb2) at
beta -> infinity), V acts for t > 0, and the contour is the Keldysh contour
0 -> t_max -> 0 on the mesh t_k = k dt, k = 0..nt-1: contour point index
p = 0..nt-1 is t_p on the forward branch, p = nt..2nt-1 is t_{2nt-1-p} on the
backward branch.  A contour function is G^>(t, t') where z is later than z'
and G^<(t, t') where z is earlier.  The contour integral is the trapezoid
rule on each branch (weight +dt on the forward and -dt on the backward
branch, halved at both ends of each branch), with every jump of the
integrand at a node: at an interior node the integrand takes the mean of its
two one-sided limits, so the equal-point diagonal of G' is (G^> + G^<)/2.
At the four branch ends (t = 0 forward, t_max forward, t_max backward, t = 0
backward) only the limit from inside the branch enters, and it differs
between the two places where G' appears in  (1 - G' W V) G = G':
as the kernel G'(z, z''), z'' -> z from inside the branch, it is G^< at a
branch start and G^> at a branch end ("row" values); as the right-hand side
it fixes the diagonal of the unknown G, which is later used as G(z'', z'),
z'' -> z' from inside the branch, so there it is G^> at a branch start and
G^< at a branch end ("rhs" values).  With the mean at the branch ends
instead, the scheme is only first order in dt.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def contour_points(nt: int, dt: float):
    """(time index, quadrature weight) of the 2 nt contour points."""
    tix = np.concatenate([np.arange(nt), np.arange(nt)[::-1]])
    w = np.full(nt, dt)
    if nt > 1:
        w[0] = w[-1] = 0.5 * dt
    else:
        w[:] = 0.0
    return tix, np.concatenate([w, -w[::-1]])


def to_contour(G_lesser: np.ndarray, G_greater: np.ndarray, role: str = "row") -> np.ndarray:
    """[nt, nt, n, n] lesser / greater meshes -> contour matrix
    [2nt * n, 2nt * n], row (p, i) = p * n + i; role "row" or "rhs" picks the
    one-sided diagonal values at the branch ends (module docstring)."""
    nt, n = G_lesser.shape[0], G_lesser.shape[2]
    tix, _ = contour_points(nt, 1.0)
    N = 2 * nt
    starts = {0, nt} if nt > 1 else set()
    ends = {nt - 1, N - 1} if nt > 1 else set()
    out = np.zeros((N, n, N, n), dtype=np.complex128)
    for p in range(N):
        for q in range(N):
            a, b = tix[p], tix[q]
            if p > q:
                blk = G_greater[a, b]
            elif p < q:
                blk = G_lesser[a, b]
            elif p in starts:
                blk = G_lesser[a, b] if role == "row" else G_greater[a, b]
            elif p in ends:
                blk = G_greater[a, b] if role == "row" else G_lesser[a, b]
            else:
                blk = 0.5 * (G_greater[a, b] + G_lesser[a, b])
            out[p, :, q, :] = blk
    return out.reshape(N * n, N * n)


def from_contour(Gz: np.ndarray, nt: int, n: int):
    """Contour matrix -> (G^<, G^>) meshes: G^<(t_a, t_b) has z = t_a on the
    forward branch and z' = t_b on the backward branch, G^> the reverse."""
    G = Gz.reshape(2 * nt, n, 2 * nt, n)
    fwd = np.arange(nt)
    bwd = 2 * nt - 1 - np.arange(nt)
    Gl = np.transpose(G[np.ix_(fwd, range(n), bwd, range(n))], (0, 2, 1, 3))
    Gg = np.transpose(G[np.ix_(bwd, range(n), fwd, range(n))], (0, 2, 1, 3))
    return np.ascontiguousarray(Gl), np.ascontiguousarray(Gg)


def bath_greens(T: np.ndarray, nt: int, dt: float, beta: float = np.inf, sites=None):
    """Eqs. (gb1), (gb2): lesser / greater Green's function of the
    uncorrelated bath with one-particle hopping matrix T (Hermitian):
    G^>(t, t') = -i [e^{-iT(t-t')} (1 + e^{-beta T})^-1],
    G^<(t, t') = +i [e^{-iT(t-t')} (e^{beta T} + 1)^-1];
    beta = inf keeps the occupied (negative) levels, zero levels (within
    1e-12 of the largest |level|) half.  sites: the rows / columns kept (all
    by default).  Returns [nt, nt, n, n] meshes."""
    e, u = np.linalg.eigh(T)
    zero = np.abs(e) <= 1e-12 * max(1.0, np.abs(e).max())     # a zero level, up to rounding
    if np.isinf(beta):
        occ = np.where(zero, 0.5, np.where(e < 0, 1.0, 0.0))
    else:
        occ = 1.0 / (np.exp(beta * e) + 1.0)
    if sites is not None:
        u = u[list(sites)]
    t = dt * np.arange(nt)
    tau = t[:, None] - t[None, :]
    ph = np.exp(-1j * e[None, None, :] * tau[:, :, None])          # [nt, nt, k]
    Gl = 1j * np.einsum("ik,abk,k,jk->abij", u, ph, occ, u.conj())
    Gg = -1j * np.einsum("ik,abk,k,jk->abij", u, ph, 1.0 - occ, u.conj())
    return Gl, Gg


def cpt_solve(Gp_lesser: np.ndarray, Gp_greater: np.ndarray, V: np.ndarray, dt: float):
    """The discretised CPT equation on the contour:
    (1 - G'_row W V) G = G'_rhs, with W the diagonal of quadrature weights
    (V is instantaneous, so the contour integral over z'' carries one
    weight) and G'_row, G'_rhs the contour matrices of G' with the row and
    rhs values at the branch ends.
    Gp_*: [nt, nt, n, n] meshes of the disconnected system; V: [n, n].
    Returns the (G^<, G^>) meshes of the connected system."""
    nt, n = Gp_lesser.shape[0], Gp_lesser.shape[2]
    _, w = contour_points(nt, dt)
    WV = np.kron(np.diag(w), V)
    A = np.eye(2 * nt * n) - to_contour(Gp_lesser, Gp_greater, "row") @ WV
    G = scipy.linalg.solve(A, to_contour(Gp_lesser, Gp_greater, "rhs"))
    return from_contour(G, nt, n)


def embed(Gc_lesser, Gc_greater, Gb_lesser, Gb_greater, boundary: int, V: float):
    """G' of the disconnected system (cluster block, then bath block) and
    the inter-cluster hopping between cluster site `boundary` and bath site 0
    (-V on the bond, the sign convention of the hopping term)."""
    nc, nb = Gc_lesser.shape[2], Gb_lesser.shape[2]
    nt = Gc_lesser.shape[0]
    n = nc + nb
    Gl = np.zeros((nt, nt, n, n), dtype=np.complex128)
    Gg = np.zeros_like(Gl)
    Gl[:, :, :nc, :nc], Gg[:, :, :nc, :nc] = Gc_lesser, Gc_greater
    Gl[:, :, nc:, nc:], Gg[:, :, nc:, nc:] = Gb_lesser, Gb_greater
    Vm = np.zeros((n, n))
    Vm[boundary, nc] = Vm[nc, boundary] = -V
    return Gl, Gg, Vm


def necpt(Gc_lesser, Gc_greater, Gb_lesser, Gb_greater, boundary: int, V: float, dt: float):
    """Cluster block [nt, nt, nc, nc] of the NE-CPT Green's function: the
    CPT equation written out for the full disconnected system (cluster plus
    every bath site), then restricted to the cluster."""
    nc = Gc_lesser.shape[2]
    Gl, Gg, Vm = embed(Gc_lesser, Gc_greater, Gb_lesser, Gb_greater, boundary, V)
    Hl, Hg = cpt_solve(Gl, Gg, Vm, dt)
    return Hl[:, :, :nc, :nc], Hg[:, :, :nc, :nc]


def free_greens(h: np.ndarray, rho: np.ndarray, nt: int, dt: float):
    """Exact G^<, G^> of free fermions with one-particle Hamiltonian h and
    initial one-particle density matrix rho (a Gaussian state):
    G^<(t, t') = i e^{-iht} rho e^{iht'}, G^>(t, t') = -i e^{-iht} (1 - rho) e^{iht'}."""
    n = h.shape[0]
    U = np.stack([scipy.linalg.expm(-1j * h * dt * k) for k in range(nt)])
    Gl = 1j * np.einsum("aij,jk,blk->abil", U, rho, U.conj())
    Gg = -1j * np.einsum("aij,jk,blk->abil", U, np.eye(n) - rho, U.conj())
    return Gl, Gg


def ground_density(h: np.ndarray, n_particles: int) -> np.ndarray:
    """One-particle density matrix of the Slater determinant filling the
    n_particles lowest levels of h (a gap above them is the caller's care)."""
    e, u = np.linalg.eigh(h)
    occ = u[:, :n_particles]
    return occ @ occ.conj().T
