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


# ---------------------------------------------------------------------------
# The Keldysh-Matsubara (L-shaped) contour: 0 -> t_max -> 0 -> -i beta.
#
# Reading (Sec. 5: the initial state of the connected system is treated by
# CPT as well, through a Matsubara branch of length beta): the contour gets
# a third branch z = -i tau, tau_j = j dtau, j = 0..ntau-1, (ntau-1) dtau =
# beta, later on the contour than both real branches; the inter-cluster
# hopping V acts on all three branches, so the solution describes the
# connected system prepared in its equilibrium state.  The vertical branch
# enters the contour integral with the weight -i dtau (trapezoid, halved at
# its ends) and follows the same equal-point rules as the real branches.
# A contour function is given by its components
#   lesser[a, b]       = G^<(t_a, t_b)          greater[a, b]  = G^>(t_a, t_b)
#   mixed[a, j]        = G^<(t_a, -i tau_j)     (the real point earlier)
#   mixed_left[j, b]   = G^>(-i tau_j, t_b)     (the imaginary point later)
#   vert_greater[d]    = G^>(-i tau_{j+d}, -i tau_j),
#   vert_lesser[d]     = G^<(-i tau_j, -i tau_{j+d})   (translation invariant),
# each [..., n, n] over the orbitals.
# ---------------------------------------------------------------------------

def fermi_exp(e: np.ndarray, x: float, beta: float) -> np.ndarray:
    """f(e) e^{e x} for 0 <= x <= beta, f = 1 / (e^{beta e} + 1), without
    overflow (beta = inf: occupation 1, 1/2, 0 for e <, =, > 0, zero within
    1e-12 of the largest |level|)."""
    e = np.asarray(e, dtype=float)
    zero = np.abs(e) <= 1e-12 * max(1.0, float(np.abs(e).max()) if e.size else 1.0)
    if np.isinf(beta):
        return np.where(zero, 0.5, np.where(e < 0, np.exp(np.minimum(e, 0.0) * x), 0.0))
    neg = e <= 0
    en = np.where(neg, e, 0.0)
    ep = np.where(neg, 0.0, e)
    return np.where(neg, np.exp(en * x) / (np.exp(beta * en) + 1.0),
                    np.exp(-ep * (beta - x)) / (1.0 + np.exp(-beta * ep)))


def hole_exp(e: np.ndarray, x: float, beta: float) -> np.ndarray:
    """(1 - f(e)) e^{-e x} for 0 <= x <= beta, without overflow."""
    return fermi_exp(-np.asarray(e, dtype=float), x, beta)


def free_greens_l(h_ini: np.ndarray, h: np.ndarray, beta: float, nt: int, dt: float, ntau: int, dtau: float):
    """Exact contour components of free fermions (one spin) with one-particle
    Hamiltonian h_ini on the imaginary branch and h on the real branches,
    initial state e^{-beta h_ini} / Z: with the contour evolution
    U(t) = e^{-iht}, U(-i tau) = e^{-tau h_ini},
        G^<(z, z') = i U(z) f(h_ini) U(z')^-1,  G^>(z, z') = -i U(z) (1 - f(h_ini)) U(z')^-1.
    Real-time evolution by scipy.linalg.expm; functions of h_ini in its
    eigenbasis (overflow-free forms)."""
    e, Q = np.linalg.eigh(h_ini)
    Qh = Q.conj().T
    U = np.stack([scipy.linalg.expm(-1j * h * dt * k) for k in range(nt)])
    f0 = (Q * fermi_exp(e, 0.0, beta)) @ Qh
    Gl = 1j * np.einsum("aij,jk,blk->abil", U, f0, U.conj())
    Gg = -1j * np.einsum("aij,jk,blk->abil", U, np.eye(h.shape[0]) - f0, U.conj())
    Fe = np.stack([(Q * fermi_exp(e, j * dtau, beta)) @ Qh for j in range(ntau)])    # f e^{tau h_ini}
    He = np.stack([(Q * hole_exp(e, j * dtau, beta)) @ Qh for j in range(ntau)])     # (1-f) e^{-tau h_ini}
    mixed = 1j * np.einsum("aij,bjk->abik", U, Fe)
    mixed_left = -1j * np.einsum("aij,blj->abil", He, U.conj())
    return {"lesser": Gl, "greater": Gg, "mixed": mixed, "mixed_left": mixed_left,
            "vert_greater": -1j * He, "vert_lesser": 1j * Fe}


def bath_greens_l(T: np.ndarray, nt: int, dt: float, ntau: int, dtau: float, beta: float, sites=None):
    """Eqs. (gb1), (gb2) on the L-shaped contour for the uncorrelated bath
    (one-particle hopping matrix T, no quench): e^{-iT(z - z')} with complex
    contour times, occupations at beta.  Components [..., n, n] for the
    rows / columns `sites` (all by default)."""
    e, u = np.linalg.eigh(T)
    if sites is not None:
        u = u[list(sites)]
    t = dt * np.arange(nt)
    ph = np.exp(-1j * e[None, :] * t[:, None])                                  # [nt, k] e^{-i e t}
    f0 = fermi_exp(e, 0.0, beta)
    Gl = 1j * np.einsum("ik,ak,k,bk,jk->abij", u, ph, f0, ph.conj(), u.conj())
    Gg = -1j * np.einsum("ik,ak,k,bk,jk->abij", u, ph, 1.0 - f0, ph.conj(), u.conj())
    fe = np.stack([fermi_exp(e, j * dtau, beta) for j in range(ntau)])           # [ntau, k]
    he = np.stack([hole_exp(e, j * dtau, beta) for j in range(ntau)])
    mixed = 1j * np.einsum("ik,ak,jk,Jk->ajiJ", u, ph, fe, u.conj())
    mixed_left = -1j * np.einsum("ik,jk,bk,Jk->jbiJ", u, he, ph.conj(), u.conj())
    vg = -1j * np.einsum("ik,dk,jk->dij", u, he, u.conj())
    vl = 1j * np.einsum("ik,dk,jk->dij", u, fe, u.conj())
    return {"lesser": Gl, "greater": Gg, "mixed": mixed, "mixed_left": mixed_left,
            "vert_greater": vg, "vert_lesser": vl}


def lcontour_points(nt: int, dt: float, ntau: int, dtau: float):
    """(branch, mesh index, quadrature weight) of the 2 nt + ntau points:
    branch 0 forward, 1 backward, 2 imaginary (weight -i dtau)."""
    br = np.concatenate([np.zeros(nt, int), np.ones(nt, int), np.full(ntau, 2)])
    idx = np.concatenate([np.arange(nt), np.arange(nt)[::-1], np.arange(ntau)])
    _, wr = contour_points(nt, dt)
    wt = np.full(ntau, dtau)
    if ntau > 1:
        wt[0] = wt[-1] = 0.5 * dtau
    else:
        wt[:] = 0.0
    return br, idx, np.concatenate([wr.astype(complex), -1j * wt])


def to_contour_l(fn: dict, role: str = "row") -> np.ndarray:
    """Contour matrix [(2 nt + ntau) n]^2 of a contour function given by its
    components (module notes above); role as in to_contour: the one-sided
    equal-point values at the ends of each of the three branches."""
    nt, n = fn["lesser"].shape[0], fn["lesser"].shape[2]
    ntau = fn["vert_greater"].shape[0] if "vert_greater" in fn else 0
    br, idx, _ = lcontour_points(nt, 1.0, ntau, 1.0)
    N = 2 * nt + ntau
    starts = ({0, nt} if nt > 1 else set()) | ({2 * nt} if ntau > 1 else set())
    ends = ({nt - 1, 2 * nt - 1} if nt > 1 else set()) | ({N - 1} if ntau > 1 else set())
    out = np.zeros((N, n, N, n), dtype=np.complex128)
    for p in range(N):
        for q in range(N):
            a, b = idx[p], idx[q]
            if br[p] < 2 and br[q] < 2:
                gg, gl = fn["greater"][a, b], fn["lesser"][a, b]
            elif br[p] < 2:
                out[p, :, q, :] = fn["mixed"][a, b]
                continue
            elif br[q] < 2:
                out[p, :, q, :] = fn["mixed_left"][a, b]
                continue
            else:
                gg, gl = fn["vert_greater"][a - b] if a >= b else None, fn["vert_lesser"][b - a] if b >= a else None
            if p > q:
                blk = gg
            elif p < q:
                blk = gl
            elif p in starts:
                blk = gl if role == "row" else gg
            elif p in ends:
                blk = gg if role == "row" else gl
            else:
                blk = 0.5 * (gg + gl)
            out[p, :, q, :] = blk
    return out.reshape(N * n, N * n)


def from_contour_l(Gz: np.ndarray, nt: int, ntau: int, n: int) -> dict:
    """Contour matrix -> components (lesser, greater, mixed, mixed_left and
    the imaginary-branch functions of tau_j - tau_0)."""
    N = 2 * nt + ntau
    G = Gz.reshape(N, n, N, n)
    fwd = np.arange(nt)
    bwd = 2 * nt - 1 - np.arange(nt)
    ver = 2 * nt + np.arange(ntau)
    pick = lambda P, Q: np.ascontiguousarray(np.transpose(G[np.ix_(P, range(n), Q, range(n))], (0, 2, 1, 3)))
    out = {"lesser": pick(fwd, bwd), "greater": pick(bwd, fwd)}
    if ntau:
        out["mixed"] = pick(fwd, ver)
        out["mixed_left"] = pick(ver, fwd)
        V = pick(ver, ver)
        out["vert_greater"] = np.ascontiguousarray(V[:, 0])     # d = 0: the start's diagonal holds G^>
        vl = np.ascontiguousarray(V[0, :])
        vl[0] = V[ntau - 1, ntau - 1]                            # d = 0: the end's diagonal holds G^<
        out["vert_lesser"] = vl
    return out


def cpt_solve_l(Gp: dict, V: np.ndarray, dt: float, dtau: float) -> dict:
    """The discretised CPT equation on the L-shaped contour,
    (1 - G'_row W V) G = G'_rhs, W the diagonal of the quadrature weights of
    the three branches.  Gp: components of the disconnected system."""
    nt, n = Gp["lesser"].shape[0], Gp["lesser"].shape[2]
    ntau = Gp["vert_greater"].shape[0]
    _, _, w = lcontour_points(nt, dt, ntau, dtau)
    WV = np.kron(np.diag(w), V)
    A = np.eye((2 * nt + ntau) * n) - to_contour_l(Gp, "row") @ WV
    G = scipy.linalg.solve(A, to_contour_l(Gp, "rhs"))
    return from_contour_l(G, nt, ntau, n)


def embed_l(Gc: dict, Gb: dict, boundary: int, V: float):
    """Block-diagonal components of the disconnected system (cluster, then
    bath) and the hopping matrix linking cluster site `boundary` to bath
    site 0 (-V on the bond)."""
    nc, nb = Gc["lesser"].shape[2], Gb["lesser"].shape[2]
    n = nc + nb
    out = {}
    for key in ("lesser", "greater", "mixed", "mixed_left", "vert_greater", "vert_lesser"):
        c, b = Gc[key], Gb[key]
        z = np.zeros(c.shape[:-2] + (n, n), dtype=np.complex128)
        z[..., :nc, :nc] = c
        z[..., nc:, nc:] = b
        out[key] = z
    Vm = np.zeros((n, n))
    Vm[boundary, nc] = Vm[nc, boundary] = -V
    return out, Vm


def necpt_l(Gc: dict, Gb: dict, boundary: int, V: float, dt: float, dtau: float) -> dict:
    """Cluster block of the NE-CPT Green's function on the L-shaped contour
    (the CPT equation for cluster plus every bath site, restricted to the
    cluster)."""
    nc = Gc["lesser"].shape[2]
    Gp, Vm = embed_l(Gc, Gb, boundary, V)
    G = cpt_solve_l(Gp, Vm, dt, dtau)
    return {k: np.ascontiguousarray(v[..., :nc, :nc]) for k, v in G.items()}


def cluster_fn(four_step_out: dict) -> dict:
    """Contour components of the cluster from the four-step outputs (its
    ground state: the zero-temperature limit of Sec. 4):
    vert_greater = i G^M(+tau), vert_lesser = i G^M(-tau), mixed = G^|(t, tau),
    mixed_left = G^|(tau, t) (oracle.greens.four_step conventions)."""
    GM = four_step_out["G_matsubara"]
    return {"lesser": four_step_out["G_lesser"], "greater": four_step_out["G_greater"],
            "mixed": four_step_out["G_mixed"], "mixed_left": four_step_out["G_mixed_left"],
            "vert_greater": 1j * GM[0], "vert_lesser": 1j * GM[1]}


def cluster_fn_kms(four_step_out: dict) -> dict:
    """The cluster's contour components on an imaginary branch of length
    beta = (ntau - 1) dtau from its ground state |0> (N particles), in the
    limit of a grand-canonical equilibrium dominated by |0> (reading of
    Sec. 5's Matsubara branch at beta = 15): besides the ground-state terms
    of cluster_fn, the states of N -+ 1 particles reached from |0> by c, c+
    enter near the far end of the branch with the weight
    e^{-(beta - tau)(E_n - E0)}, and, with e^{-tau (H_ini - E0)} projecting
    onto |0> there, those terms are the same ground-state scalar products
    read at beta - tau (the functions then obey the boundary condition
    G(-i beta, z') = -G(0, z') up to terms e^{-beta Delta}):
        G^>(-i tau, -i tau') = i G^M(+d) - i G^M(-(beta - d)),  d = tau - tau' >= 0
        G^<(-i tau, -i tau') = i G^M(-d) - i G^M(+(beta - d)),  d = tau' - tau >= 0
        G^<_ab(t, -i tau)    = G^|_ab(t, tau) + conj(G^|_ba(beta - tau, t))
        G^>_ab(-i tau, t)    = G^|_ab(tau, t) + conj(G^|_ba(t, beta - tau))
    (G^| with a real first argument: the c sweep; with an imaginary first
    argument: the c+ sweep).  The real-time components are unchanged (their
    corrections are of order e^{-beta Delta})."""
    fn = cluster_fn(four_step_out)
    vg0, vl0 = fn["vert_greater"], fn["vert_lesser"]
    mx, mxl = fn["mixed"], fn["mixed_left"]
    out = dict(fn)
    out["vert_greater"] = vg0 - vl0[::-1]
    out["vert_lesser"] = vl0 - vg0[::-1]
    out["mixed"] = mx + np.conj(np.transpose(mxl[::-1], (1, 0, 3, 2)))
    out["mixed_left"] = mxl + np.conj(np.transpose(mx[:, ::-1], (1, 0, 3, 2)))
    return out
