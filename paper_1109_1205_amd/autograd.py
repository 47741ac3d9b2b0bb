"""torch.autograd binding of the four-step Green's function.

`greens_neq(...)` returns (G^<, G^>) as complex128 CPU tensors
[nt][nt][n_orb][n_orb] that are differentiable with respect to the real
parameter vectors theta_ini (of H_ini) and theta (of H), each laid out as
(t_b for every bond, eps_up_i, eps_dn_i, U_i).  Forward and backward run in
libkgf (kgf_greens_neq, kgf_greens_neq_vjp); this module only builds the
model handles from the parameter vectors and marshals arrays.

For a complex output PyTorch's grad_output is dL/dRe G + i dL/dIm G
(= 2 dL/dG*), which is exactly the library's cotangent W defined by
dL = Re sum conj(W) dG.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np
import torch

from ._lib import Context, Model, Sector


def split_theta(L: int, n_bonds: int, theta):
    th = np.asarray(theta, dtype=np.float64).reshape(-1)
    if len(th) != n_bonds + 3 * L:
        raise ValueError(f"theta has {len(th)} entries, expected n_bonds + 3 L = {n_bonds + 3 * L}")
    return th[:n_bonds], th[n_bonds:n_bonds + L], th[n_bonds + L:n_bonds + 2 * L], th[n_bonds + 2 * L:]


def model_from_theta(ctx: Context, L: int, bonds, theta) -> Model:
    bonds = np.asarray(bonds, dtype=np.int32).reshape(-1, 2)
    t, eu, ed, U = split_theta(L, len(bonds), theta)
    return Model(ctx, L, bonds, t, eu, ed, U)


class _GreensNeq(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta_ini, theta, kctx, L, bonds_ini, bonds, sector, v0, orbitals, nt, spg, dt, kw):
        m_ini = model_from_theta(kctx, L, bonds_ini, theta_ini.detach().cpu().numpy())
        m_fin = model_from_theta(kctx, L, bonds, theta.detach().cpu().numpy())
        out = kctx.greens_neq(m_ini, m_fin, sector, v0, orbitals, nt, spg, dt, schedule=0,
                              krylov_dim=kw["krylov_dim"], reorth=kw["reorth"], gs_tol=kw["gs_tol"],
                              gs_max_iter=kw["gs_max_iter"])
        fctx.save_for_backward(theta_ini, theta)
        fctx.args = (kctx, L, bonds_ini, bonds, sector, v0, orbitals, nt, spg, dt, kw)
        return torch.from_numpy(out["G_lesser"]), torch.from_numpy(out["G_greater"])

    @staticmethod
    def backward(fctx, gl, gg):
        theta_ini, theta = fctx.saved_tensors
        kctx, L, bonds_ini, bonds, sector, v0, orbitals, nt, spg, dt, kw = fctx.args
        m_ini = model_from_theta(kctx, L, bonds_ini, theta_ini.detach().cpu().numpy())
        m_fin = model_from_theta(kctx, L, bonds, theta.detach().cpu().numpy())
        Wl = None if gl is None else gl.detach().cpu().numpy()
        Wg = None if gg is None else gg.detach().cpu().numpy()
        r = kctx.greens_neq_vjp(m_ini, m_fin, sector, v0, orbitals, nt, spg, dt, Wl, Wg,
                                krylov_dim=kw["krylov_dim"], reorth=kw["reorth"], quad_nodes=kw["quad_nodes"],
                                cg_tol=kw["cg_tol"], gs_tol=kw["gs_tol"], gs_max_iter=kw["gs_max_iter"])
        gi = torch.from_numpy(r["grad_ini"]).to(theta_ini.dtype)
        g = torch.from_numpy(r["grad"]).to(theta.dtype)
        return (gi, g) + (None,) * 11


def greens_neq(kctx: Context, L: int, bonds_ini, bonds, theta_ini: torch.Tensor, theta: torch.Tensor,
               sector: Sector, v0, orbitals: Sequence[Tuple[int, int]], nt: int, steps_per_grid: int, dt: float,
               krylov_dim: int = 15, reorth: int = 0, quad_nodes: int = 12, cg_tol: float = 1e-12,
               gs_tol: float = 1e-12, gs_max_iter: int = 300):
    """Differentiable four-step (G^<, G^>) on the mesh t_k = k steps_per_grid dt."""
    kw = dict(krylov_dim=krylov_dim, reorth=reorth, quad_nodes=quad_nodes, cg_tol=cg_tol, gs_tol=gs_tol,
              gs_max_iter=gs_max_iter)
    return _GreensNeq.apply(theta_ini, theta, kctx, L, bonds_ini, bonds, sector, v0, list(orbitals), nt,
                            steps_per_grid, dt, kw)


class _GreensNeqBatch(torch.autograd.Function):
    @staticmethod
    def forward(fctx, meta, *thetas):
        n = meta["n"]
        kctx = meta["kctx"]
        mi = [model_from_theta(kctx, meta["L"][i], meta["bonds_ini"][i], thetas[i].detach().cpu().numpy())
              for i in range(n)]
        mf = [model_from_theta(kctx, meta["L"][i], meta["bonds"][i], thetas[n + i].detach().cpu().numpy())
              for i in range(n)]
        kw = meta["kw"]
        out = kctx.greens_neq_multi(mi, mf, meta["sectors"], meta["v0"], meta["orbitals"], meta["nt"], meta["spg"],
                                    meta["dt"], krylov_dim=kw["krylov_dim"], reorth=kw["reorth"],
                                    gs_tol=kw["gs_tol"], gs_max_iter=kw["gs_max_iter"])
        fctx.meta = meta
        fctx.save_for_backward(*thetas)
        return torch.from_numpy(out["G_lesser"]), torch.from_numpy(out["G_greater"])

    @staticmethod
    def backward(fctx, gl, gg):
        meta = fctx.meta
        thetas = fctx.saved_tensors
        n, kctx, kw = meta["n"], meta["kctx"], meta["kw"]
        mi = [model_from_theta(kctx, meta["L"][i], meta["bonds_ini"][i], thetas[i].detach().cpu().numpy())
              for i in range(n)]
        mf = [model_from_theta(kctx, meta["L"][i], meta["bonds"][i], thetas[n + i].detach().cpu().numpy())
              for i in range(n)]
        Wl = None if gl is None else [gl[i].detach().cpu().numpy() for i in range(n)]
        Wg = None if gg is None else [gg[i].detach().cpu().numpy() for i in range(n)]
        rs = kctx.greens_neq_vjp_multi(mi, mf, meta["sectors"], meta["v0"], meta["orbitals"], meta["nt"], meta["spg"],
                                       meta["dt"], Wl, Wg, krylov_dim=kw["krylov_dim"], reorth=kw["reorth"],
                                       quad_nodes=kw["quad_nodes"], cg_tol=kw["cg_tol"], gs_tol=kw["gs_tol"],
                                       gs_max_iter=kw["gs_max_iter"])
        grads = [torch.from_numpy(rs[i]["grad_ini"]).to(thetas[i].dtype) for i in range(n)]
        grads += [torch.from_numpy(rs[i]["grad"]).to(thetas[n + i].dtype) for i in range(n)]
        return (None,) + tuple(grads)


def greens_neq_batch(kctx: Context, L: Sequence[int], bonds_ini, bonds, theta_ini: Sequence[torch.Tensor],
                     theta: Sequence[torch.Tensor], sectors: Sequence[Sector], v0, orbitals: Sequence[Tuple[int, int]],
                     nt: int, steps_per_grid: int, dt: float, krylov_dim: int = 15, reorth: int = 0,
                     quad_nodes: int = 12, cg_tol: float = 1e-12, gs_tol: float = 1e-12, gs_max_iter: int = 300):
    """Differentiable four-step (G^<, G^>) of n instances, stacked as
    [n][nt][nt][n_orb][n_orb].  Forward through kgf_greens_neq_multi and
    backward through kgf_greens_neq_vjp_multi: instances with one sector and
    bond list run as one batch in both."""
    n = len(theta)
    meta = dict(n=n, kctx=kctx, L=list(L), bonds_ini=list(bonds_ini), bonds=list(bonds), sectors=list(sectors),
                v0=list(v0), orbitals=list(orbitals), nt=nt, spg=steps_per_grid, dt=dt,
                kw=dict(krylov_dim=krylov_dim, reorth=reorth, quad_nodes=quad_nodes, cg_tol=cg_tol, gs_tol=gs_tol,
                        gs_max_iter=gs_max_iter))
    return _GreensNeqBatch.apply(meta, *theta_ini, *theta)
