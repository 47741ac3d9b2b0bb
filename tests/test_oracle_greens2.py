"""Pins of the four-time two-particle oracle
chi_abcd(t1,t2,t3,t4) = <0| c+_a(t1) c+_b(t2) c_c(t3) c_d(t4) |0>
against facts that do not depend on it:

* U = 0: Wick's theorem, chi = <c+_a c_d><c+_b c_c> - <c+_a c_c><c+_b c_d>
  with the two-point functions of the one-particle Hamiltonian (exact free
  propagation of the Slater determinant);
* any U: summing b = c over all spin orbitals at equal times t2 = t3 gives
  (N - 1) <c+_a(t1) c_d(t4)> (the number operator between them counts N - 1
  particles), i.e. (N - 1)(-i) G^<_da(t4, t1) of the pinned single-particle
  four-step; at t = 0, sum_ab <c+_a c+_b c_b c_a> = N (N - 1);
* H_ini = H: invariance under a common shift of the four times;
* equal times: antisymmetry in (c, d) and in (a, b)."""
import numpy as np
import scipy.linalg

import workloads as wl
from oracle import basis, greens, greens2, necpt

ALL4 = [(i, s) for s in (0, 1) for i in range(4)]


def test_u0_wick():
    H = wl.chain_siam(4, 0.0, 1.0)
    Hi = H.with_field(0, 0.2)
    times = [0.0, 0.4, 1.1]
    chi = greens2.four_time(Hi, H, 2, 2, ALL4, times)["chi"]

    def h1(M, spin):
        h = np.diag(np.asarray(M.eps_up if spin == 0 else M.eps_dn, float))
        for (i, j), t in zip(M.bonds, M.t):
            h[i, j] -= t
            h[j, i] -= t
        return h
    rho = [necpt.ground_density(h1(Hi, s), 2) for s in (0, 1)]
    Ut = {(s, k): scipy.linalg.expm(-1j * h1(H, s) * t) for s in (0, 1) for k, t in enumerate(times)}

    def cd(x, s, y, u):        # <c+_x(t_s) c_y(t_u)>
        (ix, sx), (iy, sy) = ALL4[x], ALL4[y]
        if sx != sy:
            return 0.0
        return (Ut[(sx, u)] @ rho[sx] @ Ut[(sx, s)].conj().T)[iy, ix]
    no, nt = len(ALL4), len(times)
    ref = np.zeros_like(chi)
    for i1 in range(nt):
        for i2 in range(nt):
            for i3 in range(nt):
                for i4 in range(nt):
                    for a in range(no):
                        for b in range(no):
                            for c in range(no):
                                for d in range(no):
                                    ref[i1, i2, i3, i4, a, b, c, d] = (cd(a, i1, d, i4) * cd(b, i2, c, i3)
                                                                       - cd(a, i1, c, i3) * cd(b, i2, d, i4))
    assert np.abs(ref).max() > 0.1
    assert np.abs(chi - ref).max() < 1e-12


def test_contraction_to_the_single_particle_four_step():
    H = wl.chain_siam(4, 2.0, 1.0)
    Hi = H.with_field(0, 0.2)
    nt, dtg = 3, 0.2
    out = greens2.four_time(Hi, H, 2, 2, ALL4, [k * dtg for k in range(nt)])
    chi = out["chi"]
    N = 4
    assert abs(np.einsum("abba->", chi[0, 0, 0, 0]) - N * (N - 1)) < 1e-12
    sec = basis.Sector(4, 2, 2)
    g1 = greens.four_step(Hi, H, 2, 2, ALL4, nt, dtg, 4, 15, wl.start_vector(sec.dim, 7), gs_tol=1e-13)
    assert abs(g1["E0"] - out["E0"]) < 1e-11
    for j in range(nt):
        lhs = np.einsum("pqabbd->pqad", chi[:, j, j, :])          # [i1, i4, a, d]
        rhs = (N - 1) * (-1j) * np.transpose(g1["G_lesser"], (1, 0, 3, 2))   # G^<_da(t4, t1) -> [t1, t4, a, d]
        assert np.abs(lhs - rhs).max() < 1e-9


def test_equilibrium_time_translation_and_antisymmetry():
    H = wl.chain_siam(4, 2.0, 1.0).with_field(0, 0.2)   # H_ini = H: a stationary state
    orbs = [(0, 0), (1, 0), (0, 1), (3, 1)]
    chi = greens2.four_time(H, H, 2, 2, orbs, [0.0, 0.3, 0.6, 0.9])["chi"]
    assert np.abs(chi).max() > 0.05
    assert np.abs(chi[1:, 1:, 1:, 1:] - chi[:-1, :-1, :-1, :-1]).max() < 1e-12
    for k in range(4):
        assert np.abs(chi[:, :, k, k] + np.swapaxes(chi[:, :, k, k], -1, -2)).max() < 1e-13
        assert np.abs(chi[k, k] + np.swapaxes(chi[k, k], -4, -3)).max() < 1e-13


PATTERNS = [(1, 1, 0, 0), (1, 0, 1, 0), (1, 0, 0, 1), (0, 1, 1, 0), (0, 0, 1, 1)]


def test_u0_wick_all_orderings():
    """<O1 O2 O3 O4> = <O1O2><O3O4> - <O1O3><O2O4> + <O1O4><O2O3> at U = 0
    for every ordering of two c and two c+ (<c c> = <c+ c+> = 0)."""
    H = wl.chain_siam(4, 0.0, 1.0)
    Hi = H.with_field(0, 0.2)
    orbs = [(0, 0), (1, 0), (0, 1), (2, 1)]
    times = [0.0, 0.5, 1.2]

    def h1(M, spin):
        h = np.diag(np.asarray(M.eps_up if spin == 0 else M.eps_dn, float))
        for (i, j), t in zip(M.bonds, M.t):
            h[i, j] -= t
            h[j, i] -= t
        return h
    rho = [necpt.ground_density(h1(Hi, s), 2) for s in (0, 1)]
    Ut = {(s, k): scipy.linalg.expm(-1j * h1(H, s) * t) for s in (0, 1) for k, t in enumerate(times)}

    def two(dag1, o1, k1, dag2, o2, k2):      # <O1(t_k1) O2(t_k2)>
        (i1, s1), (i2, s2) = orbs[o1], orbs[o2]
        if s1 != s2 or dag1 == dag2:
            return 0.0
        if dag1:                               # <c+_x(s) c_y(u)> = [U(u) rho U(s)^+]_{yx}
            return (Ut[(s1, k2)] @ rho[s1] @ Ut[(s1, k1)].conj().T)[i2, i1]
        return (Ut[(s1, k1)] @ (np.eye(4) - rho[s1]) @ Ut[(s1, k2)].conj().T)[i1, i2]   # <c_x(s) c+_y(u)>
    nt, no = len(times), len(orbs)
    for pat in PATTERNS:
        chi = greens2.four_time(Hi, H, 2, 2, orbs, times, pattern=pat)["chi"]
        ref = np.zeros_like(chi)
        for idx in np.ndindex(chi.shape):
            k, o = idx[:4], idx[4:]
            q = [(pat[m], o[m], k[m]) for m in range(4)]
            ref[idx] = (two(*q[0], *q[1]) * two(*q[2], *q[3]) - two(*q[0], *q[2]) * two(*q[1], *q[3])
                        + two(*q[0], *q[3]) * two(*q[1], *q[2]))
        assert np.abs(ref).max() > 0.1, pat
        assert np.abs(chi - ref).max() < 1e-12, pat


def test_number_operator_contraction_interacting():
    """U = 2, ordering c+ c c+ c: sum_a <c+_a(t) c_a(t) c+_c(t3) c_d(t4)> =
    N <c+_c(t3) c_d(t4)> (N conserved), against the single-particle four-step."""
    H = wl.chain_siam(4, 2.0, 1.0)
    Hi = H.with_field(0, 0.2)
    nt, dtg, N = 3, 0.2, 4
    chi = greens2.four_time(Hi, H, 2, 2, ALL4, [k * dtg for k in range(nt)], pattern=(1, 0, 1, 0))["chi"]
    sec = basis.Sector(4, 2, 2)
    g1 = greens.four_step(Hi, H, 2, 2, ALL4, nt, dtg, 4, 15, wl.start_vector(sec.dim, 7), gs_tol=1e-13)
    rhs = N * (-1j) * np.transpose(g1["G_lesser"], (1, 0, 3, 2))       # [t3, t4, c, d]
    for j in range(nt):
        lhs = np.einsum("pqaacd->pqcd", chi[j, j])
        assert np.abs(lhs - rhs).max() < 1e-9
