"""A four-time two-particle Green's function by the four-step idea (test
infrastructure only; the product path never imports this module).

The paper's outlook (Sec. 6) names higher-order Green's functions, with four
independent time arguments, as the next use of the Krylov approach.  This
module computes the real-time component

    chi_abcd(t1, t2, t3, t4) = <0| c+_a(t1) c+_b(t2) c_c(t3) c_d(t4) |0>,

Heisenberg operators c(t) = e^{iHt} c e^{-iHt} after the ground state |0> of
H_ini (the quench of Sec. 4).  With the two-time states

    Psi_xy(s, u) = c_x(s) c_y(u) |0>
                 = e^{iHs} c_x e^{-iH(s-u)} c_y e^{-iHu} |0>

(in the sector with two particles fewer), chi_abcd(t1, t2, t3, t4) =
<Psi_ba(t2, t1) | Psi_cd(t3, t4)>: the four-step procedure with one more
annihilator and one more propagation in between.  Any other real-time
ordering of two c and two c+, <0| O1_a(t1) O2_b(t2) O3_c(t3) O4_d(t4) |0>
with O = c or c+ (the `pattern` of dagger flags), is the scalar product of
the states O2_b(t2)^+ O1_a(t1)^+ |0> and O3_c(t3) O4_d(t4) |0>, built the
same way.  Everything here is dense and exact (eigen-decomposition of H_ini,
matrix exponentials of H), for small sectors only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .basis import Sector
from .hamiltonian import Hamiltonian, apply_ladder


def _shift(sec: Sector, spin: int, delta: int):
    nu = sec.n_up + (delta if spin == 0 else 0)
    nd = sec.n_dn + (delta if spin == 1 else 0)
    if nu < 0 or nd < 0 or nu > sec.L or nd > sec.L:
        return None
    return Sector(sec.L, nu, nd)


def four_time(H_ini, H, n_up: int, n_dn: int, orbitals, times, pattern=(1, 1, 0, 0)):
    """chi[i1, i2, i3, i4, a, b, c, d] = <0| O1_a(t_i1) O2_b(t_i2) O3_c(t_i3) O4_d(t_i4) |0>,
    O_k = c+ where pattern[k] else c (default c+ c+ c c), for orbitals =
    [(site, spin)] and the time list `times`; also returns E0.  The ground
    state of H_ini must be nondegenerate."""
    sec = Sector(H_ini.L, n_up, n_dn)
    e, v = np.linalg.eigh(Hamiltonian(H_ini, sec).dense())
    assert e[1] - e[0] > 1e-9, "degenerate ground state"
    g = v[:, 0].astype(np.complex128)
    expm = {}

    def U(s: Sector, t: float):
        key = (s.n_up, s.n_dn, t)
        if key not in expm:
            expm[key] = scipy.linalg.expm(-1j * t * Hamiltonian(H, s).dense())
        return expm[key]

    times = [float(t) for t in times]
    nt, no = len(times), len(orbitals)

    def two_time_states(dx: int, dy: int):
        """(x, y, i_s, i_u) -> (o_x(t_s) o_y(t_u)|0>, sector key), o = c+ where d = 1."""
        states = {}
        for y, (sy, spy) in enumerate(orbitals):
            s1 = _shift(sec, spy, 1 if dy else -1)
            for iu, u in enumerate(times):
                if s1 is not None and s1.dim:
                    w1, _ = apply_ladder(sec, sy, spy, bool(dy), U(sec, u) @ g)       # o_y e^{-iHu}|0>
                for x, (sx, spx) in enumerate(orbitals):
                    s2 = _shift(s1, spx, 1 if dx else -1) if s1 is not None else None
                    for is_, s_ in enumerate(times):
                        if s1 is None or s2 is None or s1.dim == 0 or s2.dim == 0:
                            states[(x, y, is_, iu)] = (None, None)
                            continue
                        w2, _ = apply_ladder(s1, sx, spx, bool(dx), U(s1, s_ - u) @ w1)   # o_x e^{-iH(s-u)} ...
                        states[(x, y, is_, iu)] = (U(s2, s_).conj().T @ w2, (s2.n_up, s2.n_dn))
        return states
    p1, p2, p3, p4 = (int(bool(q)) for q in pattern)
    kets = two_time_states(p3, p4)                       # O3_c(t3) O4_d(t4)|0>
    bras = kets if (1 - p2, 1 - p1) == (p3, p4) else two_time_states(1 - p2, 1 - p1)   # O2_b^+ O1_a^+ |0>
    chi = np.zeros((nt, nt, nt, nt, no, no, no, no), dtype=np.complex128)
    for i1 in range(nt):
        for i2 in range(nt):
            for a in range(no):
                for b in range(no):
                    bra, kb = bras[(b, a, i2, i1)]
                    if bra is None:
                        continue
                    for i3 in range(nt):
                        for i4 in range(nt):
                            for c in range(no):
                                for d in range(no):
                                    ket, kk = kets[(c, d, i3, i4)]
                                    if ket is not None and kk == kb:
                                        chi[i1, i2, i3, i4, a, b, c, d] = np.vdot(bra, ket)
    return {"chi": chi, "E0": float(e[0])}
