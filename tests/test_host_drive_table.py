"""Host logic of the driven entry points (no GPU): the binding samples the
drive at the two Gauss nodes of every commutator-free step; the stage
parameters built from that table must agree with the oracle's independent
definition of the stages."""
from types import SimpleNamespace

import numpy as np

import workloads as wl
from oracle import driven
from oracle.gradients import theta_of


def test_drive_table_matches_the_oracle_stages():
    from paper_1109_1205_amd._lib import Context
    H0 = wl.ring(6, 1.0, 2.0)
    nb, L = len(H0.bonds), H0.L
    k0 = np.zeros(nb + 3 * L)
    k0[2] = 1.0
    thetas = np.stack([theta_of(H0), k0])
    f = lambda t: [1.0, 0.7 * np.sin(1.3 * t) + 0.1 * t]
    nsteps, h, t0 = 5, 0.07, 0.3
    work = SimpleNamespace(_bi=list(range(nb)), L=L)
    me = SimpleNamespace(DRIVE_NODES=Context.DRIVE_NODES)
    th, fv = Context._drive_table(me, work, thetas, f, nsteps, h, t0)
    assert fv.shape == (nsteps, 2, 2) and np.array_equal(th, thetas)
    a1, a2 = driven.A1, driven.A2
    for n in range(nsteps):
        b1, b2 = driven.stage_thetas(thetas, f, t0 + n * h, h)
        np.testing.assert_allclose((a2 * fv[n, 0] + a1 * fv[n, 1]) @ th, b1, rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose((a1 * fv[n, 0] + a2 * fv[n, 1]) @ th, b2, rtol=1e-14, atol=1e-15)
    # no steps: a zero placeholder row, never read
    _, fz = Context._drive_table(me, work, thetas, f, 0, h, t0)
    assert fz.shape == (1, 2, 2) and not fz.any()
