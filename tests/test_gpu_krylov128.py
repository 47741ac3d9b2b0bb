"""SIL Krylov dimensions above one wavefront (65..128): the two-wavefront
tridiagonal exponential, both of its paths (Taylor substeps for moderate
||T dt||, the QL eigen-decomposition beyond), against the oracle's SIL step
at the same dimension.  The cases are well conditioned (a global phase on
the input moves the oracle's result by <= 1.2e-13 relative) and, except
m = 80 at dt = 6, converged to the exact propagator."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say, to_dev, to_host
from oracle import basis, hamiltonian, propagate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    q = wl.ring8()
    sec = basis.Sector(8, 4, 4)
    return k.Context(0), q.H, sec, hamiltonian.Hamiltonian(q.H, sec)


@pytest.mark.parametrize("m,dt,nsteps", [(100, 0.05, 2), (100, 3.0, 1), (100, 6.0, 1), (80, 6.0, 1), (128, 8.0, 1),
                                         (65, 0.05, 3)])
def test_sil_large_krylov_dimension(env, m, dt, nsteps):
    ctx, H, sec, Hh = env
    X = np.stack([wl.complex_vector(sec.dim, 50 + c) for c in range(2)])
    ref = np.stack([propagate.propagate(Hh.apply, X[c], dt, nsteps, m, -1, 0.0, "cgs2") for c in range(2)])
    say("SIL m", m, "dt", dt, "steps", nsteps)
    got = to_host(ctx.propagate(ctx.model(H), ctx.sector(8, 4, 4), to_dev(X), nsteps, dt, m, -1, 0.0, 2))
    err = rel_err(got, ref)
    say("rel err", err)
    assert err < 1e-11


def test_krylov_dimension_limit(env):
    ctx, H, sec, _ = env
    X = to_dev(wl.complex_vector(sec.dim, 50).reshape(1, -1))
    with pytest.raises(RuntimeError):
        ctx.propagate(ctx.model(H), ctx.sector(8, 4, 4), X, 1, 0.05, 129, -1, 0.0, 2)
