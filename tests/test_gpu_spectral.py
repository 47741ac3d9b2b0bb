"""Equilibrium spectra (Secs. 2-3) through the C ABI vs the oracle:
conventional Lanczos G(omega) (continued fraction on the GPU, pole sum over
Ritz pairs in the oracle), time-dependent Lanczos G(t) on a fine grid
(restarts every dt, intermediate times from each step's Krylov space,
including the single-Krylov-space case f = 1 with the eigendecomposition
path), and the damped Fourier transform."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say, to_dev, to_host
from oracle import basis, hamiltonian, lanczos, spectral

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ring8():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    ctx = k.Context(0)
    q = wl.ring8()
    sec = basis.Sector(8, 4, 4)
    H = hamiltonian.Hamiltonian(q.H, sec)
    gs = lanczos.ground_state(H.apply, wl.start_vector(sec.dim, 7), tol=1e-13, max_iter=400)
    return ctx, q.H, sec, gs.E0, gs.psi


def test_greens_omega_against_oracle(ring8):
    """Bars from the conditioning of the n-pole function at eta = 0.05: the
    oracle's own G^(L) at n = 40 moves by 2e-8 relative when only the global
    phase of |0> changes (a rounding-level change of the recursion), so
    n = 40 is held to 1e-7; n = 10 (poles well separated) to 1e-9."""
    ctx, model, sec, E0, psi0 = ring8
    om = np.linspace(-12, 12, 241)
    say("greens_omega")
    for n, bar in ((10, 1e-9), (40, 1e-7)):
        got = ctx.greens_omega(ctx.model(model), ctx.sector(8, 4, 4), to_dev(psi0), E0, (0, 0), n, om, 0.05)
        ref = spectral.lanczos_greens_omega(model, sec, psi0, E0, (0, 0), n, om, 0.05)
        assert list(got["steps"]) == [n, n]
        say("n", n, rel_err(got["G_greater"], ref["G_greater"]), rel_err(got["G_lesser"], ref["G_lesser"]))
        assert rel_err(got["G_greater"], ref["G_greater"]) < bar, n
        assert rel_err(got["G_lesser"], ref["G_lesser"]) < bar, n


@pytest.mark.parametrize("dagger", [1, 0])
@pytest.mark.parametrize("nsteps,nfine,dt,m,bar", [(6, 8, 0.4, 15, 1e-10), (1, 400, 20.0, 40, 1e-7)])
def test_greens_eq_fine_against_oracle(ring8, dagger, nsteps, nfine, dt, m, bar):
    """Restarted propagation (short steps, converged) at the G parity tolerance 1e-10;
    one Krylov space of 40 over t = 20 (f = 1, the conventional method,
    unconverged by design) at 1e-7: there the oracle itself moves by 1e-8
    relative when only the global phase of |0> changes."""
    ctx, model, sec, E0, psi0 = ring8
    say("eq_fine", dagger, nsteps, nfine, dt, m)
    got = ctx.greens_eq_fine(ctx.model(model), ctx.sector(8, 4, 4), to_dev(psi0), E0, (0, 0), dagger, nsteps, nfine,
                             dt, krylov_dim=m)
    ref = spectral.greens_time_fine(model, sec, psi0, E0, (0, 0), bool(dagger), nsteps, nfine, dt, m)
    say("rel err", rel_err(got, ref))
    assert rel_err(got, ref) < bar


def test_fourier_against_oracle(ring8):
    ctx = ring8[0]
    rng = np.random.default_rng(4)
    G = rng.standard_normal(5001) + 1j * rng.standard_normal(5001)
    om = np.linspace(-10, 10, 301)
    got = ctx.fourier(G, 0.01, 0.05, om)
    assert rel_err(got, spectral.fourier(G, 0.01, 0.05, om)) < 1e-12
