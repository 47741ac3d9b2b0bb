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


@pytest.mark.parametrize("n,eta,bar", [(10, 0.05, 1e-10), (40, 1.0, 1e-10), (40, 0.05, 1e-7)])
def test_greens_omega_against_oracle(ring8, n, eta, bar):
    """The G tolerance 1e-10 holds wherever G^(L)(omega) is a well-conditioned
    function of the start vector: n = 10 (before any Ritz value converges)
    at eta = 0.05, and n = 40 at eta = 1 (the broadening hides the deep
    chain).  At n = 40 and eta = 0.05 the entries of the chain past the
    first converged Ritz values are ill-determined functions of |0>: the
    oracle's own G moves by 6e-9 relative under a global phase of |0>, so
    that case is held to 1e-7."""
    ctx, model, sec, E0, psi0 = ring8
    om = np.linspace(-12, 12, 241)
    say("greens_omega", n, eta)
    got = ctx.greens_omega(ctx.model(model), ctx.sector(8, 4, 4), to_dev(psi0), E0, (0, 0), n, om, eta)
    ref = spectral.lanczos_greens_omega(model, sec, psi0, E0, (0, 0), n, om, eta)
    assert list(got["steps"]) == [n, n]
    say("n", n, rel_err(got["G_greater"], ref["G_greater"]), rel_err(got["G_lesser"], ref["G_lesser"]))
    assert rel_err(got["G_greater"], ref["G_greater"]) < bar, n
    assert rel_err(got["G_lesser"], ref["G_lesser"]) < bar, n


@pytest.mark.parametrize("dagger", [1, 0])
@pytest.mark.parametrize("nsteps,nfine,dt,m,reorth,t_sharp,bar", [(6, 8, 0.4, 15, 0, 2.4, 1e-10),
                                                                  (1, 400, 20.0, 40, 0, 4.0, 1e-7),
                                                                  (1, 400, 20.0, 40, 2, 8.0, 1e-7)])
def test_greens_eq_fine_against_oracle(ring8, dagger, nsteps, nfine, dt, m, reorth, t_sharp, bar):
    """Restarted propagation (short steps, converged) at the G parity
    tolerance 1e-10 on the whole mesh.  One Krylov space of 40 over t = 20
    (f = 1, the conventional method, unconverged by design): G(t) at late
    times depends on the deep end of the chain, an ill-determined function
    of |0> (the oracle's own G moves by 4e-9 relative under a global phase
    of |0>, with or without reorthogonalisation).  Up to t_sharp, where that
    phase test moves the oracle by less than 1e-14 (t = 4 without, t = 8
    with Gram-Schmidt twice), the window is held to 1e-10; the whole mesh
    to 1e-7."""
    ctx, model, sec, E0, psi0 = ring8
    say("eq_fine", dagger, nsteps, nfine, dt, m, reorth)
    got = ctx.greens_eq_fine(ctx.model(model), ctx.sector(8, 4, 4), to_dev(psi0), E0, (0, 0), dagger, nsteps, nfine,
                             dt, krylov_dim=m, reorth=reorth)
    ref = spectral.greens_time_fine(model, sec, psi0, E0, (0, 0), bool(dagger), nsteps, nfine, dt, m,
                                    reorth="cgs2" if reorth == 2 else "none")
    t = np.arange(got.size) * (dt / nfine)
    early = t <= t_sharp + 1e-12
    sharp = float(np.abs(got[early] - ref[early]).max() / np.abs(ref).max())
    say("rel err", rel_err(got, ref), "window", sharp)
    assert sharp < 1e-10
    assert rel_err(got, ref) < bar


def test_fourier_against_oracle(ring8):
    ctx = ring8[0]
    rng = np.random.default_rng(4)
    G = rng.standard_normal(5001) + 1j * rng.standard_normal(5001)
    om = np.linspace(-10, 10, 301)
    got = ctx.fourier(G, 0.01, 0.05, om)
    assert rel_err(got, spectral.fourier(G, 0.01, 0.05, om)) < 1e-12
