"""Pins of the equilibrium-spectrum oracle (CPU only): the Lanczos Green's
function at full Krylov depth equals the dense resolvent; the fine-grid
time-dependent G equals the dense exponential; the trapezoid transform of a
single exponential equals its geometric-series closed form."""
import numpy as np
import scipy.linalg as sla

import workloads as wl
from oracle import basis, hamiltonian, lanczos, spectral


def _gs(model, nu, nd):
    sec = basis.Sector(model.L, nu, nd)
    H = hamiltonian.Hamiltonian(model, sec)
    gs = lanczos.ground_state(H.apply, wl.start_vector(sec.dim, 7), tol=1e-13, max_iter=400)
    return sec, gs.E0, gs.psi


def test_lanczos_greens_omega_full_depth_is_the_resolvent():
    model = wl.ring(6, 1.0, 4.0).with_field(0, 0.3)
    sec, E0, psi0 = _gs(model, 3, 3)
    om = np.linspace(-8, 8, 41)
    eta = 0.1
    G = spectral.lanczos_greens_omega(model, sec, psi0, E0, (0, 0), 200, om, eta)
    for greater in (True, False):
        i0, tgt = hamiltonian.apply_ladder(sec, 0, 0, greater, psi0)
        Hd = hamiltonian.Hamiltonian(model, tgt).dense()
        ref = []
        for w in om:
            z = w + 1j * eta
            A = (z + E0) * np.eye(tgt.dim) - Hd if greater else (z - E0) * np.eye(tgt.dim) + Hd
            ref.append(np.vdot(i0, np.linalg.solve(A, i0)))
        got = G["G_greater" if greater else "G_lesser"]
        assert np.abs(got - np.array(ref)).max() < 1e-10 * np.abs(ref).max()


def test_greens_time_fine_matches_dense_exponential():
    model = wl.chain_siam(5, 2.0)
    sec, E0, psi0 = _gs(model, 3, 2)
    for dagger in (True, False):
        G = spectral.greens_time_fine(model, sec, psi0, E0, (0, 0), dagger, 4, 5, 0.5, 20)
        i0, tgt = hamiltonian.apply_ladder(sec, 0, 0, dagger, psi0)
        Hd = hamiltonian.Hamiltonian(model, tgt).dense()
        d = -1 if dagger else 1
        pf = -1.0 if dagger else 1.0
        t = 0.1 * np.arange(21)
        ref = [pf * 1j * np.vdot(i0, sla.expm(d * 1j * Hd * tt) @ i0) * np.exp(-1j * d * E0 * tt) for tt in t]
        assert np.abs(G - np.array(ref)).max() < 1e-12


def test_fourier_trapezoid_geometric_series():
    eps, dt, n, eta = 1.3, 0.01, 3001, 0.05
    G = -1j * np.exp(-1j * eps * dt * np.arange(n))
    om = np.linspace(-4, 4, 17)
    got = spectral.fourier(G, dt, eta, om)
    r = np.exp((1j * (om - eps) - eta) * dt)
    # sum_{k<n} r^k minus half of the first and last terms, times dt, times -i
    ref = -1j * dt * ((1 - r ** n) / (1 - r) - 0.5 - 0.5 * r ** (n - 1))
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
