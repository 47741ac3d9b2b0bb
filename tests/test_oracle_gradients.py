"""Pins of the dense gradient references (CPU only): exact derivatives
(Frechet derivative of the matrix exponential, first-order ground-state
perturbation) against central differences of the dense exact forward
computation, and the four-step G with exact exponentials against the
oracle's Krylov four-step."""
import numpy as np

import workloads as wl
from oracle import basis, gradients, greens


def test_propagation_gradient_against_differences():
    model = wl.chain_siam(5, 2.0).with_field(0, 0.3)
    sec = basis.Sector(5, 3, 2)
    psi0, chi = wl.complex_vector(sec.dim, 1), wl.complex_vector(sec.dim, 2)
    for direction in (-1, 1):
        g = gradients.propagation_gradient(model, sec, psi0, chi, 0.7, direction)
        th = gradients.theta_of(model)
        h = 1e-6
        fd = []
        for p in range(len(th)):
            e = np.zeros(len(th))
            e[p] = h
            f = [np.vdot(chi, gradients.propagation_exact(gradients.model_with_theta(model, th + s * e), sec, psi0,
                                                          0.7, direction)).real for s in (1, -1)]
            fd.append((f[0] - f[1]) / (2 * h))
        assert np.abs(g - np.array(fd)).max() <= 1e-7 * np.abs(g).max()


def test_four_step_exact_matches_krylov_oracle():
    H = wl.chain_siam(4, 2.0)
    Hi = H.with_field(0, 0.4)
    times = [0.0, 0.2, 0.4]
    ex = gradients.four_step_exact(Hi, H, 2, 2, [(0, 0), (1, 1)], times)
    sec = basis.Sector(4, 2, 2)
    kr = greens.four_step(Hi, H, 2, 2, [(0, 0), (1, 1)], 3, 0.2, 2, 14, wl.start_vector(sec.dim, 7), gs_tol=1e-13)
    assert np.abs(ex["G_lesser"] - kr["G_lesser"]).max() < 1e-11
    assert np.abs(ex["G_greater"] - kr["G_greater"]).max() < 1e-11


def test_four_step_gradient_against_differences():
    H = wl.chain_siam(4, 2.0)
    Hi = gradients.model_with_theta(H.with_field(0, 0.4), gradients.theta_of(H.with_field(0, 0.4)) * 1.03)
    orbs, times = [(0, 0), (1, 1)], [0.0, 0.3, 0.6]
    rng = np.random.default_rng(3)
    shape = (3, 3, 2, 2)
    Wl = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    Wg = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    gi, g, _ = gradients.four_step_gradient(Hi, H, 2, 2, orbs, times, Wl, Wg)

    def loss(mi, mf):
        G = gradients.four_step_exact(mi, mf, 2, 2, orbs, times)
        return float((np.sum(np.conj(Wl) * G["G_lesser"]) + np.sum(np.conj(Wg) * G["G_greater"])).real)
    h = 1e-6
    for which, grad, base in (("fin", g, H), ("ini", gi, Hi)):
        th = gradients.theta_of(base)
        fd = []
        for p in range(len(th)):
            e = np.zeros(len(th))
            e[p] = h
            mp, mm = gradients.model_with_theta(base, th + e), gradients.model_with_theta(base, th - e)
            fd.append((loss(Hi, mp) - loss(Hi, mm)) / (2 * h) if which == "fin" else
                      (loss(mp, H) - loss(mm, H)) / (2 * h))
        assert np.abs(grad - np.array(fd)).max() <= 1e-7 * np.abs(grad).max(), which
