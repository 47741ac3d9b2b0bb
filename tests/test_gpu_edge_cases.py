"""Edge cases through the C ABI: a full band (empty c+ sector), more columns
than one launch holds, degenerate sizes and the errors the library reports
for invalid input (host-side checks; no kernel runs on bad input)."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say, to_dev, to_host
from oracle import basis, greens, hamiltonian

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    return k, k.Context(0)


def test_full_band_greater_is_zero_and_lesser_matches_oracle(kctx):
    """Up band full (N_up = L): no c+ states, so G^> of the up orbital is
    exactly zero; G^< follows the oracle."""
    k, ctx = kctx
    H = wl.ring(4, 1.0, 3.0, periodic=False).with_field(1, 0.2)
    Hi = H.with_U([1.0] * 4)
    sec = basis.Sector(4, 4, 2)
    v0 = wl.start_vector(sec.dim, 7)
    say("full band")
    out = ctx.greens_neq(ctx.model(Hi), ctx.model(H), ctx.sector(4, 4, 2), to_dev(v0), orbitals=[(0, 0), (2, 1)],
                         nt=4, steps_per_grid=2, dt=0.05, krylov_dim=6, schedule=1)
    ora = greens.four_step(Hi, H, 4, 2, [(0, 0), (2, 1)], 4, 0.1, 2, 6, v0, gs_tol=1e-12, reorth="none")
    assert np.all(out["G_greater"][:, :, 0, 0] == 0)
    assert rel_err(out["G_lesser"], ora["G_lesser"]) < 1e-10
    assert rel_err(out["G_greater"], ora["G_greater"]) < 1e-10


def test_apply_h_more_columns_than_one_launch(kctx):
    k, ctx = kctx
    model = wl.ring(4, 0.8, 2.0).with_field(0, 0.1)
    sec = basis.Sector(4, 1, 0)
    Hd = hamiltonian.Hamiltonian(model, sec).dense()
    n = 70000
    rng = np.random.default_rng(9)
    V = rng.standard_normal((n, sec.dim)) + 1j * rng.standard_normal((n, sec.dim))
    say("apply_h columns", n)
    got = to_host(ctx.apply_h(ctx.model(model), ctx.sector(4, 1, 0), to_dev(V)))
    assert rel_err(got, V @ Hd.T) < 1e-14


def test_invalid_inputs_are_reported(kctx):
    k, ctx = kctx
    import torch
    with pytest.raises(RuntimeError):
        ctx.sector(4, 5, 1)                       # more particles than sites
    with pytest.raises(RuntimeError):
        ctx.sector(30, 1, 1)                      # beyond the supported L
    m4, m5 = ctx.model(wl.ring(4, 1.0, 2.0)), ctx.model(wl.ring(5, 1.0, 2.0))
    s4 = ctx.sector(4, 2, 2)
    v = to_dev(wl.start_vector(s4.dim, 1))
    with pytest.raises(RuntimeError):             # model and sector disagree on L
        ctx.greens_neq(m5, m5, s4, v, orbitals=[(0, 0)], nt=2, steps_per_grid=1, dt=0.1)
    with pytest.raises(RuntimeError):             # orbital outside the cluster
        ctx.greens_neq(m4, m4, s4, v, orbitals=[(7, 0)], nt=2, steps_per_grid=1, dt=0.1)
    with pytest.raises(RuntimeError):             # Krylov dimension beyond the supported 128
        ctx.propagate(m4, s4, v.reshape(1, -1).clone(), 1, 0.1, 129, -1)
    with pytest.raises(RuntimeError):
        ctx.greens_neq_multi([m4, m5], [m4, m5], [s4, s4], [v, v], [(0, 0)], 2, 1, 0.1)
    with pytest.raises(ValueError):               # wrong vector length (binding check)
        ctx.apply_h(m4, s4, torch.zeros(s4.dim + 1, dtype=torch.complex128, device="cuda:0"))
    # the context stays usable after errors
    w = to_host(ctx.apply_h(m4, s4, v))
    ref = hamiltonian.Hamiltonian(wl.ring(4, 1.0, 2.0), basis.Sector(4, 2, 2)).apply(to_host(v))
    assert rel_err(w, ref) < 1e-13
