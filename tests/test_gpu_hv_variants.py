"""The H.v kernel variants (single pass with the source row in LDS; two
passes: rows in LDS for the down-spin hops, L2-sized column strips for the
up-spin hops, with rows staged whole or as real and imaginary halves) vs the
oracle, and the Lanczos paths (ground state, SIL) run through each of them.

The 2x8 ladder (L = 16, the size where rows exceed LDS and the split
two-pass kernel is the default) is checked on sampled rows, which the
oracle computes one by one."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say, to_dev, to_host
from oracle import basis, hamiltonian, lanczos, propagate

pytestmark = pytest.mark.gpu

PASSES, STRIP = 1, 2


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    c = k.Context(0)
    yield c
    c.set_option(PASSES, 0)
    c.set_option(STRIP, 0)


CASES = [
    ("ring8", lambda: wl.ring8().H, 4, 4, 1),
    ("siam10_field", lambda: wl.siam10().H_ini, 5, 5, 2),
    ("hub4x3_c", lambda: wl.hub4x3().H, 5, 6, 1),
    ("chain3_ragged", lambda: wl.ring(3, 0.7, 2.0, periodic=False).with_field(0, 0.3), 1, 2, 3),
    ("empty_up", lambda: wl.ring(4, 1.0, 3.0), 0, 2, 1),
    ("full_up", lambda: wl.ring(5, 1.0, 3.0), 5, 2, 1),
]


@pytest.mark.parametrize("passes,strip", [(2, 0), (3, 0), (2, 8), (3, 16), (2, 32), (3, 64)])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_apply_h_variants(ctx, case, passes, strip):
    name, mk, nu, nd, nvec = case
    model = mk()
    say("H.v variant", name, passes, strip)
    sec = basis.Sector(model.L, nu, nd)
    H = hamiltonian.Hamiltonian(model, sec)
    V = np.stack([wl.complex_vector(sec.dim, 10 + c) for c in range(nvec)])
    ref = np.stack([H.apply(V[c]) for c in range(nvec)])
    ctx.set_option(PASSES, passes)
    ctx.set_option(STRIP, strip)
    try:
        got = to_host(ctx.apply_h(ctx.model(model), ctx.sector(model.L, nu, nd), to_dev(V)))
    finally:
        ctx.set_option(PASSES, 0)
        ctx.set_option(STRIP, 0)
    assert rel_err(got, ref) < 1e-13


@pytest.mark.parametrize("passes", [2, 3])
def test_ground_state_and_sil_through_two_pass(ctx, passes):
    say("Lanczos two-pass", passes)
    model = wl.siam10().H_ini
    sec = basis.Sector(10, 5, 5)
    H = hamiltonian.Hamiltonian(model, sec)
    v0 = wl.start_vector(sec.dim, 7)
    ora = lanczos.ground_state(H.apply, v0, tol=1e-12, max_iter=400)
    X = np.stack([wl.complex_vector(sec.dim, 30 + c) for c in range(2)])
    ref = np.stack([propagate.propagate(H.apply, X[c], 0.05, 3, 15, +1, 0.0, "cgs2") for c in range(2)])
    ctx.set_option(PASSES, passes)
    try:
        s = ctx.sector(10, 5, 5)
        E0, psi, info = ctx.ground_state(ctx.model(model), s, to_dev(v0), tol=1e-12, max_iter=400)
        got = to_host(ctx.propagate(ctx.model(model), s, to_dev(X), 3, 0.05, 15, +1, 0.0, 2))
    finally:
        ctx.set_option(PASSES, 0)
    assert info["converged"] and abs(E0 - ora.E0) <= 1e-12 * abs(ora.E0)
    assert abs(abs(np.vdot(ora.psi, to_host(psi))) - 1) < 1e-10
    assert rel_err(got, ref) < 1e-12


def test_option_rejects_bad_values(ctx):
    with pytest.raises(RuntimeError):
        ctx.set_option(PASSES, 7)
    with pytest.raises(RuntimeError):
        ctx.set_option(STRIP, 12)
    with pytest.raises(RuntimeError):
        ctx.set_option(99, 0)


def test_apply_h_ladder16_sampled_rows(ctx):
    """2x8 ladder, c-sector (7, 8): D = 11,440 x 12,870 = 147,232,800
    (2.36 GB per vector). Rows sampled across the matrix (first, last,
    ragged tail of the strip grid, random) against the oracle row by row."""
    import torch
    q = wl.ladder16()
    sec = basis.Sector(16, 7, 8)
    say("H.v ladder16 sampled rows: building oracle tables")
    H = hamiltonian.Hamiltonian(q.H, sec)
    rng = np.random.default_rng(16)
    rows = sorted({0, 1, 2, sec.d_up // 2, sec.d_up - 2, sec.d_up - 1, *rng.integers(0, sec.d_up, 6).tolist()})
    g = torch.Generator(device="cuda:0").manual_seed(5)
    x = torch.randn(sec.dim, dtype=torch.complex128, device="cuda:0", generator=g)
    say("H.v ladder16: GPU product")
    y = ctx.apply_h(ctx.model(q.H), ctx.sector(16, 7, 8), x)
    xh = x.cpu().numpy()
    yh = y.reshape(sec.d_up, sec.d_dn)[rows].cpu().numpy()
    del x, y
    torch.cuda.empty_cache()
    say("H.v ladder16: oracle rows", rows)
    ref = H.apply_rows(xh, rows)
    assert rel_err(yh, ref) < 1e-13
