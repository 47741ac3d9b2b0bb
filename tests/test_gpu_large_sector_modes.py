"""Modes for large sectors, each checked where the oracle can follow:

* the H.v kernel variants (single pass with the source row in LDS; two
  passes: rows in LDS for the down-spin hops, column strips for the up-spin
  hops, rows staged whole or as real and imaginary halves) vs the oracle,
  and the Lanczos paths (ground state, SIL) through each of them;
* the ground state with a capped (restarted) Lanczos basis;
* the four-step G with the forward mesh kept as checkpoints (bitwise equal
  to the stored mesh);
* the 2x8 ladder (L = 16, where rows exceed LDS): H.v on sampled rows against
  the oracle row by row, and a short four-step run checked against
  properties that hold at any size (equal-time anticommutator, Hermiticity,
  G^<(0,0) = i n_0 from the ground state itself)."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say, to_dev, to_host
from oracle import basis, hamiltonian, lanczos, propagate

pytestmark = pytest.mark.gpu

PASSES, STRIP, GS_MAX_BASIS, PHI_EVERY, HV_SEG = 1, 2, 3, 4, 11


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


# seg 1: the row pass with the segment hop tables (the default); 0: per-state tables
@pytest.mark.parametrize("passes,strip,seg", [(2, 0, 1), (3, 0, 1), (2, 8, 1), (3, 16, 1), (2, 32, 1), (3, 64, 1),
                                              (2, 128, 1), (4, 0, 1), (4, 16, 1), (2, 0, 0), (3, 0, 0), (4, 0, 0)])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_apply_h_variants(ctx, case, passes, strip, seg):
    name, mk, nu, nd, nvec = case
    model = mk()
    say("H.v variant", name, passes, strip, seg)
    sec = basis.Sector(model.L, nu, nd)
    H = hamiltonian.Hamiltonian(model, sec)
    V = np.stack([wl.complex_vector(sec.dim, 10 + c) for c in range(nvec)])
    ref = np.stack([H.apply(V[c]) for c in range(nvec)])
    ctx.set_option(PASSES, passes)
    ctx.set_option(STRIP, strip)
    ctx.set_option(HV_SEG, seg)
    try:
        got = to_host(ctx.apply_h(ctx.model(model), ctx.sector(model.L, nu, nd), to_dev(V)))
    finally:
        ctx.set_option(PASSES, 0)
        ctx.set_option(STRIP, 0)
        ctx.set_option(HV_SEG, 1)
    assert rel_err(got, ref) < 1e-13


@pytest.mark.parametrize("passes", [2, 3, 4])
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


@pytest.fixture(scope="module")
def ladder16_rows():
    q = wl.ladder16()
    sec = basis.Sector(16, 7, 8)
    say("H.v ladder16 sampled rows: building oracle tables")
    H = hamiltonian.Hamiltonian(q.H, sec)
    rng = np.random.default_rng(16)
    rows = sorted({0, 1, 2, sec.d_up // 2, sec.d_up - 2, sec.d_up - 1, *rng.integers(0, sec.d_up, 6).tolist()})
    return q, sec, H, rows, {}


# strip 0: the default (64 columns, one wavefront per row, rows grouped by
# the upper half's particle count: a 64-column strip is 11.7 MB); 32: the
# general strip kernel with grouped rows (5.9 MB strips); 16: rank order
# (2.9 MB strips fit one XCD's L2)
@pytest.mark.parametrize("strip", [0, 32, 16])
def test_apply_h_ladder16_sampled_rows(ctx, ladder16_rows, strip):
    """2x8 ladder, c-sector (7, 8): D = 11,440 x 12,870 = 147,232,800
    (2.36 GB per vector). Rows sampled across the matrix (first, last,
    ragged tail of the strip grid, random) against the oracle row by row."""
    import torch
    q, sec, H, rows, memo = ladder16_rows
    g = torch.Generator(device="cuda:0").manual_seed(5)
    x = torch.randn(sec.dim, dtype=torch.complex128, device="cuda:0", generator=g)
    say("H.v ladder16: GPU product, strip", strip)
    ctx.set_option(STRIP, strip)
    try:
        y = ctx.apply_h(ctx.model(q.H), ctx.sector(16, 7, 8), x)
    finally:
        ctx.set_option(STRIP, 0)
    xh = x.cpu().numpy()
    yh = y.reshape(sec.d_up, sec.d_dn)[rows].cpu().numpy()
    del x, y
    torch.cuda.empty_cache()
    if "ref" not in memo:   # the same seeded x for every strip width
        say("H.v ladder16: oracle rows", rows)
        memo["ref"] = H.apply_rows(xh, rows)
    assert rel_err(yh, memo["ref"]) < 1e-13


@pytest.mark.parametrize("cap", [12, 40])
def test_ground_state_restarted_basis(ctx, cap):
    """Ground state with the Lanczos basis capped at `cap` vectors (explicit
    restarts from the Ritz vector, the large-sector mode) vs the oracle."""
    say("GS restarted", cap)
    model = wl.siam10().H_ini
    sec = basis.Sector(10, 5, 5)
    H = hamiltonian.Hamiltonian(model, sec)
    v0 = wl.start_vector(sec.dim, 7)
    ora = lanczos.ground_state(H.apply, v0, tol=1e-12, max_iter=400)
    ctx.set_option(GS_MAX_BASIS, cap)
    try:
        E0, psi, info = ctx.ground_state(ctx.model(model), ctx.sector(10, 5, 5), to_dev(v0), tol=1e-12,
                                         max_iter=3000)
    finally:
        ctx.set_option(GS_MAX_BASIS, 0)
    say("iterations", info)
    assert info["converged"] and abs(E0 - ora.E0) <= 1e-12 * abs(ora.E0)
    psi = to_host(psi)
    assert abs(np.linalg.norm(psi) - 1) < 1e-13
    assert abs(abs(np.vdot(ora.psi, psi)) - 1) < 1e-10


@pytest.mark.parametrize("schedule", [0, 1])
def test_greens_neq_checkpointed_mesh_is_bitwise_equal(ctx, schedule):
    q = wl.siam10()
    say("four-step checkpoints", schedule)
    sec = basis.Sector(10, 5, 5)
    v0 = to_dev(wl.start_vector(sec.dim, 7))
    kw = dict(orbitals=[(0, 0), (0, 1)], nt=8, steps_per_grid=2, dt=0.05, krylov_dim=15, schedule=schedule,
              batch=3, gs_tol=1e-12)
    m_ini, m_fin, s = ctx.model(q.H_ini), ctx.model(q.H), ctx.sector(10, 5, 5)
    ref = ctx.greens_neq(m_ini, m_fin, s, v0, **kw)
    outs = []
    for K in (3, 8):
        ctx.set_option(PHI_EVERY, K)
        try:
            outs.append(ctx.greens_neq(m_ini, m_fin, s, v0, **kw))
        finally:
            ctx.set_option(PHI_EVERY, 0)
    for o in outs:
        assert o["E0"] == ref["E0"]
        assert np.array_equal(o["G_lesser"], ref["G_lesser"])
        assert np.array_equal(o["G_greater"], ref["G_greater"])


def test_four_step_ladder16_short_run(ctx):
    """Four-step G_00 on the 2x8 ladder quench (D = 165,636,900) on a 3-point
    mesh, forward mesh checkpointed every 2 points, ground-state basis capped
    at 40 vectors (restarted): equal-time anticommutator, Hermiticity and
    G^<(0,0) = i <0|n_0up|0> with the density summed on the host from the
    returned ground state and the sector's masks."""
    import torch
    q = wl.ladder16()
    s = ctx.sector(16, 8, 8)
    say("ladder16 four-step: start vector")
    v0 = torch.from_numpy(wl.start_vector(s.dim, 7)).to("cuda:0")
    psi0 = ctx.empty(s.dim)
    ctx.set_option(PHI_EVERY, 2)
    ctx.set_option(GS_MAX_BASIS, 40)
    ctx.set_progress(lambda ph, d, t: say("  ", ph, d, t))
    try:
        out = ctx.greens_neq(ctx.model(q.H_ini), ctx.model(q.H), s, v0, orbitals=[(0, 0)], nt=3, steps_per_grid=1,
                             dt=0.05, krylov_dim=20, schedule=1, gs_tol=1e-12, gs_max_iter=2000, psi0_out=psi0)
    finally:
        ctx.set_option(PHI_EVERY, 0)
        ctx.set_option(GS_MAX_BASIS, 0)
        ctx.set_progress(None)
    say("E0", out["E0"])
    Gl, Gg = out["G_lesser"][:, :, 0, 0], out["G_greater"][:, :, 0, 0]
    assert np.abs(np.diag(Gg - Gl) + 1j).max() < 1e-10
    assert np.abs(Gl + Gl.conj().T).max() < 1e-10
    assert np.abs(Gg + Gg.conj().T).max() < 1e-10
    up = s.states(0)
    occ = torch.from_numpy(((up & 1) == 1).astype(np.float64)).to("cuda:0")
    p = (psi0.reshape(s.d_up, s.d_dn).abs() ** 2).sum(dim=1)
    n0 = float((p * occ).sum())
    say("n0", n0, "G<(0,0)", Gl[0, 0])
    assert abs(Gl[0, 0] - 1j * n0) < 1e-10


def test_tuned_hv_choice_keeps_parity(ctx):
    """With the H.v tuner on, the variant it picks per sector (and form)
    still matches the oracle: H.v on three sectors, then ground state and
    SIL steps on the Anderson star (which re-uses the tuned choice)."""
    ctx.set_option(6, 1)
    try:
        for name, mk, nu, nd, nvec in CASES[:3]:
            model = mk()
            sec = basis.Sector(model.L, nu, nd)
            H = hamiltonian.Hamiltonian(model, sec)
            V = np.stack([wl.complex_vector(sec.dim, 10 + c) for c in range(nvec)])
            got = to_host(ctx.apply_h(ctx.model(model), ctx.sector(model.L, nu, nd), to_dev(V)))
            assert rel_err(got, np.stack([H.apply(V[c]) for c in range(nvec)])) < 1e-13, name
        model = wl.siam10().H_ini
        sec = basis.Sector(10, 5, 5)
        H = hamiltonian.Hamiltonian(model, sec)
        v0 = wl.start_vector(sec.dim, 7)
        ora = lanczos.ground_state(H.apply, v0, tol=1e-12, max_iter=400)
        s = ctx.sector(10, 5, 5)
        E0, psi, info = ctx.ground_state(ctx.model(model), s, to_dev(v0), tol=1e-12, max_iter=400)
        assert info["converged"] and abs(E0 - ora.E0) <= 1e-12 * abs(ora.E0)
        X = wl.complex_vector(sec.dim, 30)
        ref = propagate.propagate(H.apply, X, 0.05, 3, 15, -1, 0.0, "none")
        got = to_host(ctx.propagate(ctx.model(model), s, to_dev(X[None, :]), 3, 0.05, 15, -1))
        assert rel_err(got[0], ref) < 1e-12
    finally:
        ctx.set_option(6, 0)
