"""HIP path vs the CPU oracle, element by element, through the C ABI.

Bars: integer tables bit-exact; the ladder operator (a signed copy)
bit-exact; floating point within the parity tolerances (G: 1e-10
relative to max|G|; E0: 1e-12 relative), tighter where the arithmetic
allows (H.v: summation-order rounding only)."""
import math

import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say, to_dev, to_host
from oracle import basis, exact, greens, hamiltonian, lanczos, propagate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kgf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    return k


@pytest.fixture(scope="module")
def ctx(kgf):
    return kgf.Context(0)


# ----------------------------------------------------------------------------
# integer work: sector tables, ranks, hopping tables
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("L,nu,nd", [(1, 0, 1), (4, 2, 0), (8, 4, 4), (10, 5, 3), (12, 6, 6),
                                     (14, 7, 6), (16, 8, 16), (16, 0, 3), (13, 4, 9)])
def test_sector_tables_bit_exact(ctx, L, nu, nd):
    say("sector", L, nu, nd)
    sec = ctx.sector(L, nu, nd)
    assert (sec.d_up, sec.d_dn) == (math.comb(L, nu), math.comb(L, nd))
    np.testing.assert_array_equal(sec.states(0).astype(np.int64), basis.spin_states(L, nu))
    np.testing.assert_array_equal(sec.states(1).astype(np.int64), basis.spin_states(L, nd))


def test_sector_rank_bit_exact(ctx):
    import torch
    say("rank L=16")
    L, N = 16, 8
    sec = ctx.sector(L, N, N)
    rng = np.random.default_rng(3)
    masks = rng.integers(0, 1 << L, 5000, dtype=np.int64)
    masks[:1000] = basis.spin_states(L, N)[rng.integers(0, math.comb(L, N), 1000)]
    dev = torch.from_numpy(masks.astype(np.int32)).to("cuda:0")
    got = sec.rank(0, dev).cpu().numpy()
    table = basis.rank_table(basis.spin_states(L, N))
    ref = np.array([table.get(int(m), -1) for m in masks])
    np.testing.assert_array_equal(got, ref)


def _hop_models():
    return {"ring8": wl.ring8().H, "siam10": wl.siam10().H_ini, "hub4x3": wl.hub4x3().H,
            "ladder14": wl.ladder14().H, "chain3": wl.ring(3, 0.7, 1.0, periodic=False)}


@pytest.mark.parametrize("name", ["ring8", "siam10", "hub4x3", "ladder14", "chain3"])
def test_hop_table_bit_exact(ctx, name):
    model = _hop_models()[name]
    m = ctx.model(model)
    bonds, t, *_ = model.arrays()
    Ns = range(model.L + 1) if model.L <= 10 else [model.L // 2 - 1, model.L // 2]
    for n in Ns:
        say("hop table", name, n)
        cnt, ent, width = ctx.hop_table(m, n)
        states = basis.spin_states(model.L, n)
        T = hamiltonian.hopping_matrix(model.L, states, bonds, t, 0).tocsr()
        for r in range(len(states)):
            e = ent[:cnt[r], r]
            cols = (e & 0xFFFFFF).astype(np.int64)
            b = (e >> 24) & 127
            sgn = np.where(e >> 31, -1.0, 1.0)
            got = {}
            for c_, v_ in zip(cols, -t[b] * sgn):
                got[int(c_)] = got.get(int(c_), 0.0) + float(v_)
            row = T.getrow(r)
            ref = {int(c_): float(v_) for c_, v_ in zip(row.indices, row.data)}
            assert got == ref, (name, n, r)


# ----------------------------------------------------------------------------
# H.v and c / c+
# ----------------------------------------------------------------------------
HV_CASES = [
    ("ring8", lambda: wl.ring8().H, 4, 4, 1),
    ("siam10_field", lambda: wl.siam10().H_ini, 5, 5, 2),      # site-dependent U and eps
    ("hub4x3", lambda: wl.hub4x3().H, 6, 6, 1),
    ("chain3_ragged", lambda: wl.ring(3, 0.7, 2.0, periodic=False).with_field(0, 0.3), 1, 2, 3),
    ("empty_up", lambda: wl.ring(4, 1.0, 3.0), 0, 2, 1),
    ("full_up", lambda: wl.ring(5, 1.0, 3.0), 5, 2, 1),
    ("star_field", lambda: wl.star_siam([0.3, -0.5, 1.1, 0.2], [0.4, 0.2, -0.3, 0.35], 2.0, -1.0)
        .with_field(0, 0.25), 2, 3, 2),
]


@pytest.mark.parametrize("case", HV_CASES, ids=[c[0] for c in HV_CASES])
def test_apply_h_parity(ctx, case):
    name, mk, nu, nd, nvec = case
    model = mk()
    say("H.v", name)
    sec = basis.Sector(model.L, nu, nd)
    H = hamiltonian.Hamiltonian(model, sec)
    V = np.stack([wl.complex_vector(sec.dim, 10 + c) for c in range(nvec)])
    ref = np.stack([H.apply(V[c]) for c in range(nvec)])
    s = ctx.sector(model.L, nu, nd)
    got = to_host(ctx.apply_h(ctx.model(model), s, to_dev(V)))
    assert rel_err(got, ref) < 1e-13


@pytest.mark.parametrize("nu,nd", [(4, 4), (0, 3), (8, 1), (3, 8)])
def test_apply_c_bit_exact(ctx, nu, nd):
    L = 8
    sec = basis.Sector(L, nu, nd)
    s = ctx.sector(L, nu, nd)
    v = wl.complex_vector(sec.dim, 4)
    vd = to_dev(v)
    for site in (0, 3, 7):
        for spin in (0, 1):
            for dagger in (False, True):
                nu2 = nu + (0 if spin else (1 if dagger else -1))
                nd2 = nd + ((1 if dagger else -1) if spin else 0)
                if not (0 <= nu2 <= L and 0 <= nd2 <= L):
                    continue
                say("c", nu, nd, site, spin, dagger)
                ref, tgt = hamiltonian.apply_ladder(sec, site, spin, dagger, v)
                got = to_host(ctx.apply_c(s, ctx.sector(L, nu2, nd2), site, spin, dagger, vd))
                np.testing.assert_array_equal(got, ref)


# ----------------------------------------------------------------------------
# ground state, SIL
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["ring8", "siam10_field", "chain_siam8_field"])
def test_ground_state_parity(ctx, name):
    if name == "ring8":
        model, nu, nd = wl.ring8().H, 4, 4
    elif name == "siam10_field":
        model, nu, nd = wl.siam10().H_ini, 5, 5
    else:
        model, nu, nd = wl.chain_siam(8, 1.0).with_field(0, 0.2), 4, 4
    say("GS", name)
    sec = basis.Sector(model.L, nu, nd)
    H = hamiltonian.Hamiltonian(model, sec)
    v0 = wl.start_vector(sec.dim, 7)
    ora = lanczos.ground_state(H.apply, v0, tol=1e-12, max_iter=400)
    E0, psi, info = ctx.ground_state(ctx.model(model), ctx.sector(model.L, nu, nd), to_dev(v0), tol=1e-12,
                                     max_iter=400)
    assert info["converged"]
    assert abs(E0 - ora.E0) <= 1e-12 * abs(ora.E0)
    psi = to_host(psi)
    assert abs(np.linalg.norm(psi) - 1) < 1e-13
    assert abs(abs(np.vdot(ora.psi, psi)) - 1) < 1e-10


def test_ground_state_hub4x3_against_arpack(ctx):
    import scipy.sparse.linalg as spla
    q = wl.hub4x3()
    say("GS hub4x3")
    sec = basis.Sector(12, 6, 6)
    H = hamiltonian.Hamiltonian(q.H, sec)
    ev = spla.eigsh(H.sparse(), k=1, which="SA", tol=1e-14)[0][0]
    E0, psi, info = ctx.ground_state(ctx.model(q.H), ctx.sector(12, 6, 6), to_dev(wl.start_vector(sec.dim, 7)),
                                     tol=1e-12, max_iter=400)
    assert info["converged"] and abs(E0 - ev) <= 1e-12 * abs(ev)
    r = np.linalg.norm(H.apply(to_host(psi)) - E0 * to_host(psi))
    assert r < 1e-9


@pytest.mark.parametrize("direction", [-1, +1, 0])
@pytest.mark.parametrize("reorth", [0, 2])
def test_propagate_parity(ctx, direction, reorth):
    say("SIL", direction, reorth)
    model = wl.ring8().H
    sec = basis.Sector(8, 5, 4)
    H = hamiltonian.Hamiltonian(model, sec)
    X = np.stack([wl.complex_vector(sec.dim, 20 + c) for c in range(3)])
    shift, dt, m, n = -2.5, 0.05, 15, 12
    mode = {0: "none", 2: "cgs2"}[reorth]
    ref = np.stack([propagate.propagate(H.apply, X[c], dt, n, m, direction, shift, mode) for c in range(3)])
    got = ctx.propagate(ctx.model(model), ctx.sector(8, 5, 4), to_dev(X), n, dt, m, direction, shift, reorth)
    assert rel_err(to_host(got), ref) < 1e-12


def test_propagate_breakdown_exact(ctx):
    """Krylov dimension above the (ragged, tiny) sector dimension: the
    recursion breaks down and the step is exact."""
    say("SIL breakdown")
    model = wl.ring(3, 1.0, 2.0, periodic=False)
    sec = basis.Sector(3, 1, 2)
    Dn = exact.DenseSector(hamiltonian.Hamiltonian(model, sec).dense())
    psi = wl.complex_vector(sec.dim, 1)
    got = to_host(ctx.propagate(ctx.model(model), ctx.sector(3, 1, 2), to_dev(psi), 3, 1.3, 15, -1))
    assert np.linalg.norm(got - Dn.apply_exp(psi, 3.9)) < 1e-12


def test_propagate_zero_vector_stays_zero(ctx):
    say("SIL zero")
    model = wl.ring8().H
    z = np.zeros(basis.Sector(8, 4, 4).dim, complex)
    got = to_host(ctx.propagate(ctx.model(model), ctx.sector(8, 4, 4), to_dev(z), 2, 0.05, 15, -1))
    assert not np.any(got)


# ----------------------------------------------------------------------------
# Green's functions
# ----------------------------------------------------------------------------
def test_greens_eq_ring8_full(ctx):
    """Plain equilibrium case in full: L=8 ring, all 8 sites, 200 steps of
    dt=0.05, Krylov dim 15; GPU ground state and G vs the oracle's."""
    q = wl.ring8()
    say("G eq ring8")
    sec = basis.Sector(8, 4, 4)
    H = hamiltonian.Hamiltonian(q.H, sec)
    v0 = wl.start_vector(sec.dim, q.gs_seed)
    gs = lanczos.ground_state(H.apply, v0, tol=q.gs_tol)
    Gg, Gl = greens.equilibrium(q.H, 4, 4, q.orbitals, q.nt, q.dt_grid, 1, q.krylov_dim, gs.psi, gs.E0,
                                reorth="none")
    m = ctx.model(q.H)
    s = ctx.sector(8, 4, 4)
    E0, psi, _ = ctx.ground_state(m, s, to_dev(v0), tol=q.gs_tol)
    gg, gl = ctx.greens_eq(m, s, psi, E0, q.orbitals, q.nt, 1, q.dt_grid, q.krylov_dim, reorth=0, batch=0)
    assert abs(E0 - gs.E0) <= 1e-12 * abs(gs.E0)
    assert rel_err(gg, Gg) < 1e-10 and rel_err(gl, Gl) < 1e-10
    # one-by-one propagation gives the same numbers as the batched block
    gg1, gl1 = ctx.greens_eq(m, s, psi, E0, q.orbitals, q.nt, 1, q.dt_grid, q.krylov_dim, reorth=0, batch=1)
    assert rel_err(gg1, gg) < 1e-12 and rel_err(gl1, gl) < 1e-12
    # anticommutator at t = 0: G^>_ii(0) - G^<_ii(0) = -i
    np.testing.assert_allclose(np.diag(gg[0] - gl[0]), -1j, atol=1e-12)


@pytest.mark.parametrize("schedule", [0, 1])
def test_greens_neq_siam10_reduced_grid(ctx, schedule):
    """Anderson-impurity quench (impurity + 9 bath sites, field switched
    off), four-step G^<, G^>, Matsubara and both mixed components on a reduced
    mesh, both step-(iii) schedules, vs the oracle's literal four-step."""
    q = wl.siam10()
    say("G neq siam10 reduced", schedule)
    nt, spg, ntau, tspg = 7, 2, 5, 3
    dt, dtau = q.dt_grid / spg, q.dtau_grid / tspg
    sec = basis.Sector(10, 5, 5)
    v0 = wl.start_vector(sec.dim, q.gs_seed)
    ora = greens.four_step(q.H_ini, q.H, 5, 5, q.orbitals, nt, q.dt_grid, spg, q.krylov_dim, v0, gs_tol=q.gs_tol,
                           reorth="none", ntau=ntau, dtau_grid=q.dtau_grid, tau_steps_per_grid=tspg)
    got = ctx.greens_neq(ctx.model(q.H_ini), ctx.model(q.H), ctx.sector(10, 5, 5), to_dev(v0), q.orbitals, nt, spg,
                         dt, q.krylov_dim, reorth=0, schedule=schedule, ntau=ntau, tau_steps_per_grid=tspg,
                         dtau=dtau, gs_tol=q.gs_tol)
    assert abs(got["E0"] - ora["E0"]) <= 1e-12 * abs(ora["E0"])
    for key in ("G_lesser", "G_greater", "G_matsubara", "G_mixed", "G_mixed_left"):
        e = rel_err(got[key], ora[key])
        say(key, e)
        assert e < 1e-10, key


def test_greens_neq_schedules_agree_multi_orbital(ctx):
    """Sweep (batched) and plain (literal) schedules give the same G for
    several orbitals of both spins, with a capped block width that forces
    several sweeps."""
    H = wl.chain_siam(6, 2.0)
    H_ini = H.with_field(0, 0.4)
    orbs = [(0, 0), (2, 0), (1, 1)]
    sec = basis.Sector(6, 3, 3)
    v0 = to_dev(wl.start_vector(sec.dim, 7))
    kw = dict(nt=9, steps_per_grid=2, dt=0.1, krylov_dim=12, ntau=4, tau_steps_per_grid=2, dtau=0.1)
    a = ctx.greens_neq(ctx.model(H_ini), ctx.model(H), ctx.sector(6, 3, 3), v0, orbs, schedule=0, **kw)
    b = ctx.greens_neq(ctx.model(H_ini), ctx.model(H), ctx.sector(6, 3, 3), v0, orbs, schedule=1, batch=4, **kw)
    for key in ("G_lesser", "G_greater", "G_matsubara", "G_mixed", "G_mixed_left"):
        assert rel_err(b[key], a[key]) < 1e-12, key
    ora = greens.four_step(H_ini, H, 3, 3, orbs, 9, 0.2, 2, 12, wl.start_vector(sec.dim, 7), reorth="none",
                           ntau=4, dtau_grid=0.2, tau_steps_per_grid=2)
    for key in ("G_lesser", "G_greater", "G_matsubara", "G_mixed", "G_mixed_left"):
        assert rel_err(a[key], ora[key]) < 1e-10, key


@pytest.mark.parametrize("dt,m,direction", [(0.4, 40, -1), (3.0, 64, +1), (0.6, 30, 0)])
def test_propagate_large_norm_uses_eigendecomposition(ctx, dt, m, direction):
    """Steps with ||T dt|| well above 2 take the implicit-QL eigen-
    decomposition path (Eq. (udelta) literally); large Krylov spaces,
    including the single-space (f = 1 style) long step."""
    say("SIL large step", dt, m, direction)
    model = wl.ring8().H
    sec = basis.Sector(8, 5, 4)
    H = hamiltonian.Hamiltonian(model, sec)
    X = np.stack([wl.complex_vector(sec.dim, 40 + c) for c in range(2)])
    ref = np.stack([propagate.propagate(H.apply, X[c], dt, 3, m, direction, -1.0, "cgs2") for c in range(2)])
    got = ctx.propagate(ctx.model(model), ctx.sector(8, 5, 4), to_dev(X), 3, dt, m, direction, -1.0, 2)
    assert rel_err(to_host(got), ref) < 1e-10


def test_hub4x3_batched_equals_sequential_and_oracle_head():
    """4x3 cluster, t'=-0.3, U=8 (dim 853,776): the 24 components (12 c_i,
    12 c_i^+) propagated as one block for all 400 steps of dt=0.025 equal the
    24 one-by-one runs; the first steps of G_00 match the oracle (ground
    state of the oracle's sparse H by ARPACK)."""
    import scipy.sparse.linalg as spla
    import paper_1109_1205_amd as kgf
    ctx = kgf.Context(0)
    q = wl.hub4x3()
    say("hub4x3 G eq full")
    sec = basis.Sector(12, 6, 6)
    m = ctx.model(q.H)
    s = ctx.sector(12, 6, 6)
    E0, psi, info = ctx.ground_state(m, s, to_dev(wl.start_vector(sec.dim, q.gs_seed)), tol=1e-12, max_iter=400)
    assert info["converged"]
    gb, lb = ctx.greens_eq(m, s, psi, E0, q.orbitals, q.nt, 1, q.dt_grid, q.krylov_dim, batch=0)
    gs_, ls_ = ctx.greens_eq(m, s, psi, E0, q.orbitals, q.nt, 1, q.dt_grid, q.krylov_dim, batch=1)
    assert rel_err(gb, gs_) < 1e-12 and rel_err(lb, ls_) < 1e-12
    # anticommutator for every site at t = 0 and Hermiticity G_ij(0) = -conj(G_ji(0))
    np.testing.assert_allclose(np.diag(gb[0] - lb[0]), -1j, atol=1e-11)
    H = hamiltonian.Hamiltonian(q.H, sec)
    ev, vec = spla.eigsh(H.sparse(), k=1, which="SA", tol=1e-14)
    assert abs(ev[0] - E0) <= 1e-12 * abs(E0)
    nh = 6
    Gg, Gl = greens.equilibrium(q.H, 6, 6, [(0, 0)], nh, q.dt_grid, 1, q.krylov_dim, vec[:, 0].astype(complex),
                                float(ev[0]), reorth="none")
    assert rel_err(gb[:nh, :1, :1], Gg) < 1e-10 and rel_err(lb[:nh, :1, :1], Gl) < 1e-10


def test_siam10_full_grid_sampled_against_oracle():
    """Anderson quench on its full mesh (100 x 100 real times, 101 Matsubara
    times) on the GPU; the oracle computes the rows t_k for a sample of k
    (all t') plus the whole Matsubara branch and the mixed rows."""
    import paper_1109_1205_amd as kgf
    ctx = kgf.Context(0)
    q = wl.siam10()
    say("siam10 full grid")
    sec = basis.Sector(10, 5, 5)
    v0 = wl.start_vector(sec.dim, q.gs_seed)
    got = ctx.greens_neq(ctx.model(q.H_ini), ctx.model(q.H), ctx.sector(10, 5, 5), to_dev(v0), q.orbitals, q.nt,
                         q.steps_per_grid, q.dt, q.krylov_dim, schedule=1, ntau=q.ntau,
                         tau_steps_per_grid=q.tau_steps_per_grid, dtau=q.dtau_grid / q.tau_steps_per_grid,
                         gs_tol=q.gs_tol)
    Gl, Gg = got["G_lesser"][:, :, 0, 0], got["G_greater"][:, :, 0, 0]
    np.testing.assert_allclose(np.diag(Gg - Gl), -1j, atol=1e-11)
    np.testing.assert_allclose(Gl.conj(), -Gl.T, atol=1e-12)
    ks = [0, 41, 99]
    ora = greens.four_step(q.H_ini, q.H, 5, 5, q.orbitals, q.nt, q.dt_grid, q.steps_per_grid, q.krylov_dim, v0,
                           gs_tol=q.gs_tol, reorth="none", ntau=q.ntau, dtau_grid=q.dtau_grid,
                           tau_steps_per_grid=q.tau_steps_per_grid, times=ks)
    scale = np.abs(ora["G_lesser"]).max()
    for k in ks:
        for kp in ks:
            assert abs(got["G_lesser"][k, kp] - ora["G_lesser"][k, kp]).max() < 1e-10 * scale
            assert abs(got["G_greater"][k, kp] - ora["G_greater"][k, kp]).max() < 1e-10 * scale
        assert rel_err(got["G_mixed"][k], ora["G_mixed"][k]) < 1e-10
        assert rel_err(got["G_mixed_left"][:, k], ora["G_mixed_left"][:, k]) < 1e-10
    assert rel_err(got["G_matsubara"], ora["G_matsubara"]) < 1e-10
