"""Oracle parity at the benchmark's shape: the 2x7 ladder (L = 14) in the
c-sector (6, 7) that the backward sweep of the four-step procedure runs in,
D = 3003 x 3432 = 10,306,296.  Rows of 3432 elements are longer than the
1024-thread block of the single-pass H.v, so every thread there loops over
four row elements and carries the fused Lanczos dot across them; these are
the launch shapes the benchmark times.

* H.v (Sec. 3 Hubbard H) on three columns, through the single pass and the
  two-pass kernels, against the oracle on sampled rows (first, last and
  random rows), relative error <= 1e-13;
* one short-iterative-Lanczos step (Sec. 3, Eqs. (newstate), (udelta);
  Krylov dimension 20, dt = 0.05, backward direction as in step (iii)) on
  two columns in one batch -- the Lanczos-fused H.v, the three-term update,
  the tridiagonal exponential and the combination -- against the oracle's
  sil_step element by element, <= 1e-12; once through the single pass with
  the update pass, once through the two passes with the update folded into
  the row pass.
Inputs are seeded host vectors (workloads.complex_vector)."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say, to_dev, to_host
from oracle import basis, hamiltonian, propagate

pytestmark = pytest.mark.gpu

PASSES = 1


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    c = k.Context(0)
    yield c
    c.set_option(PASSES, 0)


@pytest.fixture(scope="module")
def oracle_h():
    q = wl.ladder14()
    sec = basis.Sector(14, 6, 7)
    say("ladder14: oracle tables")
    return q, sec, hamiltonian.Hamiltonian(q.H, sec)


@pytest.mark.parametrize("passes", [1, 2])
def test_apply_h_ladder14_sampled_rows(ctx, oracle_h, passes):
    q, sec, H = oracle_h
    assert sec.d_dn == 3432 and sec.d_up == 3003
    rng = np.random.default_rng(14)
    rows = sorted({0, 1, sec.d_up // 2, sec.d_up - 1, *rng.integers(0, sec.d_up, 8).tolist()})
    V = np.stack([wl.complex_vector(sec.dim, 140 + c) for c in range(3)])
    say("ladder14 H.v passes", passes)
    ctx.set_option(PASSES, passes)
    try:
        Y = ctx.apply_h(ctx.model(q.H), ctx.sector(14, 6, 7), to_dev(V))
        got = to_host(Y.reshape(3, sec.d_up, sec.d_dn)[:, rows])
    finally:
        ctx.set_option(PASSES, 0)
    for c in range(3):
        ref = H.apply_rows(V[c], rows)
        assert rel_err(got[c], ref) < 1e-13, c


@pytest.fixture(scope="module")
def sil_ref(oracle_h):
    q, sec, H = oracle_h
    X = np.stack([wl.complex_vector(sec.dim, 150 + c) for c in range(2)])
    refs = []
    for c in range(2):
        say("ladder14 SIL step: oracle column", c)
        refs.append(propagate.sil_step(H.apply, X[c], q.dt, q.krylov_dim, +1, reorth="none"))
    return X, np.stack(refs)


@pytest.mark.parametrize("passes", [1, 2])
def test_sil_step_ladder14(ctx, oracle_h, sil_ref, passes):
    """passes 1: the single pass plus the update pass; passes 2: the two
    passes with the update folded into the row pass (the fused step)."""
    q, sec, H = oracle_h
    X, ref = sil_ref
    say("ladder14 SIL step: GPU, passes", passes)
    ctx.set_option(PASSES, passes)
    try:
        got = to_host(ctx.propagate(ctx.model(q.H), ctx.sector(14, 6, 7), to_dev(X), 1, q.dt, q.krylov_dim, +1))
    finally:
        ctx.set_option(PASSES, 0)
    for c in range(2):
        assert rel_err(got[c], ref[c]) < 1e-12, c



def test_sil_step_ladder14_default_plan_by_width(ctx, oracle_h, sil_ref):
    """The library's own choice (no option set): one column (165 MB) keeps
    the single pass plus the update pass; two and three columns (330 and
    495 MB, beyond the 256 MB Infinity Cache) take the fused two-pass step.
    All against the oracle's SIL step, <= 1e-12."""
    q, sec, H = oracle_h
    X, ref = sil_ref
    m, s = ctx.model(q.H), ctx.sector(14, 6, 7)
    for cols, fused in ((1, False), (2, True), (3, True)):
        idx = [c % 2 for c in range(cols)]
        say("ladder14 SIL step: default plan,", cols, "columns")
        ctx.profile_begin(1)
        got = to_host(ctx.propagate(m, s, to_dev(X[idx]), 1, q.dt, q.krylov_dim, +1))
        st = ctx.profile_end()
        assert ("hv_up_lanczos" in st) == fused and ("hv_lanczos" in st) == (not fused), sorted(st)
        assert ("lanczos_update" in st) == (not fused), sorted(st)
        for c in range(cols):
            assert rel_err(got[c], ref[idx[c]]) < 1e-12, (cols, c)
