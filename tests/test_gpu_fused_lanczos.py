"""The two-pass Lanczos step with the update folded into the row pass
(KGF_OPT_HV_FUSE, the default wherever the H.v is two-pass and reorth = 0):
step k's row pass forms x_k = y - a_{k-1} v_{k-1} from the rows it stages,
writes it back and sums ||x_k||^2 (b_k of Eq. (recursion)), so no update
pass runs.  Checked against the oracle's SIL step without
reorthogonalisation (Sec. 3, Eqs. (recursion), (newstate), (udelta)) on
sectors with ragged strips and rows, empty and full spin species, several
columns and steps, through every two-pass variant, and against the unfused
step (same arithmetic up to rounding order); the per-step error estimate
(which needs b_m, taken by an update pass after the last step) agrees with
the unfused one.  Inputs are seeded host vectors (workloads)."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say, to_dev, to_host
from oracle import basis, hamiltonian, propagate

pytestmark = pytest.mark.gpu

PASSES, STRIP, HV_FUSE, HV_UP_THREADS = 1, 2, 10, 12

CASES = [
    ("ring8", lambda: wl.ring8().H, 4, 4, 2),
    ("siam10_field", lambda: wl.siam10().H_ini, 5, 5, 3),
    ("hub4x3_c", lambda: wl.hub4x3().H, 5, 6, 1),
    ("chain3_ragged", lambda: wl.ring(3, 0.7, 2.0, periodic=False).with_field(0, 0.3), 1, 2, 3),
    ("empty_up", lambda: wl.ring(4, 1.0, 3.0), 0, 2, 2),
    ("full_up", lambda: wl.ring(5, 1.0, 3.0), 5, 2, 1),
]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    c = k.Context(0)
    yield c
    c.set_option(PASSES, 0)
    c.set_option(STRIP, 0)
    c.set_option(HV_FUSE, 1)
    c.set_option(HV_UP_THREADS, 1024)


def _run(ctx, model, nu, nd, X, passes, strip, fuse, nsteps, m, err=False, up_threads=256):
    ctx.set_option(PASSES, passes)
    ctx.set_option(STRIP, strip)
    ctx.set_option(HV_FUSE, fuse)
    ctx.set_option(HV_UP_THREADS, up_threads)
    try:
        out = ctx.propagate(ctx.model(model), ctx.sector(model.L, nu, nd), to_dev(X), nsteps, 0.07, m, -1, 0.0, 0,
                            return_err=err)
    finally:
        ctx.set_option(PASSES, 0)
        ctx.set_option(STRIP, 0)
        ctx.set_option(HV_FUSE, 1)
        ctx.set_option(HV_UP_THREADS, 1024)
    if err:
        return to_host(out[0]), out[1]
    return to_host(out)


# up_threads: pass-2 block size
@pytest.mark.parametrize("passes,strip,up_threads", [(2, 0, 256), (3, 0, 256), (4, 16, 256), (2, 8, 256),
                                                     (2, 0, 1024), (3, 16, 512), (2, 128, 1024), (3, 64, 256)])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fused_sil_matches_oracle(ctx, case, passes, strip, up_threads):
    name, mk, nu, nd, ncol = case
    model = mk()
    sec = basis.Sector(model.L, nu, nd)
    H = hamiltonian.Hamiltonian(model, sec)
    m = min(12, max(sec.dim, 1))
    X = np.stack([wl.complex_vector(sec.dim, 60 + c) for c in range(ncol)])
    say("fused SIL", name, passes, strip, up_threads)
    ref = np.stack([propagate.propagate(H.apply, X[c], 0.07, 2, m, -1, 0.0, "none") for c in range(ncol)])
    got = _run(ctx, model, nu, nd, X, passes, strip, 1, 2, m, up_threads=up_threads)
    assert rel_err(got, ref) < 1e-12
    unfused = _run(ctx, model, nu, nd, X, passes, strip, 0, 2, m, up_threads=up_threads)
    assert rel_err(got, unfused) < 1e-13


def test_fused_sil_error_estimate(ctx):
    model = wl.siam10().H_ini
    X = np.stack([wl.complex_vector(63504, 70 + c) for c in range(2)])
    say("fused SIL error estimate")
    got, e1 = _run(ctx, model, 5, 5, X, 2, 0, 1, 2, 10, err=True)
    ref, e0 = _run(ctx, model, 5, 5, X, 2, 0, 0, 2, 10, err=True)
    assert rel_err(got, ref) < 1e-13
    assert e0 > 0 and abs(e1 - e0) <= 1e-8 * e0


@pytest.fixture(scope="module")
def wide_up_case():
    """2x8 ladder with 7 up and 2 down electrons: D = 11,440 x 120 =
    1,372,800; a strip of 64 (32) columns of x is 11.7 (5.9) MB, more than
    one XCD's 4 MB L2, so the strip pass walks its rows grouped by the upper
    half's particle count; strips of 16 (2.9 MB) keep rank order."""
    model = wl.ladder(8, 1.0, 4.0).with_field(3, 0.2)
    sec = basis.Sector(16, 7, 2)
    H = hamiltonian.Hamiltonian(model, sec)
    X = np.stack([wl.complex_vector(sec.dim, 90 + c) for c in range(2)])
    say("grouped strip rows: oracle SIL steps")
    ref = np.stack([propagate.propagate(H.apply, X[c], 0.07, 2, 12, -1, 0.0, "none") for c in range(2)])
    return model, X, ref


@pytest.mark.parametrize("strip", [64, 32, 16])
def test_fused_sil_grouped_strip_rows(ctx, wide_up_case, strip):
    model, X, ref = wide_up_case
    say("grouped strip rows: fused SIL, strip", strip)
    got = _run(ctx, model, 7, 2, X, 2, strip, 1, 2, 12, up_threads=1024)
    assert rel_err(got, ref) < 1e-12
