"""kgf_propagate_noalloc (for callers that cannot allocate device memory)
against kgf_propagate: two calls in a row, the second on a smaller input,
must give bitwise the same states (same kernels, same reduction order); the
size limit and the missing-table case are reported as errors."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    return k.Context(0)


def _pair(ctx, model, L, nu, nd, ncol, seed, nsteps, dt, m, direction, reorth):
    s = ctx.sector(L, nu, nd)
    mo = ctx.model(model)
    X = np.stack([wl.complex_vector(s.dim, seed + c) for c in range(ncol)])
    ref = to_dev(X)
    ctx.propagate(mo, s, ref, nsteps, dt, m, direction, 0.0, reorth)      # also builds the hopping tables
    got = to_dev(X)
    ctx.propagate_noalloc(mo, s, got, nsteps, dt, m, direction, 0.0, reorth)
    return to_host(got), to_host(ref)


def test_noalloc_matches_propagate_twice(ctx):
    say("no-alloc: 10-site star, 3 columns")
    got, ref = _pair(ctx, wl.siam10().H_ini, 10, 5, 5, 3, 70, 4, 0.05, 15, -1, 0)
    assert np.array_equal(got, ref)
    say("no-alloc: 8-site ring, 2 columns, reorthogonalised (smaller input)")
    got, ref = _pair(ctx, wl.ring8().H, 8, 4, 4, 2, 80, 3, 0.05, 12, +1, 2)
    assert np.array_equal(got, ref)


def test_noalloc_limits(ctx):
    import paper_1109_1205_amd as k
    s = ctx.sector(10, 5, 5)
    mo = ctx.model(wl.siam10().H)
    x = to_dev(np.stack([wl.complex_vector(s.dim, 90 + c) for c in range(8)]))
    ctx.apply_h(mo, s, x[0])                                      # tables built: only the size is wrong
    with pytest.raises(k.KgfError) as e:
        ctx.propagate_noalloc(mo, s, x, 1, 0.05, 20)              # 20 x 8 x 63,504 complex128 > 64 MiB
    assert e.value.code == -5 and "MiB" in str(e.value)
    fresh = ctx.model(wl.ring(6, 1.0, 2.0))
    s6 = ctx.sector(6, 3, 3)
    y = to_dev(wl.complex_vector(s6.dim, 91))
    with pytest.raises(k.KgfError) as e:
        ctx.propagate_noalloc(fresh, s6, y, 1, 0.05, 10)          # no table built for this model yet
    assert e.value.code == -1
