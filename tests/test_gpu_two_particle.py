"""The four-time two-particle function chi_abcd(t1,t2,t3,t4) =
<0| c+_a(t1) c+_b(t2) c_c(t3) c_d(t4) |0> through the C ABI
(kgf_greens2_neq) against the oracle's dense evaluation, on the Anderson
chain after the field quench (all four spin classes, two N-2 sectors)."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import say
from oracle import basis, greens2

pytestmark = pytest.mark.gpu


def test_four_time_function_against_oracle():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    ctx = k.Context(0)
    H = wl.chain_siam(4, 2.0, 1.0)
    Hi = H.with_field(0, 0.2)
    orbs = [(0, 0), (3, 0), (0, 1), (2, 1)]
    nt, dtg = 4, 0.3
    say("four-time oracle")
    ref = greens2.four_time(Hi, H, 2, 2, orbs, [k_ * dtg for k_ in range(nt)])
    sec = basis.Sector(4, 2, 2)
    s = ctx.sector(4, 2, 2)
    v0 = torch.from_numpy(wl.start_vector(sec.dim, 7)).to("cuda:0")
    say("four-time GPU")
    out = ctx.greens2_neq(ctx.model(Hi), ctx.model(H), s, v0, orbs, nt=nt, steps_per_grid=6, dt=dtg / 6,
                          krylov_dim=15, reorth=2, gs_tol=1e-13)
    assert abs(out["E0"] - ref["E0"]) < 1e-11
    err = np.abs(out["chi"] - ref["chi"]).max()
    say("max abs err", err)
    assert np.abs(ref["chi"]).max() > 0.05
    assert err < 1e-9
