"""Four-time two-particle functions chi_abcd(t1,t2,t3,t4) =
<0| O1_a(t1) O2_b(t2) O3_c(t3) O4_d(t4) |0> (O = c or c+) through the C ABI
(kgf_greens2_neq) against the oracle's dense evaluation, on the Anderson
chain after the field quench: orderings whose bra and ket states are one
family (c+ c+ c c, c c c+ c+) and two (c+ c c c+, c c+ c+ c); all spin
classes."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import say
from oracle import basis, greens2

pytestmark = pytest.mark.gpu


def test_four_time_functions_against_oracle():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    ctx = k.Context(0)
    H = wl.chain_siam(4, 2.0, 1.0)
    Hi = H.with_field(0, 0.2)
    orbs = [(0, 0), (3, 0), (0, 1), (2, 1)]
    nt, dtg = 4, 0.3
    sec = basis.Sector(4, 2, 2)
    s = ctx.sector(4, 2, 2)
    v0 = torch.from_numpy(wl.start_vector(sec.dim, 7)).to("cuda:0")
    mi, mh = ctx.model(Hi), ctx.model(H)
    for pat in [(1, 1, 0, 0), (0, 0, 1, 1), (1, 0, 0, 1), (0, 1, 1, 0)]:
        say("four-time, pattern", pat)
        ref = greens2.four_time(Hi, H, 2, 2, orbs, [k_ * dtg for k_ in range(nt)], pattern=pat)
        out = ctx.greens2_neq(mi, mh, s, v0, orbs, nt=nt, steps_per_grid=6, dt=dtg / 6, pattern=pat,
                              krylov_dim=15, reorth=2, gs_tol=1e-13)
        assert abs(out["E0"] - ref["E0"]) < 1e-11
        err = np.abs(out["chi"] - ref["chi"]).max()
        say("max abs err", err)
        assert np.abs(ref["chi"]).max() > 0.05, pat
        assert err < 1e-10 * np.abs(ref["chi"]).max(), pat      # the parity bar for G (measured ~1e-14)
    with pytest.raises(k.KgfError):
        ctx.greens2_neq(mi, mh, s, v0, orbs, nt=2, steps_per_grid=1, dt=0.1, pattern=(1, 1, 1, 0))
