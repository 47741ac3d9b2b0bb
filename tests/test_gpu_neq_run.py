"""Step-wise four-step run (kgf_neq_run_*): steps (i), (ii) at creation, then
steps (iii), (iv) of Sec. 4 one mesh interval per call.  The run must give
bitwise the G of kgf_greens_neq (sweep schedule, same block width) and match
the oracle's literal four-step to the G tolerance; the interval and
vector-step counts must follow from the chunking of the sweep."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say, to_dev
from oracle import greens

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1205_amd as k
    return k.Context(0)


def expected_counts(nt, spg, groups, jchunk_of):
    """(intervals, vector steps) of the sweeps: per spin group of na
    orbitals, a c and a c+ sweep, chunks of jchunk source times from t_max."""
    intervals = steps = 0
    for na in groups:
        jchunk = jchunk_of(na)
        for _ in range(2):
            jhi = nt - 1
            while jhi >= 0:
                jlo = max(0, jhi - jchunk + 1)
                ncur = 0
                for s in range(jhi, -1, -1):
                    if s >= jlo:
                        ncur += na
                    intervals += 1
                    if s > 0:
                        steps += ncur * spg
                jhi -= jchunk
    return intervals, steps


@pytest.mark.parametrize("batch", [0, 4, 3])
def test_run_equals_greens_neq_and_oracle(ctx, batch):
    """Anderson chain L = 6 after a field quench, orbitals of both spins
    (spin groups of 2 and 1 orbitals), nt = 7 with two SIL steps per
    interval; batch 4 and 3 cut the sweep into several chunks (ragged last
    chunk), batch 0 takes one chunk from free memory."""
    H = wl.chain_siam(6, 2.0)
    Hi = H.with_field(0, 0.4)
    orbs = [(0, 0), (2, 0), (1, 1)]
    nt, spg, dt, m = 7, 2, 0.1, 15
    say("neq run", "batch", batch)
    s = ctx.sector(6, 3, 3)
    v0 = wl.start_vector(s.dim, 7)
    mi, mf = ctx.model(Hi), ctx.model(H)
    whole = ctx.greens_neq(mi, mf, s, to_dev(v0), orbs, nt=nt, steps_per_grid=spg, dt=dt, krylov_dim=m,
                           schedule=1, batch=batch)
    run = ctx.neq_run(mi, mf, s, to_dev(v0), orbs, nt=nt, steps_per_grid=spg, dt=dt, krylov_dim=m, batch=batch)
    assert run.E0 == whole["E0"]
    with pytest.raises(RuntimeError):
        run.result()                      # intervals left
    infos = []
    while True:
        info = run.advance(1)
        if info["intervals"] == 0:
            break
        infos.append(info)
        if info["done"]:
            break
    assert infos[-1]["done"] == 1 and infos[-1]["next_width"] == 0 and infos[-1]["next_mesh_index"] == -1
    assert run.advance(5)["intervals"] == 0          # nothing left
    got = run.result()
    run.close()
    for key in ("G_lesser", "G_greater"):
        assert np.array_equal(got[key], whole[key]), key
    if batch > 0:
        jchunk_of = lambda na: min(max(1, batch // na), nt)
        n_int, n_steps = expected_counts(nt, spg, [2, 1], jchunk_of)
        assert len(infos) == n_int
        assert infos[-1]["total_vector_steps"] == n_steps == sum(i["vector_steps"] for i in infos)
        assert max(i["width"] for i in infos) <= max(jchunk_of(2) * 2, jchunk_of(1))
    ref = greens.four_step(Hi, H, 3, 3, orbs, nt, dt * spg, spg, m, v0, reorth="none")
    for key in ("G_lesser", "G_greater"):
        assert rel_err(got[key], ref[key]) < 1e-10, key
    assert abs(got["E0"] - ref["E0"]) <= 1e-12 * abs(ref["E0"])


def test_run_interleaves_with_other_calls(ctx):
    """The run keeps its own workspaces: a kgf_greens_neq on the same
    context between two intervals leaves the run's result unchanged."""
    H = wl.ring(6, 1.0, 3.0)
    Hi = H.with_field(1, 0.3)
    orbs = [(0, 0), (0, 1)]
    s = ctx.sector(6, 3, 3)
    v0 = to_dev(wl.start_vector(s.dim, 7))
    mi, mf = ctx.model(Hi), ctx.model(H)
    kw = dict(nt=5, steps_per_grid=1, dt=0.1, krylov_dim=12)
    ref = ctx.greens_neq(mi, mf, s, v0, orbs, schedule=1, **kw)
    run = ctx.neq_run(mi, mf, s, v0, orbs, **kw)
    run.advance(3)
    other = ctx.greens_neq(mf, mi, s, v0, orbs, schedule=1, **kw)      # different quench, same context
    while not run.advance(2)["done"]:
        pass
    got = run.result()
    run.close()
    assert not np.array_equal(other["G_lesser"], ref["G_lesser"])
    for key in ("G_lesser", "G_greater"):
        assert np.array_equal(got[key], ref[key]), key


def test_run_rejects_bad_input(ctx):
    H = wl.ring(4, 1.0, 2.0)
    s = ctx.sector(4, 2, 2)
    v0 = to_dev(wl.start_vector(s.dim, 7))
    m = ctx.model(H)
    with pytest.raises(RuntimeError):
        ctx.neq_run(m, m, s, v0, [(9, 0)], nt=3, steps_per_grid=1, dt=0.1)       # orbital outside the cluster
    with pytest.raises(RuntimeError):
        ctx.neq_run(m, m, s, v0, [(0, 0)], nt=0, steps_per_grid=1, dt=0.1)       # empty mesh
    run = ctx.neq_run(m, m, s, v0, [(0, 0)], nt=3, steps_per_grid=1, dt=0.1)
    with pytest.raises(RuntimeError):
        run.advance(-1)
    run.close()


def test_tuned_sweep_matches_oracle(ctx):
    """KGF_OPT_HV_TUNE picks the H.v variant and the sweep block width by
    timing; the tuned four-step still matches the oracle."""
    H = wl.chain_siam(6, 2.0)
    Hi = H.with_field(0, 0.4)
    orbs = [(0, 0), (2, 0), (1, 1)]
    s = ctx.sector(6, 3, 3)
    v0 = wl.start_vector(s.dim, 7)
    ctx.set_option(ctx.HV_TUNE, 1)
    try:
        got = ctx.greens_neq(ctx.model(Hi), ctx.model(H), s, to_dev(v0), orbs, nt=7, steps_per_grid=2, dt=0.1,
                             krylov_dim=15, schedule=1)
    finally:
        ctx.set_option(ctx.HV_TUNE, 0)
    ref = greens.four_step(Hi, H, 3, 3, orbs, 7, 0.2, 2, 15, v0, reorth="none")
    for key in ("G_lesser", "G_greater"):
        assert rel_err(got[key], ref[key]) < 1e-10, key


@pytest.mark.parametrize("batch,stop_after", [(4, 3), (3, 9), (4, 1000), (0, 4)])
def test_checkpoint_resume_equals_uninterrupted(ctx, batch, stop_after):
    """Host-spill checkpoint of a run between chunks (after at least
    `stop_after` intervals, or at the end), resumed in a run created afresh
    from the same inputs: G^< and G^> bitwise those of the uninterrupted run
    (which equals kgf_greens_neq and the oracle above); the image is refused
    inside a chunk, by a run that has advanced and by a run of other sizes."""
    import paper_1109_1205_amd as k
    H = wl.chain_siam(6, 2.0)
    Hi = H.with_field(0, 0.4)
    orbs = [(0, 0), (2, 0), (1, 1)]
    nt, spg, dt, m = 7, 2, 0.1, 15
    s = ctx.sector(6, 3, 3)
    v0 = to_dev(wl.start_vector(s.dim, 7))
    mi, mf = ctx.model(Hi), ctx.model(H)

    def new_run(n=nt):
        return ctx.neq_run(mi, mf, s, v0, orbs, nt=n, steps_per_grid=spg, dt=dt, krylov_dim=m, batch=batch)

    say("checkpoint/resume: uninterrupted run, batch", batch)
    ref = new_run()
    while not ref.advance(1)["done"]:
        pass
    want = ref.result()
    ref.close()

    say("checkpoint/resume: saved run")
    run = new_run()
    moved, info = 0, {"chunk_start": 1, "done": 0}
    refused_inside = False
    while not info["done"]:
        if not info["chunk_start"] and not refused_inside:
            with pytest.raises(k.KgfError):
                run.checkpoint()
            refused_inside = True
        if moved >= stop_after and info["chunk_start"]:
            break
        info = run.advance(1)
        moved += 1
    image = run.checkpoint()
    run.close()

    say("checkpoint/resume: resumed run after", moved, "intervals,", len(image), "bytes")
    other = new_run(nt - 1)
    with pytest.raises(k.KgfError):
        other.restore(image)
    other.close()
    res = new_run()
    res.restore(image)
    with pytest.raises(k.KgfError):
        res.restore(image)
    while not res.advance(1)["done"]:
        pass
    got = res.result()
    res.close()
    assert np.array_equal(got["G_lesser"], want["G_lesser"])
    assert np.array_equal(got["G_greater"], want["G_greater"])
