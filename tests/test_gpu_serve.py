"""The continuous-batching service: every served result equals the same chain
solved alone (same schedule, same device stopping tests, the launch variants
the batch gives its block size),
admission never exceeds the memory budget, and requests overlap on the GPU."""
import numpy as np
import pytest

import synth
from oracle import level_reduction

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _requests(count, seed, rate, L_range=(32, 400), m_choices=(8, 16, 32, 64)):
    from paper_2302_07551_amd.serve import Request
    specs = synth.served_stream(count, seed, L_range=L_range, m_choices=m_choices, rate=rate)
    reqs, gens = [], []
    for k, sp in enumerate(specs):
        g = synth.qbd(sp["L"], sp["m"], sp["seed"])
        gens.append(g)
        reqs.append(Request(k, sp["arrival"], g.blocks, g.sizes, g.b))
    return reqs, gens


def test_served_equals_alone_and_budget_holds():
    from paper_2302_07551_amd import Solver, stc
    from paper_2302_07551_amd.serve import Server
    reqs, gens = _requests(12, 2024, rate=40.0)
    tol, sw = 1e-13, 1e-6
    srv = Server(budget_bytes=1, max_chains=8, sweeps_per_round=15, tol=tol, switch_tol=sw)
    fps = [srv.footprint(r) for r in reqs]
    srv.budget = int(sum(sorted(fps)[-4:]))      # binds: at most a few chains at once
    # launch shapes tuned on probe chains first; served chains take them
    srv.autotune(reqs[:6], trial_sweeps=2)
    tiles = {(st, mp): srv.batch.tile(st, mp)["variant"]
             for st in (stc.STC_FP64, stc.STC_FP32) for mp in (8, 16, 32, 64)}
    print(tiles, flush=True)
    stats = srv.run(reqs)
    srv.close()
    summ = stats.summary()
    print(summ, flush=True)
    assert summ["completed"] == len(reqs) and not stats.rejected
    assert stats.peak_bytes <= srv.budget
    assert stats.peak_chains >= 2                 # requests overlapped on the GPU
    by_id = {r.rid: r for r in stats.results}
    for k, g in enumerate(gens):
        s = Solver(g.blocks, g.sizes, g.b, precision="mixed", switch_tol=sw, check_every=10)
        mp = 8
        while mp < g.m:
            mp *= 2
        stc.stc_set_variant(s.h, stc.STC_FP64, tiles[(stc.STC_FP64, mp)])
        stc.stc_set_variant(s.h, stc.STC_FP32, tiles[(stc.STC_FP32, mp)])
        pi, info = s.solve(tol=tol, maxit=100000, allow_maxit=False)
        s.close()
        r = by_id[k]
        assert r.sweeps == info["iters"] and r.sweeps_fp32 == info["iters_fp32"], k
        assert np.array_equal(r.pi, pi), k
        ref = level_reduction.level_reduction(g.blocks, g.sizes, g.b)
        assert np.abs(r.pi - ref).sum() <= 1e-10, k


def test_fp32_floor_promotes_in_the_served_stream():
    """With a switch tolerance no FP32 sweep reaches, every request is
    promoted at its FP32 rounding floor and completes in FP64, within 1e-10
    of its direct solution."""
    from paper_2302_07551_amd import stc
    from paper_2302_07551_amd.serve import Server
    reqs, gens = _requests(6, 77, rate=1000.0, L_range=(40, 120), m_choices=(8, 16, 32))
    srv = Server(budget_bytes=1 << 30, max_chains=8, sweeps_per_round=25, tol=1e-13,
                 switch_tol=1e-15, max_sweeps=200_000)
    stats = srv.run(reqs)
    srv.close()
    assert sorted(r.rid for r in stats.results) == list(range(6)) and not stats.rejected
    for r in stats.results:
        assert r.status == stc.STC_OK and 0 < r.sweeps_fp32 < r.sweeps, r.rid
        g = gens[r.rid]
        ref = level_reduction.level_reduction(g.blocks, g.sizes, g.b)
        assert np.abs(r.pi - ref).sum() <= 1e-10, r.rid


def test_oversized_request_is_rejected():
    from paper_2302_07551_amd.serve import Server
    reqs, _ = _requests(3, 7, rate=1000.0, L_range=(40, 60), m_choices=(16,))
    srv = Server(budget_bytes=1, max_chains=4, sweeps_per_round=10)
    fps = [srv.footprint(r) for r in reqs]
    srv.budget = min(fps) - 1                      # nothing fits
    stats = srv.run(reqs)
    srv.close()
    assert sorted(stats.rejected) == [0, 1, 2] and not stats.results


def test_failed_setup_and_sweep_cap_retire_only_their_request():
    """A request that is not a generator is rejected with its setup error,
    and the others are still served.  Under a sweep cap every unfinished
    request is retired with STC_EMAXIT and its last iterate, which equals the
    same chain solved alone with maxit at that sweep."""
    from paper_2302_07551_amd import Solver, stc
    from paper_2302_07551_amd.serve import Server
    reqs, gens = _requests(5, 99, rate=1000.0, L_range=(40, 80), m_choices=(16,))
    bad = reqs[1].blocks.copy()
    bad[3, 2, 0, 1] = -1.0            # a negative rate: not a generator
    reqs[1].blocks = bad
    cap = 60
    srv = Server(budget_bytes=1 << 30, max_chains=4, sweeps_per_round=10, max_sweeps=cap)
    stats = srv.run(reqs)
    srv.close()
    print(stats.summary(), stats.errors, flush=True)
    assert stats.rejected == [1] and f"(status {stc.STC_ENOTGEN})" in stats.errors[1]
    assert sorted(r.rid for r in stats.results) == [0, 2, 3, 4]
    for r in stats.results:
        assert r.status == stc.STC_EMAXIT and cap <= r.sweeps < cap + 10
        g = gens[r.rid]
        s = Solver(g.blocks, g.sizes, g.b, precision="mixed", switch_tol=1e-6, check_every=10)
        stc.stc_set_variant(s.h, stc.STC_FP64, 0)
        stc.stc_set_variant(s.h, stc.STC_FP32, 0)
        pi, info = s.solve(tol=1e-13, maxit=r.sweeps)
        s.close()
        assert info["status"] == stc.STC_EMAXIT and info["iters"] == r.sweeps
        assert r.sweeps_fp32 == info["iters_fp32"] and np.array_equal(r.pi, pi), r.rid


@pytest.mark.skip(reason="the threaded setup (setup_thread=True) ended twice in a host "
                         "segmentation fault inside stc_batch_sweeps on the serving thread while "
                         "stc_setup ran on the setup thread (512-request stream, Poisson "
                         "arrivals); it stays off until that cause is found")
def test_threaded_setup_serves_like_inline_setup():
    import synth
    from paper_2302_07551_amd.serve import Request, Server
    reqs = synth.served_stream(24, 42, rate=200.0)
    gens = [synth.qbd(r["L"], r["m"], r["seed"]) for r in reqs]
    out = {}
    for threaded in (False, True):
        srv = Server(budget_bytes=1 << 30, max_chains=8, sweeps_per_round=10,
                     setup_thread=threaded)
        st = srv.run([Request(k, r["arrival"], g.blocks, g.sizes, g.b)
                      for k, (r, g) in enumerate(zip(reqs, gens))])
        srv.close()
        out[threaded] = {r.rid: r.pi for r in st.results}
    assert out[False].keys() == out[True].keys()
    for k in out[False]:
        assert np.array_equal(out[False][k], out[True][k])


@pytest.mark.skip(reason="three runs of the 512-request stream with Poisson arrivals and graph "
                         "replay ended in a host segmentation fault inside stc_batch_sweeps "
                         "(the third with no other thread in the runtime); serving replays no "
                         "graph until that cause is found")
def test_served_poisson_stream_with_graph_replay():
    from paper_2302_07551_amd.serve import Server
    reqs, gens = _requests(64, 2031, rate=50.0, L_range=(32, 2048))
    srv = Server(budget_bytes=1 << 31, max_chains=64, sweeps_per_round=25, use_graph=True)
    st = srv.run(reqs)
    srv.close()
    assert st.summary()["completed"] == len(reqs)
