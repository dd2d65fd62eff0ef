"""Serving with continuous batching: with a pool too small for all requests,
requests queue, are admitted as memory frees up, overlap on the device, and
each result equals the same request run alone on its own context (FP64)."""
import numpy as np
import pytest

from paper_1406_2211_amd import inputs as I

pytestmark = pytest.mark.gpu


def _requests(n=10):
    g = np.random.default_rng(21)
    out = []
    for k in range(n):
        out.append(I.Request(rid=k, arrival=0.002 * k, side=int(g.integers(10, 22)),
                             nparticles=int(g.integers(0, 6)), tau=float(g.uniform(0.55, 1.0)),
                             fext=float(g.uniform(0, 1e-5)), steps=int(g.integers(20, 70)),
                             seed=100 + k))
    return out


def test_batched_server_matches_fifo_per_request():
    from paper_1406_2211_amd import lbc as L
    from paper_1406_2211_amd import serving as S
    reqs = _requests()
    big = max(L.ensemble_footprint(r.side, r.side, r.side, r.nparticles,
                                   **S.request_params(r, L.LB_F64)) for r in reqs)
    pool = 2 * big + 400_000  # about two boxes at a time: forces queueing
    print("[gpu] serving test with pool", pool, flush=True)
    seen = []
    every = {r.rid for r in reqs}
    bat, fb = S.serve_batched(reqs, pool, max_slots=8, storage=L.LB_F64, chunk=7, comoving=0,
                              autotune=False, log=seen.append, keep=every)
    fifo, ff = S.serve_fifo(reqs, storage=L.LB_F64, keep=every)
    assert len(bat) == len(fifo) == len(reqs)
    a = {r.rid: r.totals for r in bat}
    b = {r.rid: r.totals for r in fifo}
    for rid in a:
        scale = np.abs(b[rid]).max()
        assert np.abs(a[rid] - b[rid]).max() <= 1e-12 * max(scale, 1e-300), rid
        # the whole velocity field of each request, not only its sums
        us = np.abs(ff[rid]).max()
        assert np.abs(fb[rid] - ff[rid]).max() <= 1e-12 * max(us, 1e-300), rid
    # requests were admitted after earlier ones finished, i.e. the pool bounded concurrency
    s = S.summarize(bat)
    print("[serving]", s, flush=True)
    assert any(r.admitted > min(x.completed for x in bat) for r in bat)


def test_fp16_served_runs_within_the_stated_velocity_bound():
    """The serving form's precision claim on a sample of the serving request
    mix (the same generator, 12 requests, boxes of side 32-96 and the full
    step range): every batched FP16 run (comoving frame) against the same
    request run alone with FP32 storage, relative max-norm velocity error
    within the bound bench.py states and enforces (1e-4)."""
    import bench
    from paper_1406_2211_amd import inputs as I
    from paper_1406_2211_amd import lbc as L
    from paper_1406_2211_amd import serving as S
    reqs = [I.Request(r.rid, 0.0, r.side, r.nparticles, r.tau, r.fext, r.steps, r.seed)
            for r in I.serving_requests(12, 1.0, seed=5, side_range=(32, 96))]
    every = {r.rid for r in reqs}
    print("[gpu] serving precision sample of", len(reqs), "requests", flush=True)
    _, f16 = S.serve_batched(reqs, 8 << 30, max_slots=16, storage=L.LB_F16, keep=every)
    _, f32 = S.serve_fifo(reqs, storage=L.LB_F32, keep=every)
    worst = 0.0
    for rid in every:
        e = np.abs(f16[rid] - f32[rid]).max() / max(np.abs(f32[rid]).max(), 1e-300)
        worst = max(worst, e)
    print(f"[serving] FP16 vs FP32 velocity error, worst of {len(every)}: {worst:.2e}", flush=True)
    assert worst <= bench.SERVING_VEL_BOUND
