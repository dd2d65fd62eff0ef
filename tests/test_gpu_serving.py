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
