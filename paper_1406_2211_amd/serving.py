"""Serving of ensemble suspension runs with continuous batching.

Requests (a periodic box of its own size, particle count, tau, body force and
step count) arrive over time.  The batched server admits a request as soon as
an ensemble slot and enough pool memory (its footprint) are free, keeps the
state of every admitted run resident, advances all of them together in short
chunks of steps, and retires each run when its budget is spent, so requests
that arrive while others are running join the batch.  The per-run server
processes requests one at a time in arrival order (FIFO) with a context of its
own.  Both report time-to-result (completion minus arrival) and throughput.

The result of a run is its final mean velocity and total momentum, reduced on
the device in FP64 (lb_totals); the full fields stay available through the
slot handle until the run is retired.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import inputs as I
from . import lbc as L


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    completed: float
    steps: int
    sites: int
    totals: np.ndarray
    extra: dict = field(default_factory=dict)

    @property
    def latency(self):
        return self.completed - self.arrival


def request_params(req: I.Request, storage: int, kernel: int = L.LB_PHI2, comoving: int = 0):
    return dict(tau=req.tau, body_force=(req.fext, 0.0, 0.0), collision=L.LB_BGK,
                coupling=L.LB_COUPLE_FC if req.nparticles else L.LB_COUPLE_NONE, gamma=1.0,
                kernel=kernel, storage=storage, comoving=comoving,
                f16_scale_log2=f16_scale_for(req) if storage in (L.LB_F16, L.LB_BF16) else 0)


def f16_scale_for(req: I.Request):
    """Power-of-two scale that maps the largest expected stored value to about
    2^12 in FP16: in the comoving frame the stored values are fluctuations of
    the order of the particle-driven velocities (about 1e-3 at most here)."""
    umax = 2e-3
    return int(math.floor(math.log2(4096.0 / (umax / 6.0))))


def request_particles(req: I.Request):
    n = req.nparticles
    if n == 0:
        return None
    g = I.rng(req.seed)
    pos = g.uniform(0.0, 1.0, (n, 3)) * req.side
    vel = g.normal(0.0, 1e-3, (n, 3))
    return pos, vel, np.ones(n)


def _init_box(lat, req):
    import torch
    lat.lb_init_fluid()
    parts = request_particles(req)
    if parts is not None:
        pos, vel, mass = parts
        lat.lb_set_particles(torch.from_numpy(pos), torch.from_numpy(vel), torch.from_numpy(mass))


def serve_batched(requests, pool_bytes, max_slots=64, storage=L.LB_F16, chunk=20, comoving=1,
                  autotune=True, keep=None, log=None, prof=None):
    """Continuous batching over one ensemble.  Arrival times are honoured
    against the wall clock (requests arriving at time 0 model a saturated
    queue).  keep: optional set of request ids whose final velocity fields are
    returned (as host arrays) for accuracy checks.  prof: optional dict that
    receives the host wall time spent admitting and initialising requests,
    enqueueing steps, and polling/retiring (which waits for the device)."""
    import torch
    clock = time.perf_counter
    acc = {"admit_s": 0.0, "enqueue_s": 0.0, "poll_s": 0.0, "chunks": 0}
    ens = L.Ensemble(pool_bytes, max_slots, storage=storage, kernel=L.LB_PHI2)
    pending = sorted(requests, key=lambda r: r.arrival)
    queue, active, results, fields = [], {}, [], {}
    t0 = time.perf_counter()
    tuned = not autotune
    while pending or queue or active:
        now = time.perf_counter() - t0
        while pending and pending[0].arrival <= now:
            queue.append(pending.pop(0))
        ta = clock()
        while queue:  # continuous admission: FIFO order, as far as memory and slots allow
            req = queue[0]
            got = ens.admit(req.side, req.side, req.side, req.steps, max_particles=req.nparticles,
                            **request_params(req, storage, comoving=comoving))
            if got is None:
                break
            queue.pop(0)
            slot, lat = got
            _init_box(lat, req)
            active[slot] = (req, lat, time.perf_counter() - t0)
        acc["admit_s"] += clock() - ta
        if not active:
            if pending:
                time.sleep(max(0.0, min(0.002, pending[0].arrival - now)))
            continue
        if not tuned and len(active) >= 4:
            ens.autotune(1)
            tuned = True
        te = clock()
        ens.step(chunk)
        acc["chunks"] += 1
        tp = clock()
        acc["enqueue_s"] += tp - te
        for slot in list(active):
            done_steps, done = ens.query(slot)
            if not done:
                continue
            req, lat, t_adm = active.pop(slot)
            tot = lat.lb_totals()
            if keep is not None and req.rid in keep:
                _, u = lat.lb_moments()
                fields[req.rid] = u.cpu().numpy()
            t_done = time.perf_counter() - t0
            results.append(Result(req.rid, req.arrival, t_adm, t_done, req.steps,
                                  req.side ** 3, tot))
            ens.retire(slot)
            if log:
                log(f"done {req.rid} L={req.side} steps={req.steps} latency={t_done - req.arrival:.3f}s")
        acc["poll_s"] += clock() - tp
    ens.destroy()
    if prof is not None:
        prof.update({k: round(v, 4) if isinstance(v, float) else v for k, v in acc.items()})
    torch.cuda.synchronize()
    return results, fields


def serve_fifo(requests, storage=L.LB_F32, keep=None, log=None):
    """One run at a time in arrival order, each on a context of its own."""
    import torch
    pending = sorted(requests, key=lambda r: r.arrival)
    results, fields = [], {}
    t0 = time.perf_counter()
    for req in pending:
        now = time.perf_counter() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        t_adm = time.perf_counter() - t0
        lat = L.Lattice(req.side, req.side, req.side, max_particles=req.nparticles,
                        **request_params(req, storage))
        _init_box(lat, req)
        lat.lb_step(req.steps)
        tot = lat.lb_totals()
        if keep is not None and req.rid in keep:
            _, u = lat.lb_moments()
            fields[req.rid] = u.cpu().numpy()
        t_done = time.perf_counter() - t0
        results.append(Result(req.rid, req.arrival, t_adm, t_done, req.steps, req.side ** 3, tot))
        lat.lb_destroy()
        del lat
        if log:
            log(f"done {req.rid} L={req.side} latency={t_done - req.arrival:.3f}s")
    torch.cuda.synchronize()
    return results, fields


def summarize(results):
    lat = np.array([r.latency for r in results])
    span = max(r.completed for r in results) - min(r.arrival for r in results)
    lups = sum(r.sites * r.steps for r in results)
    return {"runs": len(results), "makespan_s": round(span, 3),
            "runs_per_s": round(len(results) / span, 3),
            "p50_s": round(float(np.percentile(lat, 50)), 4),
            "p99_s": round(float(np.percentile(lat, 99)), 4),
            "mean_s": round(float(lat.mean()), 4),
            "aggregate_mlups": round(lups / span / 1e6, 1)}
