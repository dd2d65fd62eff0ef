"""Throughput of the split-forcing D3Q19 lattice Boltzmann step with
fluid-particle coupling on one MI355X.

Default workload (force coupling at scale): periodic 256^3 box, two-rate MRT
(TRT rates, magic 3/16) with tau = 0.6, populations stored in FP32 as
deviations from w rho0 with FP32 compute; 100 bead-spring chains of 100 beads
(10^4 particles, harmonic k = 30, r0 = 1, mass 1, velocities N(0, 1e-3)),
force coupling gamma = 2 with the two-point kernel, and the multiple
time-step split with the coupling outside and 5 sub-steps per side (the bond
stiffness is beyond the stability limit of the single-step ordering at
h = 1).  Inputs are synthetic and seeded.  One step is the whole hot path:
both coupling half steps, the bond sub-steps and the fused lattice pass.

With the default workload the same JSON line also carries the cost of the
other multiple time-step scheme (the coupling inside every sub-step) and the
serving pass over the ensemble request set (batched FP16 against per-run FP32:
runs/s, p50/p99 time-to-result, and the FP16 velocity error checked against
its stated bound; the exit status is non-zero above it).

Prints one JSON line.  --gpus above 1 is refused (single-GPU build).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("MLUPS & HBM GB/s fraction (D3Q19+coupling); ensemble runs/s + p50/p99 latency")
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1406_2211_amd/csrc/lbc_kernels.hip",
                  "paper_1406_2211_amd/csrc/lbc_device.h",
                  "paper_1406_2211_amd/csrc/lbc_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stream_collide_c2.json")


def workload(name):
    from paper_1406_2211_amd import inputs as I
    if name == "c2":
        n = 256
        pos, vel, bonds = I.chains(100, 100, (n, n, n), 1.0, 1e-3, seed=2)
        return dict(
            desc="D3Q19 two-rate MRT (TRT rates) 256^3 periodic, tau=0.6, FP32 storage/compute; "
                 "10^4 particles in 100 harmonic chains (k=30, r0=1, m=1), force coupling "
                 "gamma=2, 2-point kernel, multiple time-step split with the coupling outside "
                 "the sub-steps (Sec. 6, second decomposition), n=5 sub-steps per side",
            grid=(n, n, n, 0),
            params=dict(tau=0.6, collision=1, coupling=1, gamma=2.0, kernel=2, storage=1,
                        mts_substeps=5),
            pos=pos, vel=vel, mass=np.ones(len(pos)), bonds=bonds, bond_k=30.0, bond_r0=1.0,
            bytes_per_site=152, dtype="f32")
    if name == "c2inside":
        wl = workload("c2")
        wl["desc"] = wl["desc"].replace(
            "multiple time-step split with the coupling outside the sub-steps (Sec. 6, second "
            "decomposition), n=5 sub-steps per side",
            "multiple time-step split with the coupling inside every sub-step (Eq. multistep), "
            "n=5 sub-steps per side")
        wl["params"] = dict(wl["params"], mts_inside=1)
        return wl
    if name == "c2thermal":
        wl = workload("c2")
        wl["desc"] = ("thermal c2: " + wl["desc"] + "; fluctuating collision and random coupling "
                      "force at kT=1e-5 (Philox4x32-10, seed 2)")
        wl["params"] = dict(wl["params"], kT=1e-5, seed=2)
        return wl
    if name == "c2mrt":
        wl = workload("c2")
        wl["desc"] = ("c2 with the general MRT collision: " + wl["desc"] + "; group rates bulk 1.4, "
                      "ghosts 1.2 (vector), 1.2 (pseudo-vector), 1.5 (scalar), 1.5 (tensor)")
        wl["params"] = dict(wl["params"], collision=2, mrt_rates=(1.4, 1.2, 1.2, 1.5, 1.5))
        return wl
    if name in ("c3", "c3phi2"):
        box = (128, 128, 256)
        T = I.icosphere(3, 6.0)
        cen = I.shell_centres(64, 6.0, box, True, 4.0, 3.0, seed=3)
        X = np.vstack([c + T for c in cen])
        k = 4 if name == "c3" else 2
        return dict(
            desc=f"D3Q19 BGK channel 128x128x256 with halfway bounce-back walls in y, tau=0.8, "
                 f"body force 1e-6 along z, FP32; 64 rigid icosphere shells (R=6, 642 markers each, "
                 f"tether k=0.05), immersed boundary coupling, {k}-point kernel",
            grid=box + (1,),
            params=dict(tau=0.8, body_force=(0.0, 0.0, 1e-6), collision=0, coupling=3, kernel=k,
                        storage=1),
            pos=X, vel=None, mass=None, nshell=64, template=T, tether_k=0.05,
            bytes_per_site=152, dtype="f32")
    if name == "plain256":
        n = 256
        return dict(desc="D3Q19 two-rate MRT 256^3 periodic, FP32, no particles", grid=(n, n, n, 0),
                    params=dict(tau=0.6, collision=1, storage=1), pos=None, bytes_per_site=152,
                    dtype="f32")
    if name == "c1":
        n = 32
        return dict(desc="D3Q19 BGK 32^3 periodic FP64, 1 particle, force coupling gamma=1",
                    grid=(n, n, n, 0),
                    params=dict(tau=0.8, body_force=(1e-6, 0, 0), coupling=1, gamma=1.0,
                                kernel=2, storage=0),
                    pos=I.uniform_positions(1, (n, n, n), 1), vel=np.zeros((1, 3)),
                    mass=np.ones(1), bytes_per_site=304, dtype="f64")
    raise SystemExit(f"unknown workload {name}")


def source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_record(N):
    """HBM bytes per launch of the fused lattice kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != source_hash() or rec.get("sites") != N:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(wl, steps):
    """The FP64 CPU oracle, untuned, on a bounded sample of the same workload."""
    import oracle as O
    nx, ny, nz, wall = wl["grid"]
    p = wl["params"]
    o = O.Oracle(nx=nx, ny=ny, nz=nz, wall_y=wall, tau=p["tau"], collision=p.get("collision", 0),
                 coupling=p.get("coupling", 0), gamma=p.get("gamma", 0.0),
                 kernel=p.get("kernel", 2), mts_n=p.get("mts_substeps", 0),
                 fext=p.get("body_force", (0, 0, 0)), bonds=wl.get("bonds"),
                 bond_k=wl.get("bond_k", 0.0), bond_r0=wl.get("bond_r0", 1.0),
                 nshell=wl.get("nshell", 0), shell_template=wl.get("template"),
                 tether_k=wl.get("tether_k", 0.0), kT=p.get("kT", 0.0), seed=p.get("seed", 0),
                 mrt_rates=p.get("mrt_rates", (1.0,) * 5))
    df = o.init_fluid()
    pos = None if wl.get("pos") is None else wl["pos"].copy()
    vel = None if pos is None or wl.get("vel") is None else wl["vel"].copy()
    t0 = time.perf_counter()
    o.run(df, steps, pos, vel, wl.get("mass"))
    dt = time.perf_counter() - t0
    return {"value": round(nx * ny * nz * steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": O.threads(), "kind": "oracle",
            "sample": f"{steps} full steps of the same workload ({nx}x{ny}x{nz}, all particles), "
                      f"{dt:.1f} s"}


def copy_calibration(nbytes=1 << 30, reps=3):
    import torch
    a = torch.ones(nbytes // 4, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_copy": nbytes, "copies": reps}), flush=True)


# Bound on the max-norm velocity error of a served FP16 run (comoving storage)
# against the same request run alone with FP32 storage, relative to the FP32
# field's largest velocity: 16-bit storage keeps 11 significant bits of the
# scaled deviations (2^-11 = 4.9e-4 per rounding); measured errors on the
# serving mix stay near 2e-5.
SERVING_VEL_BOUND = 1e-4


def serving_results(args):
    """Ensemble requests (256 periodic boxes, side log-uniform in [32,160],
    particles log-uniform in [10,5000], tau uniform in [0.55,1.0], body force
    uniform in [0,1e-5] along x, steps uniform in [200,2000], seed 5): the
    batched FP16-stored server (continuous batching over one ensemble,
    comoving storage frame) against the plain per-run FP32 FIFO.  Throughput is
    measured with every request queued at time 0; latency with Poisson arrivals
    at 0.8 times the measured FIFO capacity.  Returns the summary dict."""
    from paper_1406_2211_amd import inputs as I
    from paper_1406_2211_amd import serving as S
    nreq = args.requests
    base = I.serving_requests(nreq, 1.0, seed=5)
    sat = [I.Request(r.rid, 0.0, r.side, r.nparticles, r.tau, r.fext, r.steps, r.seed)
           for r in base]
    keep = {r.rid for r in base[:: max(1, nreq // 16)]}
    pool = int(args.pool_gb * (1 << 30))
    def phase(name):
        print(f"[c5] {name} ({time.strftime('%H:%M:%S')})", file=sys.stderr, flush=True)

    phase("saturated, per-run FP32 FIFO")
    fifo_sat, f32_fields = S.serve_fifo(sat, keep=keep)
    fifo_sum = S.summarize(fifo_sat)
    phase("saturated, batched FP16")
    host = {}
    ens_sat, f16_fields = S.serve_batched(sat, pool, max_slots=args.slots, keep=keep, prof=host)
    ens_sum = S.summarize(ens_sat)
    ens_sum["host"] = host
    errs = []
    for rid in keep:
        a, b = f16_fields[rid], f32_fields[rid]
        errs.append(float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)))
    rate = 0.8 * fifo_sum["runs_per_s"]
    scale = base[-1].arrival
    poisson = [I.Request(r.rid, r.arrival / scale * (nreq / rate), r.side, r.nparticles, r.tau,
                         r.fext, r.steps, r.seed) for r in base]
    phase("Poisson arrivals, per-run FP32 FIFO")
    fifo_p = S.summarize(S.serve_fifo(poisson)[0])
    phase("Poisson arrivals, batched FP16")
    ens_p = S.summarize(S.serve_batched(poisson, pool, max_slots=args.slots)[0])
    return {
        "workload": f"c5: {nreq} ensemble requests, periodic D3Q19 boxes side logU[32,160], "
                    "particles logU[10,5000] (FC, 2-point), tau U[0.55,1], body force "
                    "U[0,1e-5], steps U{200..2000}, seed 5",
        "pool_gb": args.pool_gb, "slots": args.slots,
        "saturated": {"batched_fp16": ens_sum, "fifo_fp32": fifo_sum,
                      "speedup_runs_per_s": round(ens_sum["runs_per_s"] / fifo_sum["runs_per_s"], 3)},
        "poisson": {"rate_per_s": round(rate, 3), "batched_fp16": ens_p, "fifo_fp32": fifo_p},
        "velocity_error_fp16_vs_fp32": {"max_rel": max(errs), "median_rel": float(np.median(errs)),
                                        "runs_checked": len(errs), "bound": SERVING_VEL_BOUND,
                                        "within_bound": bool(max(errs) <= SERVING_VEL_BOUND)},
    }


def bench_serving(args):
    """The serving workload alone, as its own JSON line."""
    sv = serving_results(args)
    sat = sv["saturated"]["batched_fp16"]
    out = {
        "metric": METRIC, "value": sat["runs_per_s"], "unit": "runs/s", "n_gpus": 1,
        "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f16 storage / f32 compute",
        "data": "synthetic",
        "config": {"workload": sv["workload"], "pool_gb": args.pool_gb, "slots": args.slots,
                   "parallelism": "single-gpu"},
        "serving": sv,
    }
    print(json.dumps(out), flush=True)
    if not sv["velocity_error_fp16_vs_fp32"]["within_bound"]:
        print("bench.py: FP16 serving velocity error above its bound", file=sys.stderr)
        sys.exit(1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--timing-stride", type=int, default=8,
                    help="time one lattice pass in every k of the timed steps with HIP events")
    ap.add_argument("--cpu-steps", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="c2: skip the serving pass (c5 request set) carried in the same line")
    ap.add_argument("--no-mts-inside", action="store_true",
                    help="c2: skip timing the coupling-inside multiple time-step scheme")
    ap.add_argument("--requests", type=int, default=256, help="c5: number of requests")
    ap.add_argument("--pool-gb", type=float, default=48.0, help="c5: ensemble pool size")
    ap.add_argument("--slots", type=int, default=64, help="c5: ensemble slots")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy three times (for scaling the "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "c5":
        bench_serving(args)
        return

    import torch

    wl = workload(args.workload)
    nx, ny, nz, wall = wl["grid"]
    N = nx * ny * nz
    npart = 0 if wl.get("pos") is None else len(wl["pos"])
    dt, lat_ms, passes = timed_run(wl, wl["params"], args.steps, args.warmup, args.timing_stride)
    mlups = N * args.steps / dt / 1e6
    bps = wl["bytes_per_site"]
    kern_s = lat_ms / 1e3 / max(passes, 1)
    achieved = bps * N / kern_s / 1e9
    traffic = traffic_record(N)
    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": wl["dtype"], "data": "synthetic",
        "config": {"workload": args.workload + ": " + wl["desc"], "sites": N,
                   "particles": npart, "parallelism": "single-gpu"},
        "hbm_gbs_step": round(bps * N * args.steps / dt / 1e9, 1),
        "roofline": {"bound": "hbm", "kernel": "k_stream_collide", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "avg_launch_us": round(kern_s * 1e6, 2),
                     "timed_launches": int(passes),
                     "algorithmic_bytes_per_launch": bps * N},
    }
    if wl["params"].get("mts_substeps", 0) > 0 and not args.no_mts_inside:
        # the other multiple time-step scheme of the same workload (Eq. multistep:
        # the coupling inside every sub-step, more accurate, 2n coupling
        # evaluations per step), timed the same way
        k = max(args.steps // 4, 1)
        dt2, _, _ = timed_run(wl, dict(wl["params"], mts_inside=1), k, min(args.warmup, 10), 0)
        out["mts_coupling_inside"] = {"steps": k, "ms_per_step": round(dt2 * 1e3 / k, 4),
                                      "mlups": round(N * k / dt2 / 1e6, 2)}
    torch.cuda.empty_cache()
    if args.workload == "c2" and not args.no_serving:
        out["serving"] = serving_results(args)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
    print(json.dumps(out), flush=True)
    sv = out.get("serving")
    if sv is not None and not sv["velocity_error_fp16_vs_fp32"]["within_bound"]:
        print("bench.py: FP16 serving velocity error above its bound", file=sys.stderr)
        sys.exit(1)


def timed_run(wl, params, steps, warmup, stride):
    """Builds the workload's context, runs warmup steps, then times steps
    (wall clock between two device synchronisations; with stride > 0 also the
    fused lattice passes with HIP events on the context stream).  Returns
    (seconds, summed lattice-pass ms, timed passes)."""
    import torch
    from paper_1406_2211_amd import lbc as L
    nx, ny, nz, wall = wl["grid"]
    pos = wl.get("pos")
    npart = 0 if pos is None else len(pos)
    bonds = wl.get("bonds")
    nshell = wl.get("nshell", 0)
    tmpl = wl.get("template")
    lat = L.Lattice(nx, ny, nz, wall_y=wall, max_particles=npart,
                    max_bonds=0 if bonds is None else len(bonds), max_shells=nshell,
                    max_shell_size=0 if tmpl is None else len(tmpl), **params)
    lat.lb_init_fluid()
    if npart:
        vel = None if wl.get("vel") is None else torch.from_numpy(wl["vel"])
        mass = None if wl.get("mass") is None else torch.from_numpy(wl["mass"])
        lat.lb_set_particles(torch.from_numpy(pos), vel, mass)
    if bonds is not None:
        lat.lb_set_bonds(bonds, wl["bond_k"], wl["bond_r0"])
    if nshell:
        lat.lb_set_shells(nshell, tmpl, wl["tether_k"])
    lat.lb_step(warmup)
    torch.cuda.synchronize()
    if stride > 0:
        lat.lb_timing(steps, stride)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.lb_step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat_ms, passes = lat.lb_timing_read() if stride > 0 else (0.0, 0)
    tot = lat.lb_totals()
    lat.lb_destroy()
    del lat
    if not np.all(np.isfinite(tot)):
        print("bench.py: non-finite state after the timed steps", file=sys.stderr)
        sys.exit(1)
    return dt, lat_ms, passes


if __name__ == "__main__":
    main()
