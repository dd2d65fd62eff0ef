"""Accuracy and cost of the multiple time-step schemes of Sec. 6 on the GPU
path: the coupling inside every sub-step (Eq. multistep, 2n coupling
evaluations per step), the coupling outside the sub-steps (F_h^1/2 around
[P F_int P]^n (C S) [P F_int P]^n, 2 coupling evaluations), and the Alg. 3
ordering without sub-steps.  Prints one JSON line per case.

  pair:   a bonded pair (harmonic, zero rest length) in a one-site fluid.  The
          fluid velocity cancels in the relative motion, which then obeys
          m w' = -gamma w - 2 k d: errors against the exact damped
          oscillator, for a unit-density cell and a heavy one.
  chains: bonded chains in a 64^3 fluid with the bond stiffness of the
          force-coupling workload (k = 30, m = 1, gamma = 2, tau = 0.6),
          from n = 3 sub-steps per side (the stability limit); bead
          positions and velocities and the fluid velocity against the
          coupling-inside run with the most sub-steps.
  cost:   milliseconds per step of the force-coupling workload (256^3, 10^4
          beads, FP32) with either scheme.

    python -m paper_1406_2211_amd.mts_study [--parts pair chains cost]
"""
import argparse
import json
import time

import numpy as np


def _lattice(n, **kw):
    from . import lbc as L
    return L.Lattice(n, n, n, **kw)


def pair_run(n, inside, rho0, steps=6, gamma=0.9, m=1.3, k=2.5):
    import torch
    lat = _lattice(1, max_particles=2, max_bonds=1, tau=0.8, coupling=1, gamma=gamma, kernel=2,
                   storage=0, mts_substeps=n, mts_inside=inside, rho0=rho0)
    lat.lb_init_fluid(None, torch.tensor([2e-3, 0.0, 0.0], dtype=torch.float64).reshape(3, 1, 1, 1))
    pos = torch.tensor([[0.56, 0.4, 0.6], [0.44, 0.4, 0.6]], dtype=torch.float64)
    vel = torch.tensor([[6e-3, 0.0, 0.0], [-4e-3, 0.0, 0.0]], dtype=torch.float64)
    lat.lb_set_particles(pos, vel, torch.full((2,), m, dtype=torch.float64))
    lat.lb_set_bonds(np.array([[0, 1]]), k, 0.0)
    lat.lb_step(steps)
    p, v = lat.lb_get_particles()
    p, v = p.cpu().numpy(), v.cpu().numpy()
    lat.lb_destroy()
    d = p[0, 0] - p[1, 0]
    d -= np.round(d)
    return d, v[0, 0] - v[1, 0]


def pair_part(out):
    from scipy.linalg import expm
    gamma, m, k, T = 0.9, 1.3, 2.5, 6
    ex = expm(np.array([[0.0, 1.0], [-2 * k / m, -gamma / m]]) * T) @ np.array([0.12, 0.01])
    for rho0 in (1.0, 1e6):
        for form, inside, ns in (("alg3", 0, (0,)), ("outside", 0, (1, 2, 4, 8, 16)),
                                 ("inside", 1, (1, 2, 4, 8, 16))):
            for n in ns:
                d, w = pair_run(n, inside, rho0, T, gamma, m, k)
                out({"part": "pair", "rho0": rho0, "form": form, "n": n,
                     "err_d": abs(d - ex[0]) / abs(ex[0]), "err_w": abs(w - ex[1]) / abs(ex[1])})


def chains_run(form, n, steps, size=64, nch=16, nb=50, seed=2, storage=0):
    import torch
    from . import inputs as I
    pos, vel, bonds = I.chains(nch, nb, (size, size, size), 1.0, 1e-3, seed)
    lat = _lattice(size, max_particles=len(pos), max_bonds=len(bonds), tau=0.6, collision=1,
                   coupling=1, gamma=2.0, kernel=2, storage=storage, mts_substeps=n,
                   mts_inside=1 if form == "inside" else 0)
    lat.lb_init_fluid()
    lat.lb_set_particles(torch.from_numpy(pos), torch.from_numpy(vel),
                         torch.ones(len(pos), dtype=torch.float64))
    lat.lb_set_bonds(bonds, 30.0, 1.0)
    lat.lb_step(steps)
    _, u = lat.lb_moments()
    p, v = lat.lb_get_particles()
    res = (p.cpu().numpy(), v.cpu().numpy(), u.cpu().numpy())
    lat.lb_destroy()
    return res


def chains_part(out, steps=200, nref=64, size=64):
    ref = chains_run("inside", nref, steps, size)
    L = float(size)
    # Alg. 3 and n <= 2 are beyond the stability limit of these bonds
    # (omega^2 = 4k/m for the fastest chain mode, omega dt < 2 needs n >= 3).
    for form, ns in (("outside", (3, 5, 10, 20, 40)), ("inside", (3, 5, 10, 20, 32))):
        for n in ns:
            p, v, u = chains_run(form, n, steps, size)
            dp = p - ref[0]
            dp -= L * np.round(dp / L)
            rec = {"part": "chains", "form": form, "n": n, "steps": steps, "ref": f"inside n={nref}",
                   "finite": bool(np.all(np.isfinite(v))),
                   "pos_err": float(np.abs(dp).max()),
                   "vel_rel": float(np.abs(v - ref[1]).max() / np.abs(ref[1]).max()),
                   "u_rel": float(np.abs(u - ref[2]).max() / np.abs(ref[2]).max()),
                   "vmax": float(np.abs(v).max())}
            out(rec)


def cost_part(out, steps=50, warmup=5):
    import torch
    from . import inputs as I
    n = 256
    pos, vel, bonds = I.chains(100, 100, (n, n, n), 1.0, 1e-3, 2)
    for form, ns in (("outside", (3, 5)), ("inside", (3, 5))):
        for sub in ns:
            lat = _lattice(n, max_particles=len(pos), max_bonds=len(bonds), tau=0.6, collision=1,
                           coupling=1, gamma=2.0, kernel=2, storage=1, mts_substeps=sub,
                           mts_inside=1 if form == "inside" else 0)
            lat.lb_init_fluid()
            lat.lb_set_particles(torch.from_numpy(pos), torch.from_numpy(vel),
                                 torch.ones(len(pos), dtype=torch.float64))
            lat.lb_set_bonds(bonds, 30.0, 1.0)
            lat.lb_step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lat.lb_step(steps)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            lat.lb_destroy()
            out({"part": "cost", "workload": "256^3 FP32, 10^4 beads, k = 30", "form": form,
                 "n": sub, "ms_per_step": round(ms, 4)})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--parts", nargs="+", default=["pair", "chains", "cost"])
    a = ap.parse_args()

    def out(rec):
        print(json.dumps(rec), flush=True)

    t0 = time.time()
    if "pair" in a.parts:
        pair_part(out)
    if "chains" in a.parts:
        chains_part(out)
    if "cost" in a.parts:
        cost_part(out)
    out({"elapsed_s": round(time.time() - t0, 1)})


if __name__ == "__main__":
    main()
