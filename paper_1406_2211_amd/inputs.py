"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

This module holds no arithmetic of the lattice Boltzmann method or of the
coupling: it only draws random numbers and builds geometry (chain random
walks, icosphere shells, non-overlapping centres, request mixes), so both the
GPU path and the CPU oracle can be fed the very same arrays.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(int(seed))


def noise_velocity(shape_zyx, amplitude: float, seed: int) -> np.ndarray:
    """u0 ~ U(-amplitude, amplitude) per component, layout [3, nz, ny, nx]."""
    g = rng(seed)
    return g.uniform(-amplitude, amplitude, size=(3,) + tuple(shape_zyx))


def uniform_positions(n: int, box, seed: int) -> np.ndarray:
    g = rng(seed)
    return g.uniform(0.0, 1.0, size=(n, 3)) * np.asarray(box, dtype=np.float64)[None, :]


def chains(nchains: int, nbeads: int, box, bond_length: float, vel_sd: float, seed: int):
    """Bead-spring chains: uniform-random heads, then a random walk whose steps
    have length ``bond_length`` and uniformly distributed directions.  Returns
    (pos [n,3], vel [n,3], bonds [nchains*(nbeads-1), 2] int32)."""
    g = rng(seed)
    box = np.asarray(box, dtype=np.float64)
    pos = np.zeros((nchains, nbeads, 3))
    pos[:, 0, :] = g.uniform(0.0, 1.0, size=(nchains, 3)) * box
    d = g.normal(size=(nchains, nbeads - 1, 3))
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    pos[:, 1:, :] = pos[:, :1, :] + np.cumsum(bond_length * d, axis=1)
    pos = pos.reshape(-1, 3)
    pos = pos - box * np.floor(pos / box)
    vel = g.normal(0.0, vel_sd, size=pos.shape)
    idx = np.arange(nchains * nbeads).reshape(nchains, nbeads)
    bonds = np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], axis=1).astype(np.int32)
    return pos, vel, bonds


def icosphere(subdivisions: int, radius: float) -> np.ndarray:
    """Vertices of a subdivided icosahedron projected onto a sphere of the given
    radius and centred on the origin (642 vertices for 3 subdivisions)."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
             (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdivisions):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    v = radius * np.array(verts)
    return v - v.mean(axis=0, keepdims=True)


def shell_centres(n: int, radius: float, box, wall_y: bool, min_gap: float, wall_gap: float,
                  seed: int, max_tries: int = 200000) -> np.ndarray:
    """Rejection-sample n centres with pairwise distance >= 2*radius + min_gap
    (minimum image in periodic directions) and, with y walls, at least
    radius + wall_gap from each wall plane y = -1/2 and y = ny - 1/2."""
    g = rng(seed)
    box = np.asarray(box, dtype=np.float64)
    out = []
    tries = 0
    while len(out) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place all shells")
        c = g.uniform(0.0, 1.0, size=3) * box
        if wall_y:
            lo, hi = -0.5 + radius + wall_gap, box[1] - 0.5 - radius - wall_gap
            if hi < lo:
                raise RuntimeError("channel too narrow for the shells")
            c[1] = lo + (hi - lo) * g.uniform()
        ok = True
        for o in out:
            d = c - o
            for a in range(3):
                if a == 1 and wall_y:
                    continue
                d[a] -= box[a] * np.round(d[a] / box[a])
            if np.linalg.norm(d) < 2 * radius + min_gap:
                ok = False
                break
        if ok:
            out.append(c)
    return np.array(out)


@dataclass
class Request:
    """One ensemble request of the serving workload."""
    rid: int
    arrival: float
    side: int
    nparticles: int
    tau: float
    fext: float
    steps: int
    seed: int
    extra: dict = field(default_factory=dict)


def serving_requests(n: int, rate: float, seed: int, side_range=(32, 160),
                     np_range=(10, 5000), tau_range=(0.55, 1.0), fext_max=1e-5,
                     steps_range=(200, 2000)):
    """Poisson arrivals at ``rate`` per second; side and particle count
    log-uniform, tau and body force uniform, step count uniform integer."""
    g = rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += g.exponential(1.0 / rate)
        side = int(round(math.exp(g.uniform(math.log(side_range[0]), math.log(side_range[1])))))
        npart = int(round(math.exp(g.uniform(math.log(np_range[0]), math.log(np_range[1])))))
        out.append(Request(rid=k, arrival=t, side=side, nparticles=npart,
                           tau=float(g.uniform(*tau_range)), fext=float(g.uniform(0.0, fext_max)),
                           steps=int(g.integers(steps_range[0], steps_range[1] + 1)),
                           seed=int(g.integers(0, 2**31 - 1))))
    return out
