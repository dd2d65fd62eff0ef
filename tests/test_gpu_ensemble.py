"""Batched ensembles of uneven periodic boxes: every slot against the oracle run
alone, the same request alone and in a mix, admission by footprint, uneven
step budgets and the autotuner."""
import numpy as np
import pytest

from paper_1406_2211_amd import inputs as I
from parity import Case, compare, run_oracle, to_oracle_order

pytestmark = pytest.mark.gpu

SPECS = [
    # side, particles, tau, body force (x), steps, coupling, collision, seed
    (20, 5, 0.7, 3e-6, 30, 1, 0, 11),
    (13, 3, 0.9, 0.0, 17, 2, 1, 12),
    (32, 0, 0.55, 1e-5, 30, 0, 1, 13),
    (9, 7, 0.62, 2e-6, 24, 1, 1, 14),
]


def _case(spec, storage=0, steps=None):
    n, npart, tau, fx, st, coupling, col, seed = spec
    pos = I.uniform_positions(npart, (n, n, n), seed) if npart else None
    vel = np.random.default_rng(seed).normal(0, 1e-3, (npart, 3)) if npart else None
    return Case(name=f"ens_{n}_{npart}", nx=n, ny=n, nz=n, tau=tau,
                steps=st if steps is None else steps, fext=(fx, 0.0, 0.0), collision=col,
                coupling=coupling, gamma=1.3, kernel=2, storage=storage, u_noise=1e-4, seed=seed,
                pos=pos, vel=vel, mass=None if pos is None else np.ones(npart))


def _admit(ens, c):
    import torch
    from parity import initial_fields
    got = ens.admit(c.nx, c.ny, c.nz, c.steps, max_particles=0 if c.pos is None else len(c.pos),
                    tau=c.tau, body_force=c.fext, collision=c.collision, coupling=c.coupling,
                    gamma=c.gamma, kernel=c.kernel, storage=c.storage,
                    f16_scale_log2=c.f16_scale_log2)
    assert got is not None
    slot, lat = got
    _, u = initial_fields(c)
    lat.lb_init_fluid(None, torch.from_numpy(np.ascontiguousarray(u)))
    if c.pos is not None:
        lat.lb_set_particles(torch.from_numpy(c.pos), torch.from_numpy(c.vel),
                             torch.from_numpy(c.mass))
        lat.np = len(c.pos)
    return slot, lat


def _read(ens, slot, lat, c):
    ens.query(slot)
    rho, u = lat.lb_moments()
    df = lat.lb_populations()
    out = dict(df=df.cpu().numpy(), rho=rho.cpu().numpy(), u=u.cpu().numpy(), pos=None, vel=None)
    if c.pos is not None:
        p, v = lat.lb_get_particles()
        out["pos"], out["vel"] = p.cpu().numpy(), v.cpu().numpy()
    return out


def _pool_for(cases, extra=1.2, slack=8 << 20):
    from paper_1406_2211_amd import lbc as L
    tot = 0
    for c in cases:
        tot += L.ensemble_footprint(c.nx, c.ny, c.nz, 0 if c.pos is None else len(c.pos),
                                    tau=c.tau, storage=c.storage, kernel=c.kernel,
                                    coupling=c.coupling, gamma=c.gamma) + 4096
    return int(tot * extra) + slack


def test_ensemble_slots_match_oracle_fp64():
    from paper_1406_2211_amd import lbc as L
    cases = [_case(s) for s in SPECS]
    ens = L.Ensemble(_pool_for(cases), max_slots=8, storage=L.LB_F64, kernel=2)
    handles = [_admit(ens, c) for c in cases]
    print("[gpu] ensemble fp64 with", len(cases), "slots", flush=True)
    ens.step(max(c.steps for c in cases) + 5)  # every slot stops at its own budget
    for c, (slot, lat) in zip(cases, handles):
        done, fin = ens.query(slot)
        assert done == c.steps and fin
        g = _read(ens, slot, lat, c)
        compare(c, g, run_oracle(c), 1e-12)
    ens.destroy()


@pytest.mark.parametrize("det", [1, 0])
@pytest.mark.parametrize("storage,tol", [(1, 1e-6), (2, 1e-4)])
def test_same_alone_and_in_the_mix(storage, tol, det):
    """Each request run alone and in a mix of uneven boxes.  With the
    deterministic spread (det = 1) the results are bitwise equal, particles
    included; with atomic spreading only boxes without particles are, and the
    others agree to the storage precision's round-off (measured up to about
    1e-7 in FP32 and 2e-5 in FP16)."""
    from paper_1406_2211_amd import lbc as L
    cases = [_case(s, storage=storage) for s in SPECS]
    for c in cases:
        c.f16_scale_log2 = 20
    mix = L.Ensemble(_pool_for(cases), max_slots=8, storage=storage, kernel=2, deterministic=det)
    hs = [_admit(mix, c) for c in cases]
    mix.step(40)
    for i, c in enumerate(cases):
        alone = L.Ensemble(_pool_for([c]), max_slots=1, storage=storage, kernel=2,
                           deterministic=det)
        slot, lat = _admit(alone, c)
        alone.step(40)
        a = _read(alone, slot, lat, c)
        m = _read(mix, hs[i][0], hs[i][1], c)
        scale = np.abs(a["u"]).max()
        err = np.abs(a["u"] - m["u"]).max() / scale
        print(f"[ensemble] storage={storage} det={det} slot {i}: alone vs mix u err {err:.2e}",
              flush=True)
        assert err <= tol
        if det or c.pos is None:  # no order-dependent sums: identical
            for k in ("df", "u", "pos", "vel"):
                assert a[k] is None or np.array_equal(a[k], m[k]), (i, k)
        alone.destroy()
    mix.destroy()


def test_admission_by_footprint_and_retire():
    """A pool sized for two boxes refuses a third (LB_EBUSY) and accepts it once
    one is retired; a full slot table refuses as well."""
    from paper_1406_2211_amd import lbc as L
    small = _case(SPECS[0])
    # room for the ensemble tables (< 200 kB here) and exactly two boxes
    ens = L.Ensemble(_pool_for([small, small], extra=1.0, slack=200_000), max_slots=4,
                     storage=L.LB_F64, kernel=2)
    a = _admit(ens, small)
    _admit(ens, small)
    kw = dict(max_particles=5, tau=0.7, storage=L.LB_F64, coupling=1, gamma=1.3)
    assert ens.admit(small.nx, small.ny, small.nz, 5, **kw) is None  # footprint does not fit
    ens.step(3)
    ens.retire(a[0])
    got = ens.admit(small.nx, small.ny, small.nz, 5, **kw)
    assert got is not None and got[0] == a[0]
    ens.destroy()
    ens = L.Ensemble(_pool_for([small] * 3), max_slots=2, storage=L.LB_F64, kernel=2)
    _admit(ens, small)
    _admit(ens, small)
    assert ens.admit(small.nx, small.ny, small.nz, 5, **kw) is None  # slot table full
    ens.destroy()


def test_autotune_steps_are_real_steps():
    from paper_1406_2211_amd import lbc as L
    cases = [_case(s, steps=200) for s in SPECS]
    ens = L.Ensemble(_pool_for(cases), max_slots=4, storage=L.LB_F64, kernel=2)
    hs = [_admit(ens, c) for c in cases]
    lg, pg = ens.autotune(2)
    assert lg > 0 and pg > 0
    ens.step(9)
    for c, (slot, lat) in zip(cases, hs):
        done, _ = ens.query(slot)
        c.steps = done
        compare(c, _read(ens, slot, lat, c), run_oracle(c), 1e-12)
    ens.destroy()
