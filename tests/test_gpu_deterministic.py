"""Deterministic spreading (lb_params.deterministic = 1): the sum at each
site of the spread contributions (Eq. IBM-spreading) is formed exactly in
fixed point, so runs are bitwise reproducible.  Checked against the oracle
(FP64, 1e-12) for every coupling path, run to run (bitwise, FP32 and FP16),
and against the atomic spread (round-off)."""
import numpy as np
import pytest

from paper_1406_2211_amd import inputs as I
from parity import Case, compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def _chains(name, n, mts, inside=0, storage=0, k=0.02, steps=12, coupling=1):
    pos, vel, bonds = I.chains(3, 10, (n, n, n), 1.0, 2e-2, 6)
    c = Case(name=name, nx=n, ny=n, nz=n, tau=0.7, steps=steps, collision=1, coupling=coupling,
             gamma=1.5, kernel=2, storage=storage, mts=mts, u_noise=1e-3, pos=pos, vel=vel,
             mass=np.full(len(pos), 2.0), bonds=bonds, bond_k=k, bond_r0=1.0,
             fext=(1e-6, -2e-6, 0.0))
    c.extra["mts_inside"] = inside
    c.extra["deterministic"] = 1
    return c


def _ib(name, kernel, storage=0, steps=12):
    T = I.icosphere(1, 4.0)
    cen = I.shell_centres(2, 4.0, (24, 24, 32), True, 2.0, 3.0, seed=3)
    X = np.vstack([c + T for c in cen])
    X = X + 0.15 * np.random.default_rng(5).standard_normal(X.shape)
    c = Case(name=name, nx=24, ny=24, nz=32, tau=0.8, steps=steps, wall_y=1,
             fext=(0.0, 0.0, 1e-6), coupling=3, kernel=kernel, storage=storage, u_noise=0.0,
             pos=X, nshell=2, template=T, tether_k=0.05)
    c.extra["deterministic"] = 1
    return c


CASES = {
    "alg3_fc": lambda: _chains("det_alg3", 20, 0),
    "alg3_ebf_phi3": lambda: (lambda c: (setattr(c, "kernel", 3), setattr(c, "coupling", 2), c)[-1])(
        _chains("det_ebf", 18, 0)),
    "mts_outside": lambda: _chains("det_mts", 20, 3),
    "mts_inside": lambda: _chains("det_mts_in", 20, 2, inside=1),
    "ib_tiles_phi4": lambda: _ib("det_ib4", 4),
    "ib_direct_phi2": lambda: _ib("det_ib2", 2),
}


@pytest.mark.parametrize("which", sorted(CASES))
def test_deterministic_spread_matches_oracle_fp64(which):
    c = CASES[which]()
    compare(c, run_gpu(c), run_oracle(c), 1e-12)


def _bitwise_twice(c):
    a, b = run_gpu(c), run_gpu(c)
    for k in ("df", "u", "pos", "vel"):
        assert np.array_equal(a[k], b[k]), k
    return a


@pytest.mark.parametrize("storage", [1, 2])
def test_runs_are_bitwise_reproducible(storage):
    """Chains with many shared stencil sites (multiple time steps) and dense
    IB shells, each run twice in 16-bit and FP32 storage: identical bits."""
    c = _chains("det_rep", 32, 3, storage=storage, steps=30)
    c.f16_scale_log2 = 20
    _bitwise_twice(c)
    d = _ib("det_rep_ib", 4, storage=storage, steps=20)
    d.f16_scale_log2 = 22
    _bitwise_twice(d)


def test_deterministic_and_atomic_spread_agree_to_round_off():
    c = _chains("det_vs_atomic", 32, 3, storage=1, steps=30)
    a = run_gpu(c)
    c.extra["deterministic"] = 0
    b = run_gpu(c)
    err = np.abs(a["u"] - b["u"]).max() / np.abs(b["u"]).max()
    print(f"[det] FP32 deterministic vs atomic spread: u {err:.2e}", flush=True)
    assert err < 1e-6
