"""CPU checks of the C ABI: the built library loads and exports every entry
point that include/lbc.h declares, and host-side validation rejects invalid
configurations before anything touches a device."""
import os
import re

import numpy as np

import pytest

from paper_1406_2211_amd import lbc as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lbc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    syms = declared_symbols()
    assert len(syms) >= 16
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing
    assert set(syms) <= set(L.EXPORTS) | set(syms)


def test_lattice_velocities_are_d3q19():
    c = L.lattice_velocities()
    assert c.shape == (19, 3)
    s = set(map(tuple, c.tolist()))
    assert len(s) == 19 and (0, 0, 0) in s
    assert all(tuple(-v for v in t) in s for t in s)
    assert sorted((abs(c).sum(1)).tolist()) == [0] + [1] * 6 + [2] * 12


def _g(nx=8, ny=8, nz=8, wall=0):
    return L.lb_grid(nx, ny, nz, wall)


def _lim(n=0, nb=0, ns=0, ms=0):
    return L.lb_limits(n, nb, ns, ms)


def test_workspace_size_scales_with_storage():
    sizes = [L.workspace_size(_g(64, 64, 64), L.make_params(0.8, storage=s), _lim())
             for s in (L.LB_F64, L.LB_F32, L.LB_F16)]
    assert sizes[0] > sizes[1] > sizes[2]
    # two population buffers dominate: 2 * 19 * N * bytes
    N = 64 ** 3
    assert sizes[1] >= 2 * 19 * N * 4


@pytest.mark.parametrize("storage,vec", [(L.LB_F32, 16), (L.LB_F64, 32)])
def test_workspace_of_coupling_inside_substeps(storage, vec):
    """The coupling inside the sub-steps holds min(n - 1, 4) force fields of
    its own and a second copy of the particle state; the deterministic mode,
    which keeps three launches per sub-step, holds neither."""
    g, N, npart = _g(32, 32, 32), 32 ** 3, 100
    base = dict(coupling=L.LB_COUPLE_FC, gamma=1.0, storage=storage, mts_substeps=1)

    def size(**kw):
        return L.workspace_size(g, L.make_params(0.8, **dict(base, **kw)), _lim(n=npart, nb=99))

    outside = size()
    for n, fields in ((1, 0), (2, 1), (5, 4), (9, 4)):
        extra = size(mts_substeps=n, mts_inside=1) - size(mts_substeps=n)
        assert fields * N * vec <= extra < fields * N * vec + 64 * 1024, (n, extra)
    assert size(mts_substeps=5, mts_inside=1, deterministic=1) - size(
        mts_substeps=5, deterministic=1) < 64 * 1024
    assert outside > 0


@pytest.mark.parametrize("bad", [
    dict(tau=0.5), dict(tau=0.3), dict(tau=float("nan")), dict(tau=0.8, rho0=0.0),
    dict(tau=0.8, collision=7), dict(tau=0.8, coupling=9), dict(tau=0.8, kernel=5),
    dict(tau=0.8, storage=9), dict(tau=0.8, coupling=L.LB_COUPLE_FC, gamma=0.0),
    dict(tau=0.8, coupling=L.LB_COUPLE_IB, mts_substeps=3), dict(tau=0.8, mts_substeps=-1),
    dict(tau=0.8, body_force=(float("inf"), 0, 0)),
    dict(tau=0.8, csc=1), dict(tau=1.2, collision=1, trt_magic=3.0 / 16.0, csc=1),
    dict(tau=1.2, csc=2), dict(tau=0.8, coupling=1, gamma=1.0, mts_inside=1),
    dict(tau=0.8, coupling=1, gamma=1.0, mts_substeps=2, mts_inside=2),
    dict(tau=0.8, collision=2, mrt_rates=(1.0, 2.0, 1.0, 1.0, 1.0)),
    dict(tau=0.8, collision=2, mrt_rates=(0.0, 1.0, 1.0, 1.0, 1.0)),
    dict(tau=1.2, collision=2, csc=1), dict(tau=0.8, collision=2, comoving=1),
    dict(tau=0.8, kT=-1.0), dict(tau=1.2, kT=1e-4, csc=1), dict(tau=0.8, kT=1e-4, comoving=1),
])
def test_invalid_parameters_rejected(bad):
    with pytest.raises(L.LbcError) as e:
        L.workspace_size(_g(), L.make_params(**bad), _lim())
    assert e.value.status == L.LB_EINVAL


@pytest.mark.parametrize("grid", [(0, 8, 8, 0), (8, -1, 8, 0), (8, 1, 8, 1), (8, 8, 8, 2)])
def test_invalid_grid_rejected(grid):
    with pytest.raises(L.LbcError):
        L.workspace_size(L.lb_grid(*grid), L.make_params(0.8), _lim())


def test_invalid_limits_rejected():
    with pytest.raises(L.LbcError):
        L.workspace_size(_g(), L.make_params(0.8), _lim(n=-5))


def test_create_rejects_small_workspace_without_device():
    import ctypes as C
    g, p, m = _g(), L.make_params(0.8), _lim()
    need = L.workspace_size(g, p, m)
    ctx = C.c_void_p()
    st = L.load().lb_create(C.byref(g), C.byref(p), C.byref(m), C.c_void_p(256), need - 1, None,
                            C.byref(ctx))
    assert st == L.LB_ENOMEM and not ctx.value
    assert b"workspace" in L.load().lb_last_error(None)


def test_status_strings():
    lib = L.load()
    for s in range(6):
        assert lib.lb_status_string(s)


def test_serving_request_generator_ranges():
    from paper_1406_2211_amd import inputs as I
    reqs = I.serving_requests(256, 10.0, seed=5)
    sides = np.array([r.side for r in reqs])
    nps = np.array([r.nparticles for r in reqs])
    assert sides.min() >= 32 and sides.max() <= 160
    assert nps.min() >= 10 and nps.max() <= 5000
    assert all(0.55 <= r.tau <= 1.0 and 0 <= r.fext <= 1e-5 and 200 <= r.steps <= 2000 for r in reqs)
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) > 0)
    assert 15.0 < arr[-1] < 40.0  # 256 arrivals at 10/s


@pytest.mark.parametrize("ok", [dict(tau=1.0, csc=1), dict(tau=1.0, collision=1, trt_magic=0.25, csc=1),
                                dict(tau=1.2, collision=1, trt_magic=0.5, csc=1)])
def test_collide_stream_collide_accepts_rates_up_to_one(ok):
    """The exact half collision sqrt(1 - lambda) is real for every rate <= 1
    (lambda = 1 included: the half collision then returns the equilibrium)."""
    assert L.workspace_size(_g(), L.make_params(**ok), _lim()) > 0
