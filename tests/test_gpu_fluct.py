"""GPU parity of the fluctuating lattice Boltzmann method (Eq. mrt-fluct) and
of the random force of the force coupling (Eq. viscous-coupling) against the
FP64 oracle, which draws the same Philox4x32-10 numbers and adds the noise in
moment space with its own basis.  Tolerances as in the other parity tests
(FP64 storage 1e-12, for bonded chains 20 times the oracle's one-ulp
sensitivity if larger; FP32 storage 1e-5).  A property check at a larger
size: the populations of the thermalised fluid have the equilibrium variance
mu rho0 w_i (mu = 3 k_B T) and are uncorrelated."""
import numpy as np
import pytest

from paper_1406_2211_amd import inputs as I
from parity import Case, compare, run_gpu, run_oracle, ulp_sensitivity

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
KT = 1e-5


def _fl(c, kT=KT, seed=(7 << 32) + 123):
    c.extra.update(kT=kT, seed=seed)
    return c


def _parts(n, box, seed):
    pos = I.uniform_positions(n, box, seed)
    vel = np.random.default_rng(seed).normal(0.0, 1e-3, (n, 3))
    return pos, vel, np.ones(n)


def _check(c, tol):
    o = run_oracle(c)
    sens = ulp_sensitivity(c, o) if c.bonds is not None else 0.0
    return compare(c, run_gpu(c), o, tol, sens=sens)


def test_bgk_ragged_box_body_force_fp64():
    c = Case(name="fl_bgk", nx=12, ny=10, nz=14, tau=0.8, steps=30, fext=(1e-6, 0.0, 0.0))
    _check(_fl(c), TOL64)


def test_trt_walls_row_layout_fp64():
    c = Case(name="fl_trt_walls", nx=64, ny=9, nz=6, tau=0.7, steps=25, wall_y=1, collision=1,
             fext=(0.0, 0.0, 1e-6))
    _check(_fl(c), TOL64)


@pytest.mark.parametrize("kernel", [2, 3])
def test_force_coupling_with_random_force_fp64(kernel):
    pos, vel, m = _parts(30, (16, 16, 16), 5)
    c = Case(name=f"fl_fc_phi{kernel}", nx=16, ny=16, nz=16, tau=0.9, steps=30, coupling=1,
             gamma=1.2, kernel=kernel, pos=pos, vel=vel, mass=m, fext=(0.0, 1e-6, 0.0))
    _check(_fl(c), TOL64)


def test_ebf_and_ib_fluid_noise_fp64():
    pos, vel, m = _parts(10, (14, 14, 14), 6)
    c = Case(name="fl_ebf", nx=14, ny=14, nz=14, tau=0.8, steps=20, coupling=2, gamma=1.0,
             kernel=3, pos=pos, vel=vel, mass=m)
    _check(_fl(c), TOL64)
    T = I.icosphere(1, 3.0)
    # markers off the template shape, as in the other IB cases: with the
    # markers exactly on it the rigid fit is ill-conditioned
    X = np.array([8.0, 8.2, 9.1]) + T + 0.15 * np.random.default_rng(5).standard_normal(T.shape)
    c = Case(name="fl_ib", nx=16, ny=16, nz=18, tau=0.8, steps=20, wall_y=1, coupling=3,
             kernel=4, u_noise=0.0, pos=X, nshell=1, template=T, tether_k=0.05)
    _check(_fl(c), TOL64)


@pytest.mark.parametrize("inside", [0, 1])
def test_chains_multiple_time_steps_fp64(inside):
    pos, vel, bonds = I.chains(2, 10, (20, 20, 20), 1.0, 1e-3, 3)
    c = Case(name=f"fl_mts_in{inside}", nx=20, ny=20, nz=20, tau=0.7, steps=20, collision=1,
             coupling=1, gamma=2.0, kernel=2, mts=3, pos=pos, vel=vel,
             mass=np.ones(len(pos)), bonds=bonds, bond_k=2.0, bond_r0=1.0)
    c.extra["mts_inside"] = inside
    _check(_fl(c), TOL64)


def test_step_counter_continues_across_calls():
    """The random streams are indexed by the step count, so a run split into
    several calls draws the same numbers as one call."""
    pos, vel, m = _parts(12, (12, 12, 12), 9)
    c = Case(name="fl_chunks", nx=12, ny=12, nz=12, tau=0.8, steps=24, coupling=1, gamma=1.0,
             pos=pos, vel=vel, mass=m)
    c.extra["chunks"] = [1, 5, 3, 15]
    _check(_fl(c), TOL64)


def test_force_coupling_fp32():
    pos, vel, m = _parts(40, (24, 24, 24), 10)
    c = Case(name="fl_fc32", nx=24, ny=24, nz=24, tau=0.8, steps=40, coupling=1, gamma=1.0,
             storage=1, pos=pos, vel=vel, mass=m)
    _check(_fl(c), TOL32)


@pytest.mark.parametrize("collision,tau", [(0, 0.8), (1, 0.6)])
def test_thermal_equilibrium_populations_64cubed_fp32(collision, tau):
    """Property at a larger size (64^3, FP32, the row-mapped pass): after
    thermalisation every population deviation has variance mu rho0 w_i and
    neighbouring directions are uncorrelated (the equilibrium of the
    fluctuating LB), to within 2 %."""
    import torch
    from paper_1406_2211_amd import lbc as L
    kT = 1e-4
    lat = L.Lattice(64, 64, 64, tau=tau, collision=collision, storage=1, kT=kT, seed=99)
    lat.lb_init_fluid()
    print(f"[gpu] thermal equilibrium 64^3 collision={collision} tau={tau}", flush=True)
    lat.lb_step(400)
    acc = np.zeros(19)
    cross = 0.0
    nsamp = 20
    for _ in range(nsamp):
        lat.lb_step(5)
        df = lat.lb_populations().cpu().numpy().reshape(19, -1)
        acc += (df ** 2).mean(axis=1)
        cross += (df[1] * df[3]).mean()
    torch.cuda.synchronize()
    lat.lb_destroy()
    c = L.lattice_velocities()
    w = np.where(np.abs(c).sum(1) == 0, 1 / 3, np.where(np.abs(c).sum(1) == 1, 1 / 18, 1 / 36))
    ratio = acc / nsamp / (3 * kT * w)
    print(f"[fluct] variance / (mu rho0 w_i): min {ratio.min():.4f} max {ratio.max():.4f}",
          flush=True)
    assert np.all(np.abs(ratio - 1.0) < 0.02), ratio
    assert abs(cross / nsamp) < 0.02 * 3 * kT / 18


def test_full_size_thermal_force_coupling_fp32():
    """The thermal force-coupling workload at full size, in the launch
    configuration the benchmark times: 256^3 two-rate MRT, FP32 storage,
    10^4 bonded particles with the multiple time-step split, kT = 1e-5; every
    output compared with the oracle after 2 steps."""
    pos, vel, bonds = I.chains(100, 100, (256, 256, 256), 1.0, 1e-3, 2)
    c = Case(name="c2thermal_full", nx=256, ny=256, nz=256, tau=0.6, steps=2, collision=1,
             coupling=1, gamma=2.0, kernel=2, storage=1, mts=5, u_noise=0.0, pos=pos, vel=vel,
             mass=np.ones(len(pos)), bonds=bonds, bond_k=30.0, bond_r0=1.0)
    _check(_fl(c, kT=1e-5, seed=2), TOL32)
