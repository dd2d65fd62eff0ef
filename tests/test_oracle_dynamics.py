"""Pins of the oracle's full time step against what the paper and the
mathematics fix: rest is a fixed point, mass and momentum balance, the
viscosity of the scheme (shear-wave decay), Poiseuille flow between walls,
exact advection of IB markers, and the stiffness reading for bonded chains."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1406_2211_amd import inputs as I

RNG = np.random.default_rng(3)


def _random_state(o, amp_u=1e-3, amp_neq=1e-5, seed=0):
    g = np.random.default_rng(seed)
    rho = 1.0 + 1e-3 * g.standard_normal(o.shape)
    u = amp_u * g.standard_normal((3,) + o.shape)
    df = o.init_fluid(rho, u)
    return df + amp_neq * g.standard_normal(df.shape)


@pytest.mark.parametrize("collision", [O.BGK, O.TRT])
@pytest.mark.parametrize("wall", [0, 1])
def test_rest_is_a_fixed_point(collision, wall):
    """f = f^eq(rho0, 0) with no force stays exactly at rest (C f^eq = 0),
    including particles at rest under force coupling."""
    o = O.Oracle(nx=6, ny=5, nz=4, tau=0.7, collision=collision, wall_y=wall,
                 coupling=O.FC, gamma=1.0, kernel=2)
    df = o.init_fluid()
    pos = np.array([[1.3, 2.2, 3.1], [4.5, 2.5, 0.2]])
    vel = np.zeros((2, 3))
    o.run(df, 20, pos, vel, np.ones(2))
    assert np.all(df == 0.0) and np.all(vel == 0.0)


@pytest.mark.parametrize("collision", [O.BGK, O.TRT])
@pytest.mark.parametrize("wall", [0, 1])
def test_mass_conservation(collision, wall):
    o = O.Oracle(nx=7, ny=6, nz=5, tau=0.62, collision=collision, wall_y=wall,
                 fext=(1e-5, 0.0, -2e-5))
    df = _random_state(o)
    m0 = o.totals(df)[0]
    o.run(df, 30)
    assert abs(o.totals(df)[0] - m0) < 1e-13


@pytest.mark.parametrize("collision", [O.BGK, O.TRT])
def test_uniform_body_force_momentum(collision):
    """A constant body force raises the total momentum by h F N per step
    (Eq. LB-force-moments)."""
    F = np.array([1e-6, -2e-6, 5e-7])
    o = O.Oracle(nx=8, ny=6, nz=5, tau=0.8, collision=collision, fext=F)
    df = _random_state(o)
    p0 = o.totals(df)[1:4]
    o.run(df, 25)
    assert np.abs(o.totals(df)[1:4] - (p0 + 25 * o.N * F)).max() < 1e-13


def _chain_setup(coupling, mts_n=0, n=10, k=0.5):
    pos, vel, bonds = I.chains(1, n, (12, 12, 12), 1.0, 1e-3, 4)
    pos = pos + 0.1 * RNG.standard_normal(pos.shape)
    o = O.Oracle(nx=12, ny=12, nz=12, tau=0.7, coupling=coupling, gamma=1.5, kernel=3,
                 mts_n=mts_n, bonds=bonds, bond_k=k, bond_r0=1.0, collision=O.TRT)
    return o, pos, vel, np.full(n, 0.8)


@pytest.mark.parametrize("coupling,mts", [(O.FC, 0), (O.EBF, 0), (O.FC, 3), (O.EBF, 2)])
def test_fluid_plus_particle_momentum_conserved(coupling, mts):
    """Equal and opposite coupling forces (Sec. 5.2) with sum delta = 1 and
    internal bond forces summing to zero conserve fluid + particle momentum."""
    o, pos, vel, m = _chain_setup(coupling, mts)
    df = _random_state(o, amp_u=1e-4, amp_neq=0.0)
    t0 = o.totals(df, vel, m)
    o.run(df, 15, pos, vel, m)
    t1 = o.totals(df, vel, m)
    assert np.abs(vel).max() > 1e-6
    assert np.abs((t1[1:4] + t1[4:7]) - (t0[1:4] + t0[4:7])).max() < 1e-14
    assert abs(t1[0] - t0[0]) < 1e-13


def test_ib_momentum_conserved_with_body_force():
    """IB with tethered markers: the spread intrinsic forces sum to zero, so the
    fluid momentum only grows by the body-force impulse."""
    T = I.icosphere(1, 3.0)
    F = np.array([0.0, 0.0, 1e-6])
    o = O.Oracle(nx=16, ny=16, nz=16, tau=0.8, coupling=O.IB, kernel=4, fext=F,
                 nshell=1, shell_template=T, tether_k=0.05)
    X = np.array([8.0, 8.2, 7.9]) + T + 0.2 * RNG.standard_normal(T.shape)
    df = o.init_fluid()
    p0 = o.totals(df)[1:4]
    o.run(df, 10, X)
    assert np.abs(df).max() > 1e-6
    assert np.abs(o.totals(df)[1:4] - (p0 + 10 * o.N * F)).max() < 1e-13


def test_ib_markers_advect_exactly_in_uniform_flow():
    """In a uniform flow with no forces the IB position update (trapezoidal rule
    of Sec. 5.1) moves every marker by h u per step."""
    T = I.icosphere(0, 3.0)
    o = O.Oracle(nx=16, ny=16, nz=16, tau=0.8, coupling=O.IB, kernel=3,
                 nshell=1, shell_template=T, tether_k=0.05)
    u0 = np.array([1e-3, -2e-3, 5e-4])
    df = o.init_fluid(None, np.broadcast_to(u0[:, None, None, None], (3,) + o.shape))
    X0 = np.array([7.3, 8.1, 6.6]) + T
    X = X0.copy()
    o.run(df, 12, X)
    assert np.abs(X - (X0 + 12 * u0)).max() < 1e-13


def _shear_decay_nu(n, tau, collision):
    o = O.Oracle(nx=1, ny=n, nz=1, tau=tau, collision=collision)
    y = np.arange(n)
    U = 1e-5
    u = np.zeros((3, 1, n, 1))
    u[0, 0, :, 0] = U * np.sin(2 * np.pi * y / n)
    df = o.init_fluid(None, u)
    k = 2 * np.pi / n

    def amp():
        _, uu = o.moments(df)
        return 2.0 / n * (uu[0, 0, :, 0] * np.sin(k * y)).sum()

    o.run(df, 50)
    a1 = amp()
    T = 400
    o.run(df, T)
    a2 = amp()
    return -math.log(a2 / a1) / (k * k * T)


@pytest.mark.parametrize("collision", [O.BGK, O.TRT])
def test_shear_wave_viscosity(collision):
    """The shear mode decays with nu = cs2 (tau - 1/2) (Sec. 4 viscosity with the
    lattice relaxation time), with second-order convergence in k."""
    tau = 0.8
    nu = (tau - 0.5) / 3.0
    e = [abs(_shear_decay_nu(n, tau, collision) / nu - 1.0) for n in (16, 32)]
    assert e[1] < 4e-3
    assert 3.5 < e[0] / e[1] < 4.5


def _poiseuille(ny, tau, collision, steps):
    F = 1e-6
    o = O.Oracle(nx=1, ny=ny, nz=1, tau=tau, collision=collision, wall_y=1, fext=(0, 0, F))
    nu = (tau - 0.5) / 3.0
    y = np.arange(ny) + 0.0
    exact = F / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
    u = np.zeros((3, 1, ny, 1))
    u[2, 0, :, 0] = exact
    df = o.init_fluid(None, u)
    o.run(df, steps)
    _, uu = o.moments(df)
    prev = uu[2, 0, :, 0].copy()
    o.run(df, 200)
    _, uu = o.moments(df)
    uz = uu[2, 0, :, 0]
    assert np.abs(uz - prev).max() < 1e-6 * np.abs(exact).max()  # steady
    return np.abs(uz - exact).max() / np.abs(exact).max()


def test_poiseuille_second_order_bgk():
    """Body-force driven flow between halfway bounce-back walls approaches the
    parabola u = F/(2 rho nu) (y + 1/2)(ny - 1/2 - y) at second order."""
    errs = [_poiseuille(n, 0.8, O.BGK, 40 * n * n) for n in (8, 16, 32)]
    assert errs[2] < 2e-3
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_poiseuille_exact_trt_magic():
    """With the two-rate collision at magic 3/16 the halfway bounce-back walls
    sit exactly half-way and the parabola is reproduced to round-off."""
    for n in (8, 16):
        assert _poiseuille(n, 0.8, O.TRT, 40 * n * n) < 1e-11


def test_stiff_chain_needs_multiple_time_steps():
    """Bonds with k = 30, m = 1 at h = 1 are beyond the stability limit of the
    Alg. 3 ordering; the multiple time-step split (Sec. 6, coupling outside)
    with n = 3 sub-steps per side is stable."""
    res = {}
    for n in (0, 3):
        pos, vel, bonds = I.chains(1, 20, (16, 16, 16), 1.0, 1e-3, 2)
        o = O.Oracle(nx=16, ny=16, nz=16, tau=0.6, collision=O.TRT, coupling=O.FC, gamma=2.0,
                     kernel=2, mts_n=n, bonds=bonds, bond_k=30.0, bond_r0=1.0)
        df = o.init_fluid()
        with np.errstate(all="ignore"):
            o.run(df, 30, pos, vel, np.ones(20))
        res[n] = np.abs(vel).max()
    assert not res[0] < 1.0
    assert res[3] < 1e-2


def test_ib_markers_in_accelerating_flow_follow_trapezoidal_rule():
    """A uniform flow accelerated by a body force has u(t) = u0 + F t / rho at
    step boundaries; the trapezoidal position update of Sec. 5.1, which uses
    u(t) and the physical u(t+h) after the second half force, moves markers
    along X0 + u0 t + F t^2 / 2 exactly."""
    T = I.icosphere(0, 2.5)
    F = np.array([2e-6, -1e-6, 3e-6])
    o = O.Oracle(nx=12, ny=12, nz=12, tau=0.7, coupling=O.IB, kernel=4, fext=F,
                 nshell=1, shell_template=T, tether_k=0.05)
    u0 = np.array([1e-3, 5e-4, -2e-4])
    df = o.init_fluid(None, np.broadcast_to(u0[:, None, None, None], (3,) + o.shape))
    X0 = np.array([6.1, 5.7, 6.4]) + T
    X = X0.copy()
    t = 9
    o.run(df, t, X)
    assert np.abs(X - (X0 + u0 * t + 0.5 * F * t * t)).max() < 1e-12


@pytest.mark.parametrize("kernel", [2, 4])
def test_one_cell_fluid_reduces_to_lumped_force_coupling(kernel):
    """On a one-site periodic lattice the fluid seen by a particle is a single
    cell of mass rho a^3, and each coupling half step is the Crank-Nicolson
    update of Sec. 5.2 with h/2: v - u contracts by
    (1 - (alpha+beta)/2)/(1 + (alpha+beta)/2) per half step while m v + rho u
    is conserved."""
    gamma, m = 1.7, 0.6
    o = O.Oracle(nx=1, ny=1, nz=1, tau=0.9, coupling=O.FC, gamma=gamma, kernel=kernel)
    u0 = np.array([1e-3, -4e-4, 2e-4])
    df = o.init_fluid(None, u0.reshape(3, 1, 1, 1))
    pos = np.array([[0.3, 0.6, 0.2]])
    v0 = np.array([[-2e-3, 1e-3, 5e-4]])
    vel = v0.copy()
    n = 7
    o.run(df, n, pos, vel, np.array([m]))
    rho = 1.0
    al, be = gamma * 0.5 / m, gamma * 0.5 / rho
    kappa = (1 - (al + be) / 2) / (1 + (al + be) / 2)
    _, u = o.moments(df)
    u = u.ravel()
    d0 = v0[0] - u0
    assert np.abs((vel[0] - u) - kappa ** (2 * n) * d0).max() < 1e-15
    assert np.abs((m * vel[0] + rho * u) - (m * v0[0] + rho * u0)).max() < 1e-17


def test_one_cell_fluid_modified_ebf_sticks():
    """Modified EBF (Eq. modified-ebf) on a one-cell fluid: no slip after every
    half step, and the common velocity is the momentum-weighted mean."""
    m = 0.35
    o = O.Oracle(nx=1, ny=1, nz=1, tau=0.9, coupling=O.EBF, gamma=0.8, kernel=3)
    u0 = np.array([1e-3, -4e-4, 2e-4])
    df = o.init_fluid(None, u0.reshape(3, 1, 1, 1))
    v0 = np.array([[-2e-3, 1e-3, 5e-4]])
    vel = v0.copy()
    o.run(df, 3, np.array([[0.5, 0.5, 0.5]]), vel, np.array([m]))
    _, u = o.moments(df)
    common = (m * v0[0] + 1.0 * u0) / (m + 1.0)
    assert np.abs(vel[0] - common).max() < 1e-17
    assert np.abs(u.ravel() - common).max() < 1e-17
