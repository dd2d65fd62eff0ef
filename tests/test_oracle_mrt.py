"""Pins of the general multiple-relaxation-time collision (Eq. mrt-coll with
a rate per moment group) in the oracle: the basis, its symmetry, the
two-rate special case, conservation, and the transport coefficients the
rates set: the shear viscosity from 1/tau alone, the bulk viscosity from the
bulk rate (sound attenuation)."""
import numpy as np
import pytest

import oracle as O
from paper_1406_2211_amd import inputs as I

RATES = (0.8, 1.3, 0.7, 1.9, 1.1)  # bulk, vector ghosts, pseudo-vector ghosts, scalar, tensor


def test_group_basis_is_orthogonal_with_integer_rows():
    E, b = O.group_basis()
    _, w, _ = O.lattice()
    G = (E * w) @ E.T
    assert np.abs(G - np.diag(b)).max() < 1e-15
    assert np.all(b > 0)
    assert np.array_equal(E, np.round(E))  # integer-valued polynomials of c


def test_two_rate_special_case():
    """Group rates (l+, l-, l-, l+, l+) are the two-rate collision."""
    tau, magic = 0.7, 3.0 / 16.0
    lp = 1.0 / tau
    lm = 1.0 / (0.5 + magic / (tau - 0.5))
    a = O.Oracle(nx=6, ny=5, nz=4, tau=tau, collision=O.TRT, magic=magic)
    b = O.Oracle(nx=6, ny=5, nz=4, tau=tau, collision=O.MRT, mrt_rates=(lp, lm, lm, lp, lp))
    df = a.stream(a.init_fluid(None, I.noise_velocity(a.shape, 3e-2, 1)))
    df = a.stream(a.collide(df))  # off equilibrium
    x, y = a.collide(df), b.collide(df)
    assert np.abs(x - y).max() < 1e-15 * max(1.0, np.abs(x).max()) * 10


def _perm(f):
    """Index permutation of the oracle's velocities under a map of vectors."""
    c, _, _ = O.lattice()
    fc = np.array([f(v) for v in c])
    return np.array([int(np.where((c == fc[i]).all(1))[0][0]) for i in range(19)])


@pytest.mark.parametrize("sym", ["rot_z", "swap_yz", "mirror_x"])
def test_collision_commutes_with_cubic_symmetry(sym):
    """With a rate per group the collision is isotropic: it commutes with the
    lattice symmetries.  A row relaxed at the rate of another group would
    break this for distinct rates."""
    f = {"rot_z": lambda v: np.array([-v[1], v[0], v[2]]),
         "swap_yz": lambda v: np.array([v[0], v[2], v[1]]),
         "mirror_x": lambda v: np.array([-v[0], v[1], v[2]])}[sym]
    P = _perm(f)
    o = O.Oracle(nx=1, ny=1, nz=1, tau=0.9, collision=O.MRT, mrt_rates=RATES)
    rng = np.random.default_rng(4)
    _, w, _ = O.lattice()
    site = w * (1.0 + 0.05 * rng.standard_normal(19)) - w
    a = o.collide_site(site)
    g = np.zeros(19)
    g[P] = site            # population of c_i moves to f(c_i)
    bb = o.collide_site(g)
    ref = np.zeros(19)
    ref[P] = a
    assert np.abs(bb - ref).max() < 1e-15


def test_mass_and_momentum_conserved():
    o = O.Oracle(nx=6, ny=7, nz=5, tau=0.8, collision=O.MRT, mrt_rates=RATES,
                 fext=(1e-6, 0.0, 2e-6))
    df = o.init_fluid(None, I.noise_velocity(o.shape, 1e-2, 2))
    t0 = o.totals(df)
    o.run(df, 10)
    t1 = o.totals(df)
    assert abs(t1[0] - t0[0]) < 1e-13
    assert np.abs(t1[1:4] - t0[1:4] - 10 * o.N * np.array([1e-6, 0.0, 2e-6])).max() < 1e-13


def _shear_decay(collision, rates, n, steps, tau=0.8):
    o = O.Oracle(nx=4, ny=n, nz=4, tau=tau, collision=collision, mrt_rates=rates)
    y = np.arange(n)
    u = np.zeros((3,) + o.shape)
    u[0] = 1e-4 * np.sin(2 * np.pi * y / n)[None, :, None]
    df = o.init_fluid(None, u)
    o.run(df, steps)
    _, uu = o.moments(df)
    amp = np.sum(uu[0, 0, :, 0] * np.sin(2 * np.pi * y / n)) * 2.0 / n
    return -np.log(amp / 1e-4) / steps


def test_shear_viscosity_set_by_tau_alone():
    """The shear modes relax at 1/tau whatever the other rates: the decay rate
    of a shear wave converges to nu k^2, nu = c_s^2 (tau - 1/2), at second
    order in k for the general rates as for BGK (the rates differ only in
    the O(k^2) corrections)."""
    errs = []
    for n in (16, 32, 64):
        k = 2 * np.pi / n
        g = _shear_decay(O.MRT, RATES, n=n, steps=int(0.4 * n * n))
        errs.append(abs(g / ((0.8 - 0.5) / 3.0 * k * k) - 1.0))
    assert errs[2] < 1e-4
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


@pytest.mark.parametrize("lb", [0.8, 1.6])
def test_bulk_rate_sets_sound_attenuation(lb):
    """A standing sound wave decays at Gamma = (k^2/2rho)(4 eta/3 + eta_b) with
    eta = rho c_s^2 (1/l_s - 1/2) and bulk viscosity eta_b = (2/3) rho c_s^2
    (1/l_b - 1/2) (the trace of the stress relaxes at the bulk rate)."""
    n, tau = 64, 0.8
    rates = (lb, 1.3, 0.7, 1.9, 1.1)
    o = O.Oracle(nx=n, ny=1, nz=1, tau=tau, collision=O.MRT, mrt_rates=rates)
    x = np.arange(n)
    k = 2 * np.pi / n
    A = 1e-5
    rho = 1.0 + A * np.cos(k * x)[None, None, :]
    df = o.init_fluid(rho, None)
    cs = np.sqrt(1.0 / 3.0)
    ts, es = [], []
    for t in range(0, 1200, 10):
        r, u = o.moments(df)
        ar = np.sum((r[0, 0] - 1.0) * np.cos(k * x)) * 2.0 / n
        au = np.sum(u[0, 0, 0] * np.sin(k * x)) * 2.0 / n
        ts.append(t)
        es.append(ar * ar + (au / cs) ** 2)
        o.run(df, 10)
    ts, es = np.array(ts), np.array(es)
    # energy decays as exp(-2 Gamma t) (oscillating by O(Gamma/omega) around it)
    slope = np.polyfit(ts, np.log(es), 1)[0]
    gam = -0.5 * slope
    cs2 = 1.0 / 3.0
    expect = 0.5 * k * k * (4.0 / 3.0 * cs2 * (1.0 / 1.25 - 0.5) + 2.0 / 3.0 * cs2 * (1.0 / lb - 0.5))
    assert abs(gam / expect - 1.0) < 0.03, (gam, expect)
