"""Temporal order of the coupled splitting (Sec. 5.1, Eq. IBM-scheme; Sec. 5.2,
Eq. fc-splitting): the symmetric sequences P^1/2 F^1/2 (C S) F^1/2 P^1/2 of
Alg. 2 and Alg. 3 are second order in h, the sequence P S C F that Sec. 5.1
contrasts them with is first order, and so is a misordered variant planted in
the oracle (``order=2``: the final P^1/2 of Alg. 3 moved before the second
coupling half; Alg. 2 without the position predictor).

Refinement in time at a fixed lattice spacing.  With a = 1 and a time step
h = 1/M in the units of the coarsest run, the run at level M takes lattice
parameters gamma/M, bond stiffness k/M^2, body force F/M^2, velocities v/M,
tau - 1/2 scaled by 1/M (fixed viscosity) and M times as many steps; positions
are unchanged and velocities are compared after multiplying back by M.

Two settings isolate the coupling from the lattice's own dependence on h:
  * force coupling in a one-site periodic lattice, where collision and
    streaming leave density and momentum alone and the step is a time
    integrator of Eq. fc-vel (plus the body force), compared with the matrix
    exponential of that linear system;
  * passive immersed-boundary markers (no intrinsic force, so they do not act
    on the fluid) in a slowly decaying two-dimensional flow, compared with a
    fourth-order Runge-Kutta integration of dX/dt = I[X]u through a cubic
    interpolation in time of the same run's velocity fields.

P, C and S act on disjoint parts of the state (positions, populations), so the
place of P^1/2 relative to the lattice update is immaterial; what the order
pins is its place relative to the coupling halves and the intrinsic forces."""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O

SECOND = (3.6, 4.4)
FIRST = (1.7, 2.6)


def _ratios(errs):
    e = np.asarray(errs)
    return e[:-1] / e[1:]


def _within(r, band):
    return bool(np.all((r > band[0]) & (r < band[1])))


# -- force coupling: one free particle in a one-site fluid -------------------

G1, M1, RHO1, T1 = 0.8, 1.5, 1.0, 12


def _single(level, order, F):
    o = O.Oracle(nx=1, ny=1, nz=1, tau=0.5 + 0.3 / level, coupling=O.FC, gamma=G1 / level,
                 kernel=2, fext=(F / level ** 2, 0.0, 0.0), rho0=RHO1, order=order)
    df = o.init_fluid(None, np.array([1e-3 / level, 0.0, 0.0]).reshape(3, 1, 1, 1))
    pos = np.array([[0.3, 0.4, 0.5]])
    vel = np.array([[-2e-3 / level, 0.0, 0.0]])
    o.run(df, T1 * level, pos, vel, np.array([M1]))
    _, u = o.moments(df)
    return vel[0, 0] * level, u[0].ravel()[0] * level, pos[0, 0]


def _single_exact(F):
    """v, u, x at T of m v' = -gamma (v - u), rho u' = gamma (v - u) + F, x' = v."""
    A = np.zeros((4, 4))
    A[0, :2] = [-G1 / M1, G1 / M1]
    A[1, :3] = [G1 / RHO1, -G1 / RHO1, F / RHO1]
    A[3, 0] = 1.0
    return expm(A * T1) @ np.array([-2e-3, 1e-3, 1.0, 0.3])


def _single_errors(order, F):
    ex = _single_exact(F)
    errs = []
    for level in (1, 2, 4, 8, 16):
        v, u, x = _single(level, order, F)
        dx = (x - ex[3] + 0.5) % 1.0 - 0.5
        errs.append(max(abs(v - ex[0]), abs(u - ex[1]), abs(dx)))
    return errs


@pytest.mark.parametrize("F", [0.0, 2e-3])
def test_force_coupling_one_particle_is_second_order(F):
    """Alg. 3 integrates particle, fluid and position at second order, also
    under a body force (which the fluid feels inside the implicit coupling
    solve); the P S C F sequence and the planted misordering converge at first
    order."""
    r = _ratios(_single_errors(0, F))
    assert _within(r, SECOND), r
    for order in (1, 2):
        r1 = _ratios(_single_errors(order, F))
        assert _within(r1, FIRST), (order, r1)


# -- force coupling: bonded pair, relative motion ----------------------------

G2, M2, K2, T2 = 0.8, 1.3, 2.5, 6


def _pair(level, order):
    """Heavy one-site fluid (rho0 = 1e6): beta -> 0, so the lumped implicit
    coupling of each particle is exact for the pair's relative motion, a damped
    oscillator whose spring acts at the drifted positions."""
    o = O.Oracle(nx=1, ny=1, nz=1, tau=0.5 + 0.3 / level, coupling=O.FC, gamma=G2 / level,
                 kernel=2, bonds=np.array([[0, 1]]), bond_k=K2 / level ** 2, bond_r0=0.0,
                 rho0=1e6, order=order)
    df = o.init_fluid()
    d0, w0 = 0.12, 0.01
    pos = np.array([[0.5 + d0 / 2, 0.4, 0.6], [0.5 - d0 / 2, 0.4, 0.6]])
    vel = np.array([[w0 / 2, 0.0, 0.0], [-w0 / 2, 0.0, 0.0]]) / level
    o.run(df, T2 * level, pos, vel, np.full(2, M2))
    d = pos[0, 0] - pos[1, 0]
    d -= np.round(d)
    return d, (vel[0, 0] - vel[1, 0]) * level


def _pair_errors(order):
    ex = expm(np.array([[0.0, 1.0], [-2 * K2 / M2, -G2 / M2]]) * T2) @ np.array([0.12, 0.01])
    errs = []
    for level in (4, 8, 16, 32):
        d, w = _pair(level, order)
        errs.append(max(abs(d - ex[0]), abs(w - ex[1])))
    return errs


def test_force_coupling_bonded_pair_is_second_order():
    """Drift halves around the coupling halves and F_int at the midpoint
    positions: the relative motion converges at second order.  Moving the final
    P^1/2 before the second coupling half (planted) or the P S C F sequence
    drops it to first order."""
    r = _ratios(_pair_errors(0))
    assert _within(r, SECOND), r
    for order in (1, 2):
        r1 = _ratios(_pair_errors(order))
        assert _within(r1, FIRST), (order, r1)


# -- immersed boundary: passive markers in a decaying flow -------------------

L, T3, U3 = 16, 24, 0.004
X0 = np.array([[3.3, 5.1, 0.2], [10.2, 2.7, 0.5], [7.7, 12.9, 0.1], [14.4, 8.8, 0.6]])


def _flow(U):
    """u_x = U sin(2 pi y / L), u_y = 0.7 U sin(2 pi x / L + 0.3): divergence
    free, so the markers cross both velocity gradients."""
    y = np.arange(L)[:, None]
    x = np.arange(L)[None, :]
    u = np.zeros((3, 1, L, L))
    u[0, 0] = U * np.sin(2 * np.pi * y / L) * np.ones((1, L))
    u[1, 0] = 0.7 * U * np.sin(2 * np.pi * x / L + 0.3) * np.ones((L, 1))
    return u


def _ib_run(level, order):
    tau = 0.5 + 0.3 / level
    df = O.Oracle(nx=L, ny=L, nz=1, tau=tau).init_fluid(None, _flow(U3 / level))
    # let the initial layer of the equilibrium start decay before the markers enter
    O.Oracle(nx=L, ny=L, nz=1, tau=tau).run(df, 12 * level)
    o = O.Oracle(nx=L, ny=L, nz=1, tau=tau, coupling=O.IB, kernel=4, order=order)
    X = X0.copy()
    us = [o.moments(df)[1].copy()]
    for _ in range(T3 * level):
        o.run(df, 1, X)
        us.append(o.moments(df)[1].copy())
    return X, us, o


def _lagrange(us, t):
    """Cubic interpolation in time through four neighbouring velocity fields."""
    n = len(us) - 1
    i0 = min(max(int(np.floor(t)) - 1, 0), n - 3)
    ts = np.arange(i0, i0 + 4)
    out = 0.0
    for j in range(4):
        w = np.prod([(t - ts[k]) / (ts[j] - ts[k]) for k in range(4) if k != j])
        out = out + w * us[ts[j]]
    return out


def _rk4_markers(us, o, sub=2):
    rho = np.ones(o.shape)

    def f(X, t):
        return o.interp(X, rho, _lagrange(us, t))[1]

    X, h = X0.copy(), 1.0 / sub
    for n in range((len(us) - 1) * sub):
        t = n * h
        k1 = f(X, t)
        k2 = f(X + 0.5 * h * k1, t + 0.5 * h)
        k3 = f(X + 0.5 * h * k2, t + 0.5 * h)
        k4 = f(X + h * k3, t + h)
        X = X + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return X


def _ib_errors(order):
    errs = []
    for level in (1, 2, 4, 8):
        X, us, o = _ib_run(level, order)
        d = X - _rk4_markers(us, o)
        d -= L * np.round(d / L)
        errs.append(np.abs(d).max())
    return errs


def test_immersed_boundary_markers_are_second_order():
    """Alg. 2's position update (predictor X~, trapezoidal quadrature of the
    interpolated velocity at X~) converges at second order to the markers'
    trajectory through the run's own flow; P S C F (X += h I[X(t)] u(t+h)) and
    the planted update without the predictor converge at first order."""
    r = _ratios(_ib_errors(0))
    assert _within(r, SECOND), r
    for order in (1, 2):
        r1 = _ratios(_ib_errors(order))
        assert _within(r1, FIRST), (order, r1)


def test_first_order_sequences_conserve_momentum():
    """The test-only orderings still exchange equal and opposite forces, so
    they differ from the splitting only in accuracy: fluid + particle momentum
    grows by exactly h F N per step."""
    F = np.array([1e-5, 0.0, -2e-5])
    for order in (1, 2):
        o = O.Oracle(nx=6, ny=6, nz=6, tau=0.7, coupling=O.FC, gamma=1.0, kernel=3,
                     fext=F, bonds=np.array([[0, 1]]), bond_k=0.3, bond_r0=1.0, order=order)
        df = o.init_fluid()
        pos = np.array([[1.2, 2.3, 3.1], [2.6, 2.0, 3.4]])
        vel = np.array([[1e-3, 0.0, -2e-3], [0.0, 1e-3, 0.0]])
        m = np.array([1.0, 1.5])
        t0 = o.totals(df, vel, m)
        o.run(df, 10, pos, vel, m)
        t1 = o.totals(df, vel, m)
        gain = (t1[1:4] + t1[4:7]) - (t0[1:4] + t0[4:7])
        assert np.abs(gain - 10 * o.N * F).max() < 1e-14, order
