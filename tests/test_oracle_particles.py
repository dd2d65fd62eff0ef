"""Pins of the oracle's particle side: delta functions (Appendix A),
interpolation/spreading (Sec. 5.1), the coupling forces (Sec. 5.2-5.3) and
the intrinsic forces."""
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1406_2211_amd import inputs as I

RNG = np.random.default_rng(11)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line.split())
    return rows


def _expr(s):
    return float(eval(s, {"sqrt": math.sqrt, "__builtins__": {}}))


def test_delta_values_golden():
    for k, r, v in _read_golden("delta_values.txt"):
        for sgn in (1.0, -1.0):
            assert abs(O.phi(int(k), sgn * float(r)) - _expr(v)) < 1e-15


@pytest.mark.parametrize("kernel", [2, 3, 4])
def test_delta_postulates(kernel):
    """Eqs. delta1-delta3: sum phi = 1, sum j phi = r, sum phi^2 = C."""
    Cs = {int(k): _expr(c) for k, c in _read_golden("kernel_sums.txt")}
    for r in np.concatenate([RNG.uniform(-3, 3, 200), [0.0, 0.5, 1.0, -1.5]]):
        js = np.arange(math.floor(r) - 3, math.floor(r) + 4)
        ph = np.array([O.phi(kernel, r - j) for j in js])
        assert abs(ph.sum() - 1.0) < 1e-14
        assert abs((js * ph).sum() - r) < 1e-13
        if kernel in Cs:
            assert abs((ph**2).sum() - Cs[kernel]) < 1e-14
        else:
            assert 0.5 - 1e-15 <= (ph**2).sum() <= 1.0 + 1e-15
        # Schwarz form, Eq. delta4
        r2 = r + RNG.uniform(-2, 2)
        ph2 = np.array([O.phi(kernel, r2 - j) for j in js])
        if kernel in Cs:
            assert abs((ph * ph2).sum()) <= Cs[kernel] + 1e-14


def _cfg(kernel, wall=0, n=(12, 10, 14)):
    return O.Oracle(nx=n[0], ny=n[1], nz=n[2], tau=0.8, kernel=kernel, wall_y=wall)


@pytest.mark.parametrize("kernel", [2, 3, 4])
def test_linear_fields_interpolate_exactly(kernel):
    """delta1 + delta2 make interpolation exact for linear fields (Appendix A)."""
    o = _cfg(kernel)
    z, y, x = np.meshgrid(np.arange(o.nz), np.arange(o.ny), np.arange(o.nx), indexing="ij")
    a = np.array([0.3, -0.2, 0.7])
    field = np.stack([1 + a[0] * x + a[1] * y, 2 - a[2] * z + 0 * x, 0.5 * y + 0.1 * z])
    rho = 1.0 + 0.01 * x
    pos = RNG.uniform(3, 7, size=(50, 3))  # away from the periodic seam
    rp, up = o.interp(pos, rho, field)
    X, Y, Z = pos.T
    assert np.abs(up[:, 0] - (1 + a[0] * X + a[1] * Y)).max() < 1e-12
    assert np.abs(up[:, 1] - (2 - a[2] * Z)).max() < 1e-12
    assert np.abs(up[:, 2] - (0.5 * Y + 0.1 * Z)).max() < 1e-12
    assert np.abs(rp - (1 + 0.01 * X)).max() < 1e-13


@pytest.mark.parametrize("kernel", [2, 3, 4])
def test_spread_conserves_force_and_torque(kernel):
    """Appendix A: total force and torque on the grid equal those of the
    Lagrangian forces; interpolation and spreading are adjoint."""
    o = _cfg(kernel)
    pos = RNG.uniform(3, 7, size=(30, 3))
    Fp = RNG.standard_normal((30, 3))
    Fg = o.spread(pos, Fp)
    assert np.abs(Fg.reshape(3, -1).sum(1) - Fp.sum(0)).max() < 1e-12
    z, y, x = np.meshgrid(np.arange(o.nz), np.arange(o.ny), np.arange(o.nx), indexing="ij")
    xs = np.stack([x, y, z]).reshape(3, -1)
    tg = np.cross(xs.T, Fg.reshape(3, -1).T).sum(0)
    assert np.abs(tg - np.cross(pos, Fp).sum(0)).max() < 1e-11
    u = RNG.standard_normal((3,) + o.shape)
    _, up = o.interp(pos, np.ones(o.shape), u)
    assert abs((Fg * u).sum() - (Fp * up).sum()) < 1e-11


def test_periodic_wrap_and_wall_truncation():
    o = _cfg(4)
    u = RNG.standard_normal((3,) + o.shape)
    rho = np.ones(o.shape)
    p = np.array([[0.3, 5.2, 13.6]])
    shift = p + np.array([[o.nx, 0, -o.nz]])
    assert np.allclose(o.interp(p, rho, u)[1], o.interp(shift, rho, u)[1], rtol=0, atol=1e-14)
    ow = _cfg(4, wall=1)
    # a marker within the kernel support of the wall loses the weight beyond it
    Fg = ow.spread(np.array([[5.0, 0.4, 6.0]]), np.array([[0.0, 0.0, 1.0]]))
    assert 0.0 < Fg[2].sum() < 1.0


# ---------------------------------------------------------------- coupling
def _lumped(gamma, m, rho, hh, v, u, Fint, kind):
    if kind == "fc":
        Fh = O.fc_force(gamma, m, rho, hh, v, u, Fint)
        v1 = v + hh / m * (Fh + Fint)
    else:
        Fh, v1 = O.ebf_update(gamma, m, rho, hh, v, u, Fint)
    u1 = u - hh / rho * Fh  # the one-cell fluid feels -F^h
    return Fh, v1, u1


@pytest.mark.parametrize("trial", range(6))
def test_force_coupling_matches_crank_nicolson(trial):
    """Eq. modified-force is the midpoint force consistent with the
    Crank-Nicolson updates of Eq. fc-cn: the v and u closed forms that follow
    it, and the slip recurrence."""
    gamma, m, rho, hh = RNG.uniform(0.2, 3.0), RNG.uniform(0.1, 5.0), RNG.uniform(0.9, 1.1), 0.5
    v, u, Fint = RNG.standard_normal(3), RNG.standard_normal(3), RNG.standard_normal(3)
    Fh, v1, u1 = _lumped(gamma, m, rho, hh, v, u, Fint, "fc")
    al, be = gamma * hh / m, gamma * hh / rho
    den = 1 + al / 2 + be / 2
    d = v - u
    assert np.allclose(v1, v - (al / gamma) / den * (gamma * d - (2 + be) / 2 * Fint), atol=1e-13)
    assert np.allclose(u1, u + (be / gamma) / den * (gamma * d + al / 2 * Fint), atol=1e-13)
    slip = (1 - al / 2 - be / 2) / den * d + al / den * Fint / gamma
    assert np.allclose(v1 - u1, slip, atol=1e-13)
    # momentum of particle + cell changes only by the intrinsic impulse
    assert np.allclose(m * v1 + rho * u1, m * v + rho * u + hh * Fint, atol=1e-13)


def test_gamma_condition_gives_the_slip_formula():
    """Eq. gamma-cond: gamma = (rho a^3/h) 2/(1 + rho a^3/m) removes the
    velocity-difference term and leaves the slip (h/2m) F_int (Eq. slip)."""
    for m in (0.3, 1.0, 4.0):
        rho, hh = 1.0, 0.5
        gamma = rho / hh * 2.0 / (1.0 + rho / m)
        v, u, Fint = RNG.standard_normal(3), RNG.standard_normal(3), RNG.standard_normal(3)
        _, v1, u1 = _lumped(gamma, m, rho, hh, v, u, Fint, "fc")
        assert np.allclose(v1 - u1, hh / (2 * m) * Fint, atol=1e-13)


@pytest.mark.parametrize("m", [1e-9, 1e-3, 0.5, 1.0, 7.0, 1e6])
def test_modified_ebf_no_slip_and_immersion_number(m):
    """Eq. modified-ebf gives v' = u' for any mass; a fraction
    r = 1/(1 + m/(rho a^3)) of F_int reaches the fluid (Eq. immersion)."""
    gamma, rho, hh = 1.3, 1.05, 0.5
    v, u, Fint = RNG.standard_normal(3), RNG.standard_normal(3), RNG.standard_normal(3)
    Fh, v1, u1 = _lumped(gamma, m, rho, hh, v, u, Fint, "ebf")
    scale = 1 + np.abs(u1).max()
    assert np.abs(v1 - u1).max() < 1e-12 * scale * max(1.0, hh / m * 1e-6)
    # with v = u the fluid receives exactly r F_int
    Fh2, _, _ = _lumped(gamma, m, rho, hh, u, u, Fint, "ebf")
    r = 1.0 / (1.0 + m / rho)
    assert np.allclose(-Fh2, r * Fint, rtol=1e-12, atol=1e-300)


def test_zero_mass_limit_is_immersed_boundary():
    """m -> 0 in the modified EBF: the fluid force tends to +F_int (IB) with an
    O(m) error and the particle moves with the fluid (Sec. 5.3)."""
    gamma, rho, hh = 1.0, 1.0, 0.5
    v, u, Fint = RNG.standard_normal(3), RNG.standard_normal(3), RNG.standard_normal(3)
    errs = []
    for m in (1e-2, 1e-4, 1e-6):
        Fh, v1, u1 = _lumped(gamma, m, rho, hh, v, u, Fint, "ebf")
        errs.append(np.abs(-Fh - Fint).max())
        assert np.allclose(v1, u1, atol=1e-10)
    assert errs[1] < errs[0] * 2e-2 and errs[2] < errs[1] * 2e-2


# ---------------------------------------------------------------- intrinsic forces
def test_fene_bond_at_maximum_extension_is_nan():
    """FENE's energy -k r0^2/2 ln(1 - |d|^2/r0^2) is infinite from |d| = r0 on:
    the force of such a bond is NaN (not the sign-flipped value of the
    formula), the bond just inside r0 is finite and pulls the pair together."""
    o = O.Oracle(nx=10, ny=10, nz=10, tau=0.8, bonds=np.array([[0, 1], [2, 3]]), bond_k=1.0,
                 bond_r0=1.5, bond_type=O.FENE)
    pos = np.array([[1.0, 1.0, 1.0], [2.4, 1.0, 1.0], [5.0, 5.0, 5.0], [6.6, 5.0, 5.0]])
    F = o.bond_forces(pos)
    assert np.all(np.isfinite(F[:2])) and F[0, 0] > 0 and F[1, 0] < 0
    assert np.all(np.isnan(F[2:, 0]))


@pytest.mark.parametrize("btype", [O.HARMONIC, O.FENE])
def test_bond_forces_are_minus_energy_gradient(btype):
    k, r0 = 30.0, (1.0 if btype == O.HARMONIC else 1.5)
    pos, _, bonds = I.chains(3, 6, (20, 20, 20), 0.9, 0.0, 5)
    o = O.Oracle(nx=20, ny=20, nz=20, tau=0.8, bonds=bonds, bond_k=k, bond_r0=r0, bond_type=btype)

    def energy(p):
        d = p[bonds[:, 1]] - p[bonds[:, 0]]
        d -= 20 * np.round(d / 20)
        L = np.linalg.norm(d, axis=1)
        if btype == O.HARMONIC:
            return 0.5 * k * ((L - r0) ** 2).sum()
        return (-0.5 * k * r0**2 * np.log(1 - (L / r0) ** 2)).sum()

    F = o.bond_forces(pos)
    eps = 1e-6
    for p in range(pos.shape[0]):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[p, a] += eps
            pm[p, a] -= eps
            g = (energy(pp) - energy(pm)) / (2 * eps)
            assert abs(F[p, a] + g) < 1e-6 * (1 + abs(g))
    assert np.abs(F.sum(0)).max() < 1e-12


def _kabsch_svd(P, T):
    """Least-squares rotation R with P ~ R T (SVD solution)."""
    H = T.T @ P
    U, S, Vt = np.linalg.svd(H)
    d = np.sign(np.linalg.det(Vt.T @ U.T))
    D = np.diag([1, 1, d])
    return Vt.T @ D @ U.T


def _rot(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def test_tether_forces_rigid_template():
    """Shell tethers: zero for any rigid motion of the template, total force and
    torque zero for any deformation (least-squares rotation), and the rotation
    agrees with the SVD solution of the same fit."""
    T = I.icosphere(2, 5.0)
    M = T.shape[0]
    o = O.Oracle(nx=40, ny=40, nz=40, tau=0.8, nshell=2, shell_template=T, tether_k=0.05)
    R1, R2 = _rot([1, 2, 3], 0.7), _rot([-1, 0.5, 0.2], 2.5)
    c1, c2 = np.array([10.0, 12, 13]), np.array([39.5, 20, 0.5])  # second shell straddles the seam
    pos = np.vstack([c1 + T @ R1.T, c2 + T @ R2.T])
    pos = pos % 40.0
    F, rot = o.tether_forces(pos, want_rot=True)
    assert np.abs(F).max() < 1e-13
    assert np.abs(rot[0] - R1).max() < 1e-12 and np.abs(rot[1] - R2).max() < 1e-12
    defo = pos + 0.3 * RNG.standard_normal(pos.shape)
    F, rot = o.tether_forces(defo, want_rot=True)
    for s in range(2):
        Fs = F[s * M:(s + 1) * M]
        Ps = defo[s * M:(s + 1) * M].copy()
        Ps = Ps[0] + ((Ps - Ps[0] + 20) % 40 - 20)
        cen = Ps.mean(0)
        assert np.abs(Fs.sum(0)).max() < 1e-12
        assert np.abs(np.cross(Ps - cen, Fs).sum(0)).max() < 1e-11
        Rs = _kabsch_svd(Ps - cen, T)
        assert np.abs(rot[s] - Rs).max() < 1e-10
        assert np.allclose(Fs, -0.05 * (Ps - cen - T @ Rs.T), atol=1e-12)
