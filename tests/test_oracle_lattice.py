"""Pins of the oracle's local operators: lattice, equilibrium, force term,
collision (Sec. 2, Sec. 3.2-3.3 of the paper)."""
import itertools

import numpy as np
import pytest

import oracle as O

RNG = np.random.default_rng(7)


def _lat():
    c, w, opp = O.lattice()
    return c.astype(float), w, opp


def test_lattice_isotropy():
    """D3Q19 quadrature: weights sum to 1, second moment cs2 I with cs2 = 1/3,
    odd moments vanish, fourth moment cs4 (dd + dd + dd)."""
    c, w, opp = _lat()
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(w @ c).max() < 1e-16
    assert np.abs(np.einsum("i,ia,ib->ab", w, c, c) - np.eye(3) / 3).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, c, c, c)).max() < 1e-16
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.abs(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c) - iso).max() < 1e-15
    assert np.all(c[opp] == -c)


@pytest.mark.parametrize("trial", range(5))
def test_equilibrium_moments(trial):
    """sum f^eq = rho, sum f^eq c = rho u, sum f^eq c c = rho u u + rho cs2 I
    (the hydrodynamic moments of Sec. 2)."""
    c, w, _ = _lat()
    rho0 = 1.0
    rho = 1.0 + 0.05 * RNG.standard_normal()
    u = 0.05 * RNG.standard_normal(3)
    f = O.feq_dev(rho, rho0, u) + w * rho0
    assert abs(f.sum() - rho) < 1e-14
    assert np.abs(f @ c - rho * u).max() < 1e-15
    P = np.einsum("i,ia,ib->ab", f, c, c)
    assert np.abs(P - rho * np.outer(u, u) - rho / 3 * np.eye(3)).max() < 1e-15


@pytest.mark.parametrize("trial", range(5))
def test_force_term_moments(trial):
    """Eq. force-moments: sum G = 0, sum c G = F, sum c c G = F u + u F."""
    c, w, _ = _lat()
    u = 0.05 * RNG.standard_normal(3)
    F = 1e-3 * RNG.standard_normal(3)
    G = O.force_term(u, F)
    assert abs(G.sum()) < 1e-18
    assert np.abs(G @ c - F).max() < 1e-18
    P = np.einsum("i,ia,ib->ab", G, c, c)
    assert np.abs(P - np.outer(F, u) - np.outer(u, F)).max() < 1e-18


@pytest.mark.parametrize("trial", range(5))
def test_half_force_is_equilibrium_shift(trial):
    """A midpoint half force equals an equilibrium difference:
    (h/2) G(F, u + hF/4rho) = f^eq(rho, u + hF/2rho) - f^eq(rho, u), and two
    consecutive half forces equal one shift by hF/rho (Sec. 3.3)."""
    o = O.Oracle(nx=1, ny=1, nz=1, tau=0.8)
    rho = 1.0 + 0.01 * RNG.standard_normal()
    u = 0.02 * RNG.standard_normal(3)
    F = 1e-3 * RNG.standard_normal(3)
    neq = 1e-4 * RNG.standard_normal(19)
    neq -= neq.mean()  # keeps the stored state generic
    f = (O.feq_dev(rho, 1.0, u)).reshape(19, 1, 1, 1)
    # the oracle's F^1/2 with the constant body force F
    o2 = O.Oracle(nx=1, ny=1, nz=1, tau=0.8, fext=F)
    f1 = o2.force_half(f)
    expect = O.feq_dev(rho, 1.0, u + 0.5 * F / rho)
    assert np.abs(f1.ravel() - expect).max() < 2e-17
    f2 = o2.force_half(f1)
    expect2 = O.feq_dev(rho, 1.0, u + F / rho)
    assert np.abs(f2.ravel() - expect2).max() < 4e-17


def test_force_commutes_with_nonequilibrium():
    """F acts only on the equilibrium part (Sec. 3.3): f - f^eq is unchanged by
    F^1/2 (exactly, since the half force is an equilibrium shift)."""
    c, w, _ = _lat()
    rho = 1.02
    u = np.array([0.01, -0.02, 0.005])
    F = np.array([2e-4, 1e-4, -3e-4])
    neq = 1e-4 * RNG.standard_normal(19)
    # project out density and momentum so the moments stay those of f^eq
    M = np.vstack([np.ones(19), c.T])
    neq -= M.T @ np.linalg.solve(M @ M.T, M @ neq)
    f = O.feq_dev(rho, 1.0, u) + neq
    o = O.Oracle(nx=1, ny=1, nz=1, tau=0.8, fext=F)
    f1 = o.force_half(f.reshape(19, 1, 1, 1)).ravel()
    u1 = u + 0.5 * F / rho
    assert np.abs((f1 - O.feq_dev(rho, 1.0, u1)) - neq).max() < 1e-18


def test_mrt_basis_orthogonal_and_parity():
    c, w, _ = _lat()
    E, b = O.mrt_basis()
    G = E @ np.diag(w) @ E.T
    assert np.abs(G - np.diag(b)).max() < 1e-15
    assert np.all(b > 1e-3)
    assert np.allclose(E[0], 1.0) and np.allclose(E[1:4], c.T)
    _, _, opp = O.lattice()
    odd = [1, 2, 3] + list(range(10, 16))
    for k in range(19):
        sgn = -1.0 if k in odd else 1.0
        assert np.abs(E[k][opp] - sgn * E[k]).max() < 1e-15
    # ghost rows are w-orthogonal to every polynomial of degree <= 2 in c,
    # hence the ghost moments of the second-order equilibrium vanish
    f = O.feq_dev(1.03, 1.0, np.array([0.02, -0.01, 0.03]))
    m = E @ f
    assert np.abs(m[10:]).max() < 1e-17


def _trt_population(f, tau, magic, rho0=1.0):
    """Two-relaxation-time collision written in population space (an
    independent formulation of the moment-space collision)."""
    c, w, opp = _lat()
    rho = rho0 + f.sum()
    u = (f @ c) / rho
    cu = c @ u
    feq = w * (rho - rho0) + w * rho * (3 * cu + 4.5 * cu**2 - 1.5 * u @ u)
    neq = f - feq
    lp = 1.0 / tau
    lm = 1.0 / (0.5 + magic / (tau - 0.5))
    sym = 0.5 * (neq + neq[opp])
    anti = 0.5 * (neq - neq[opp])
    return feq + (1 - lp) * sym + (1 - lm) * anti


@pytest.mark.parametrize("tau", [0.55, 0.6, 0.8, 1.0, 1.7])
def test_mrt_with_two_rates_equals_trt(tau):
    """MRT collision in moment space (Eq. mrt-coll) with even/odd rates equals
    the two-relaxation-time collision in population space."""
    o = O.Oracle(nx=1, ny=1, nz=1, tau=tau, collision=O.TRT, magic=3.0 / 16.0)
    for _ in range(5):
        f = O.feq_dev(1.01, 1.0, 0.03 * RNG.standard_normal(3)) + 1e-4 * RNG.standard_normal(19)
        got = o.collide_site(f)
        exp = _trt_population(f, tau, 3.0 / 16.0)
        assert np.abs(got - exp).max() < 1e-16


@pytest.mark.parametrize("collision", [O.BGK, O.TRT])
def test_collision_conserves_and_keeps_equilibrium(collision):
    """C conserves rho and rho u and leaves f^eq invariant (C f^eq = 0, Sec. 3.2);
    BGK scales f - f^eq by 1 - 1/tau."""
    c, w, _ = _lat()
    tau = 0.7
    o = O.Oracle(nx=1, ny=1, nz=1, tau=tau, collision=collision)
    feq = O.feq_dev(1.02, 1.0, np.array([0.01, 0.02, -0.03]))
    assert np.abs(o.collide_site(feq) - feq).max() < 1e-16
    f = feq + 1e-4 * RNG.standard_normal(19)
    g = o.collide_site(f)
    assert abs(g.sum() - f.sum()) < 1e-15
    assert np.abs(g @ c - f @ c).max() < 1e-15


def test_rates():
    o = O.Oracle(nx=1, ny=1, nz=1, tau=0.6, collision=O.TRT, magic=3.0 / 16.0)
    lam = o.rates()
    assert abs(lam[4] - 1 / 0.6) < 1e-15
    # (1/lp - 1/2)(1/lm - 1/2) = magic
    assert abs((1 / lam[4] - 0.5) * (1 / lam[10] - 0.5) - 3.0 / 16.0) < 1e-15
    assert abs(lam[10] - 0.42105263157894735) < 1e-15


def test_stream_is_a_permutation_with_bounce_back():
    """S moves f_i by c_i (Sec. 3.1); with y walls the populations that would
    leave are reflected, so S is still a permutation of the stored values."""
    for wall in (0, 1):
        o = O.Oracle(nx=5, ny=4, nz=3, tau=0.8, wall_y=wall)
        f = RNG.standard_normal((19, 3, 4, 5))
        g = o.stream(f)
        assert np.allclose(np.sort(g.ravel()), np.sort(f.ravel()), rtol=0, atol=0)
        c, _, opp = O.lattice()
        for i in range(19):
            for z, y, x in itertools.product(range(3), range(4), range(5)):
                ys = y - c[i, 1]
                if wall and (ys < 0 or ys >= 4):
                    assert g[i, z, y, x] == f[opp[i], z, y, x]
                else:
                    assert g[i, z, y, x] == f[i, (z - c[i, 2]) % 3, ys % 4, (x - c[i, 0]) % 5]
