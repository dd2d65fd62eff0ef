"""GPU parity of multiple time stepping with the coupling inside every
sub-step (Eq. multistep) against the FP64 oracle, which runs the 2n coupled
sub-steps one after the other with the lattice force applied after each.
Tolerances as in the other parity tests: FP64 storage 1e-12 (for stiff
bonds 20 times the oracle's own one-ulp sensitivity, if larger), FP32
storage 1e-5."""
import numpy as np
import pytest

from paper_1406_2211_amd import inputs as I
from parity import Case, compare, run_gpu, run_oracle, ulp_sensitivity

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _chains(name, n, nch, nb, steps, mts, k=2.0, storage=0, coupling=1, kernel=2, **kw):
    pos, vel, bonds = I.chains(nch, nb, (n, n, n), 1.0, 1e-3, 2)
    c = Case(name=name, nx=n, ny=n, nz=n, tau=kw.pop("tau", 0.7), steps=steps, collision=1,
             coupling=coupling, gamma=2.0, kernel=kernel, storage=storage, mts=mts,
             u_noise=1e-4, pos=pos, vel=vel, mass=np.full(len(pos), 0.9), bonds=bonds,
             bond_k=k, bond_r0=1.0, **kw)
    c.extra["mts_inside"] = 1
    return c


def _check(c, tol):
    o = run_oracle(c)
    sens = ulp_sensitivity(c, o) if c.bonds is not None else 0.0
    return compare(c, run_gpu(c), o, tol, sens=sens)


@pytest.mark.parametrize("n", [1, 3, 7])
def test_soft_chains_fc_fp64(n):
    """n = 7: six sub-steps per side write fields of their own, more than are
    held before a fold, so each side folds twice."""
    _check(_chains(f"in_soft_n{n}", 24, 2, 12, 30, n), TOL64)


def test_ebf_chains_phi3_body_force_walls_fp64():
    c = _chains("in_ebf", 20, 2, 8, 25, 2, coupling=2, kernel=3, fext=(1e-6, 0.0, -2e-6))
    c.wall_y = 1
    _check(c, TOL64)


def test_stiff_chains_fp64():
    """The bond stiffness of the force-coupling workload (k = 30, m = 1)."""
    c = _chains("in_stiff", 32, 4, 20, 30, 5, k=30.0, tau=0.6)
    c.mass = np.ones(len(c.pos))
    c.u_noise = 0.0
    _check(c, TOL64)


def test_free_particles_body_force_comoving_phi4_fp64():
    """No intrinsic forces: the first drift of each sub-step is folded into the
    coupling launch; the body force enters the fluid velocity seen by each
    sub-step in pieces of dt; comoving storage frame."""
    pos = I.uniform_positions(40, (20, 20, 20), 8)
    c = Case(name="in_free", nx=20, ny=20, nz=20, tau=0.8, steps=30, fext=(3e-6, 0.0, 1e-6),
             coupling=1, gamma=1.4, kernel=4, mts=4, pos=pos,
             vel=np.random.default_rng(8).normal(0, 1e-3, (40, 3)), mass=np.full(40, 0.5))
    c.extra.update(mts_inside=1, comoving=1)
    _check(c, TOL64)


def test_step_calls_split_into_chunks():
    """The moment cache carries over between lb_step calls (reads in between)."""
    c = _chains("in_chunks", 24, 2, 12, 30, 3)
    c.extra["chunks"] = [1, 7, 2, 20]
    _check(c, TOL64)


def test_one_site_lattice_pair():
    """A bonded pair in a one-site fluid (both particles share every stencil node)."""
    c = Case(name="in_one_site", nx=1, ny=1, nz=1, tau=0.8, steps=12, coupling=1, gamma=0.9,
             kernel=2, mts=3, u_noise=0.0, pos=np.array([[0.56, 0.4, 0.6], [0.44, 0.4, 0.6]]),
             vel=np.array([[6e-3, 0.0, 0.0], [-4e-3, 0.0, 0.0]]), mass=np.full(2, 1.3),
             bonds=np.array([[0, 1]]), bond_k=2.5, bond_r0=0.0)
    c.extra["mts_inside"] = 1
    _check(c, TOL64)


def test_soft_chains_fc_fp32():
    _check(_chains("in_soft32", 32, 3, 16, 60, 3, storage=1), TOL32)


def test_many_substeps_phi4_fp32():
    """Ten sub-steps per side (three folds each), 4-point kernel, FP32."""
    _check(_chains("in_many32", 24, 2, 10, 20, 10, storage=1, kernel=4), TOL32)


def test_crossing_chains_row_mask_fp64():
    """Two chains laid side by side half a site apart, so beads of different
    chains (far apart in index) share stencil nodes; 64-site rows, so the
    force mask is kept as one word per row and the fold walks that layout;
    n = 6 puts five sub-steps per side into fields of their own, one more
    than are held before a fold."""
    nb = 20
    x = 20.3 + np.arange(nb, dtype=np.float64)
    a = np.stack([x, np.full(nb, 7.2), np.full(nb, 8.4)], axis=1)
    b = np.stack([x[::-1] + 0.45, np.full(nb, 7.7), np.full(nb, 8.9)], axis=1)
    pos = np.vstack([a, b])
    idx = np.arange(2 * nb).reshape(2, nb)
    bonds = np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], axis=1).astype(np.int32)
    vel = np.random.default_rng(5).normal(0.0, 1e-3, pos.shape)
    c = Case(name="in_cross_rows", nx=64, ny=16, nz=16, tau=0.7, steps=20, collision=1,
             coupling=1, gamma=2.0, kernel=2, storage=0, mts=6, u_noise=1e-4, pos=pos, vel=vel,
             mass=np.full(len(pos), 0.9), bonds=bonds, bond_k=2.0, bond_r0=1.0)
    c.extra["mts_inside"] = 1
    _check(c, TOL64)


def test_benchmark_chains_at_64_cubed_fp64():
    """The coupling-inside form of the force-coupling workload at a reduced
    size: 64^3 two-rate MRT, tau = 0.6, 10 chains of 100 beads (k = 30, m = 1),
    n = 5 sub-steps per side, 40 steps, against the oracle (bound: 1e-12 or 20x
    the oracle's one-ulp sensitivity of these stiff chains)."""
    pos, vel, bonds = I.chains(10, 100, (64, 64, 64), 1.0, 1e-3, 2)
    c = Case(name="in_c2_64", nx=64, ny=64, nz=64, tau=0.6, steps=40, collision=1, coupling=1,
             gamma=2.0, kernel=2, storage=0, mts=5, u_noise=0.0, pos=pos, vel=vel,
             mass=np.ones(len(pos)), bonds=bonds, bond_k=30.0, bond_r0=1.0)
    c.extra["mts_inside"] = 1
    _check(c, TOL64)
