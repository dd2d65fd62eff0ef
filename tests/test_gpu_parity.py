"""GPU parity: the HIP library (called through its C ABI) against the FP64 CPU
oracle on the same seeded inputs.  Tolerances (max norm, relative to the
oracle's largest magnitude): FP64 storage 1e-12, FP32 storage 1e-5."""
import numpy as np
import pytest

from paper_1406_2211_amd import inputs as I
from parity import Case, compare, run_gpu, run_oracle, ulp_sensitivity

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _chains_case(name, n, nchains, nbeads, steps, storage, mts=5, seed=2, k=30.0):
    pos, vel, bonds = I.chains(nchains, nbeads, (n, n, n), 1.0, 1e-3, seed)
    return Case(name=name, nx=n, ny=n, nz=n, tau=0.6, steps=steps, collision=1, coupling=1,
                gamma=2.0, kernel=2, storage=storage, mts=mts, u_noise=0.0, pos=pos, vel=vel,
                mass=np.ones(len(pos)), bonds=bonds, bond_k=k, bond_r0=1.0)


def _c1_case(n, steps, storage=0, seed=1):
    pos = I.uniform_positions(1, (n, n, n), seed)
    return Case(name=f"c1_{n}_{steps}_s{storage}", nx=n, ny=n, nz=n, tau=0.8, steps=steps,
                fext=(1e-6, 0.0, 0.0), coupling=1, gamma=1.0, kernel=2, storage=storage,
                pos=pos, vel=np.zeros((1, 3)), mass=np.ones(1), seed=seed)


def _ib_case(name, kernel, storage=0, steps=30):
    T = I.icosphere(1, 4.0)
    box = (24, 24, 32)
    cen = I.shell_centres(2, 4.0, box, True, 2.0, 3.0, seed=3)
    X = np.vstack([c + T for c in cen])
    X = X + 0.15 * np.random.default_rng(5).standard_normal(X.shape)
    return Case(name=name, nx=24, ny=24, nz=32, tau=0.8, steps=steps, wall_y=1,
                fext=(0.0, 0.0, 1e-6), coupling=3, kernel=kernel, storage=storage, u_noise=0.0,
                pos=X, nshell=2, template=T, tether_k=0.05)


def check(c, tol, ptol=None, conditioned=False, progress=None):
    """conditioned=True: the trajectory is ill-conditioned (stiff bonds), so the
    bound is raised to 20x the oracle's own one-ulp sensitivity if larger.
    progress: see run_oracle."""
    o = run_oracle(c, progress)
    sens = ulp_sensitivity(c, o, progress) if conditioned else 0.0
    g = run_gpu(c)
    return compare(c, g, o, tol, ptol, sens=sens)


# ------------------------------------------------------------------- FP64
def test_c1_small_fp64():
    check(_c1_case(16, 60), TOL64)


def test_c1_full_fp64():
    """The plain-method configuration at full size: 32^3, 500 steps."""
    check(_c1_case(32, 500), TOL64)


def test_rest_state_stays_exactly_zero():
    c = Case(name="rest", nx=20, ny=6, nz=5, tau=0.7, steps=25, collision=1, wall_y=1,
             coupling=1, gamma=1.0, u_noise=0.0, pos=np.array([[3.2, 2.5, 1.1]]),
             vel=np.zeros((1, 3)), mass=np.ones(1))
    g = run_gpu(c)
    assert np.all(g["df"] == 0.0) and np.all(g["vel"] == 0.0)


def test_ragged_walls_trt_ebf_bonds_phi3():
    """nx = 70 (one full 64-site row word and a ragged tail), y walls, TRT,
    modified EBF with a bonded chain, 3-point kernel, body force."""
    pos = np.array([[10.2, 2.1, 1.3], [11.0, 2.4, 1.6], [11.8, 2.2, 2.1], [68.9, 1.9, 0.4]])
    c = Case(name="ragged", nx=70, ny=5, nz=3, tau=0.66, steps=40, wall_y=1,
             fext=(1e-6, 0.0, 2e-6), collision=1, coupling=2, gamma=0.7, kernel=3,
             pos=pos, vel=1e-3 * np.random.default_rng(9).standard_normal((4, 3)),
             mass=np.array([0.5, 1.0, 2.0, 0.3]), bonds=np.array([[0, 1], [1, 2]]),
             bond_k=0.3, bond_r0=0.9)
    check(c, TOL64)


def test_one_site_lattice_fc():
    """Degenerate 1x1x1 periodic lattice: the fluid is one cell."""
    c = Case(name="one_site", nx=1, ny=1, nz=1, tau=0.9, steps=7, coupling=1, gamma=1.7,
             kernel=4, pos=np.array([[0.3, 0.6, 0.2]]), vel=np.array([[-2e-3, 1e-3, 5e-4]]),
             mass=np.array([0.6]))
    check(c, TOL64)


def test_thin_box_no_particles():
    c = Case(name="thin", nx=1, ny=8, nz=6, tau=0.55, steps=30, fext=(3e-6, 1e-6, 0.0),
             collision=1)
    check(c, TOL64)


def test_particles_at_periodic_seam_phi4():
    pos = np.array([[19.995, 0.002, 7.0], [0.001, 11.999, 19.9999], [10.0, 10.0, 10.0]])
    c = Case(name="seam", nx=20, ny=12, nz=20, tau=0.8, steps=30, coupling=1, gamma=1.2,
             kernel=4, pos=pos, vel=np.array([[3e-3, -2e-3, 1e-3], [-1e-3, 2e-3, 4e-3],
                                              [0.0, 0.0, 0.0]]), mass=np.ones(3))
    check(c, TOL64)


@pytest.mark.parametrize("kernel,coupling", [(2, 1), (3, 2), (4, 1)])
def test_moment_cache_zero_weight_nodes_and_cell_crossings(kernel, coupling):
    """The second coupling half caches the moments it gathers; the next first
    half reuses them while a particle's first stencil node is unchanged.
    Particle 0 sits exactly on a zero-weight node boundary along x at the
    first midpoint (so one node of its cached stencil has zero weight, and a
    nonzero weight one step later); particle 1 crosses cells every few steps
    (cache misses); particle 2 is slow."""
    xs = 10.0 if kernel != 3 else 10.5  # phi2/phi4: integer; phi3: half-integer
    pos = np.array([[xs - 0.125, 6.3, 9.7], [3.2, 12.9, 4.4], [8.1, 2.2, 13.6]])
    vel = np.array([[0.25, 0.0, 0.0], [0.35, -0.3, 0.2], [1e-3, -2e-3, 3e-3]])
    c = Case(name=f"mcache_k{kernel}", nx=16, ny=16, nz=16, tau=0.75, steps=25,
             coupling=coupling, gamma=0.7, kernel=kernel, pos=pos, vel=vel, mass=np.ones(3),
             u_noise=1e-3, seed=8)
    check(c, TOL64)


@pytest.mark.parametrize("which", ["ib_tiled", "mts", "alg3"])
def test_step_calls_split_into_chunks(which):
    """lb_step(n) ends at a step boundary: a run split into several calls (with
    reads in between) matches the oracle run of the total step count.  Covers
    the deferred final advection of the tiled IB path, the bond sub-steps on
    the auxiliary stream, and the coupling moment cache across calls."""
    if which == "ib_tiled":
        c = _ib_case("chunks_ib", 4, steps=20)
    elif which == "mts":
        pos, vel, bonds = I.chains(2, 8, (20, 20, 20), 1.0, 2e-2, 6)
        c = Case(name="chunks_mts", nx=20, ny=20, nz=20, tau=0.7, steps=20, collision=1,
                 coupling=1, gamma=1.0, kernel=2, storage=0, mts=3, u_noise=1e-3, pos=pos,
                 vel=vel, mass=np.full(len(pos), 2.0), bonds=bonds, bond_k=0.02, bond_r0=1.0)
    else:
        pos = np.array([[3.2, 12.9, 4.4], [8.1, 2.2, 13.6]])
        c = Case(name="chunks_alg3", nx=16, ny=16, nz=16, tau=0.75, steps=20, coupling=1,
                 gamma=0.7, kernel=2, pos=pos, vel=np.array([[0.2, -0.1, 0.05], [1e-3, 0, 0]]),
                 mass=np.ones(2), u_noise=1e-3, seed=8)
    c.extra["chunks"] = [1, 3, 5, 2, 9]
    check(c, TOL64)


def test_mts_stiff_chains_fp64():
    """The bead-spring parameters of the force-coupling workload (k = 30):
    ill-conditioned, so the bound follows the oracle's one-ulp sensitivity."""
    check(_chains_case("mts64", 24, 3, 10, 30, storage=0), TOL64, conditioned=True)


def test_mts_soft_chains_fp64_strict():
    """Multiple time stepping on a well-conditioned chain (soft bonds, faster
    beads): the plain 1e-12 bound applies."""
    pos, vel, bonds = I.chains(2, 8, (20, 20, 20), 1.0, 2e-2, 6)
    c = Case(name="mts_soft", nx=20, ny=20, nz=20, tau=0.7, steps=8, collision=1, coupling=2,
             gamma=1.0, kernel=3, storage=0, mts=3, u_noise=1e-3, pos=pos, vel=vel,
             mass=np.full(len(pos), 2.0), bonds=bonds, bond_k=0.02, bond_r0=1.0)
    check(c, TOL64)


@pytest.mark.parametrize("nx,walls", [(128, 0), (320, 1)])
def test_mts_bond_substeps_inside_the_lattice_launch_fp64(nx, walls):
    """Rows of 128 or more sites use the row-mapped pass, whose first z slab of
    workgroups then runs the bond sub-steps of the multiple time-step split
    (a bond group of 128 particles fits a workgroup); 320 sites make two row
    chunks (256 and a ragged 64), and y walls select the other pass variant.
    Soft bonds keep the trajectory well conditioned, so the plain 1e-12 bound
    applies."""
    rng = np.random.default_rng(11)
    pos = np.array([[5.0 + 40.0 * c + 0.95 * k, 5.0 + 3.0 * c, 6.0] for c in range(3)
                    for k in range(12)]) + rng.uniform(-0.2, 0.2, (36, 3))
    vel = rng.normal(0.0, 2e-2, (36, 3))
    bonds = np.array([[12 * c + k, 12 * c + k + 1] for c in range(3) for k in range(11)])
    c = Case(name=f"mts_row{nx}", nx=nx, ny=16, nz=12, tau=0.7, steps=10, collision=1,
             coupling=1, gamma=1.0, kernel=2, storage=0, mts=3, u_noise=1e-3, pos=pos, vel=vel,
             mass=np.full(len(pos), 2.0), bonds=bonds, bond_k=0.02, bond_r0=1.0, wall_y=walls)
    check(c, TOL64)


def _soft_alg3_case(name="alg3", steps=25):
    pos, vel, bonds = I.chains(2, 8, (20, 20, 20), 1.0, 2e-2, 8)
    return Case(name=name, nx=20, ny=20, nz=20, tau=0.6, steps=steps, collision=1, coupling=1,
                gamma=2.0, kernel=2, storage=0, mts=0, u_noise=1e-3, pos=pos, vel=vel,
                mass=np.full(len(pos), 2.0), bonds=bonds, bond_k=0.02, bond_r0=1.0)


def test_alg3_soft_chain_fp64():
    check(_soft_alg3_case(), TOL64)


@pytest.mark.parametrize("mts", [0, 3])
def test_fene_soft_chain_fp64(mts):
    """FENE bonds (maximum extension r0 = 2, bonds start at 1 and stay below
    1.05) against the oracle at the strict bound: in the Alg. 3 ordering, where
    the bond groups drift and evaluate F_int in one launch, and with the
    multiple time-step split, whose sub-steps run in the lattice launch."""
    pos, vel, bonds = I.chains(2, 8, (20, 20, 20), 1.0, 1e-2, 8)
    c = Case(name=f"fene_mts{mts}", nx=20, ny=20, nz=20, tau=0.6, steps=25, collision=1,
             coupling=1, gamma=2.0, kernel=2, storage=0, mts=mts, u_noise=1e-3, pos=pos,
             vel=vel, mass=np.full(len(pos), 2.0), bonds=bonds, bond_k=0.02, bond_r0=2.0,
             bond_type=1)
    o = run_oracle(c)
    d = o["pos"][bonds[:, 1]] - o["pos"][bonds[:, 0]]
    d -= 20 * np.round(d / 20)
    assert np.linalg.norm(d, axis=1).max() < 1.1  # far from the maximum extension
    compare(c, run_gpu(c), o, TOL64)


@pytest.mark.parametrize("kernel", [2, 4])
def test_ib_shells_fp64(kernel):
    check(_ib_case(f"ib_phi{kernel}", kernel), TOL64)


def test_empty_particle_set():
    c = Case(name="empty", nx=16, ny=16, nz=16, tau=0.7, steps=20, coupling=1, gamma=1.0,
             fext=(0.0, 1e-6, 0.0))
    check(c, TOL64)


def test_full_size_force_coupling_fp64(capsys):
    """The benchmark workload at full size with FP64 storage (the reference of
    the precision study): 256^3 two-rate MRT, 10^4 bonded particles with the
    multiple time-step split, 100 steps against the oracle.  The stiff bonds
    make the trajectory ill-conditioned, so the bound follows the oracle's own
    one-ulp sensitivity where that exceeds 1e-12.  The two oracle runs take
    minutes: their progress goes to the terminal past the output capture."""
    def progress(msg):
        with capsys.disabled():
            print(msg, flush=True)

    c = _chains_case("c2_full_fp64", 256, 100, 100, 100, storage=0)
    check(c, TOL64, conditioned=True, progress=progress)


# ------------------------------------------------------------------- FP32
# FP32 storage rounds every stored population once per step (2^-24 of
# |f - w rho0|).  In a nearly uniform flow this rounding is correlated across
# sites and the velocity error grows linearly with the step count; the bound
# for a run of n steps is therefore max(1e-5, FP32_PER_STEP * n) of the
# oracle's largest velocity.
FP32_PER_STEP = 2.5e-8


def test_c1_fp32_full():
    """The plain-method case at its full length (32^3, 500 steps) with FP32
    storage: about 2.2e-8 of max|u| per step of correlated rounding, so the
    step-dependent bound applies."""
    check(_c1_case(32, 500, storage=1), max(TOL32, FP32_PER_STEP * 500))


def test_c1_fp32_full_comoving():
    """The same run with the populations stored in the comoving frame (an exact
    change of variables, pinned in FP64).  The frame takes the uniform flow out
    of the stored values but not out of the FP32 arithmetic of the pass, which
    still forms the equilibrium at the full velocity: the error is the same
    (1.12e-5 against 1.14e-5 at 500 steps), so the same step-dependent bound
    applies."""
    c = _c1_case(32, 500, storage=1)
    c.extra["comoving"] = 1
    check(c, max(TOL32, FP32_PER_STEP * 500))


def test_full_size_force_coupling_fp32_vs_fp64_1000_steps():
    """The benchmark workload for its full 1000 steps: the FP32-storage
    velocity field against the FP64-storage run on the GPU (itself pinned to
    the oracle above), relative to the field's current largest velocity, within
    the step-dependent FP32 bound."""
    g64 = run_gpu(_chains_case("c2_1000_fp64", 256, 100, 100, 1000, storage=0))
    g32 = run_gpu(_chains_case("c2_1000_fp32", 256, 100, 100, 1000, storage=1))
    e = np.abs(g32["u"] - g64["u"]).max() / np.abs(g64["u"]).max()
    print(f"[parity] c2 1000 steps FP32 vs FP64: u={e:.3e}", flush=True)
    assert e <= FP32_PER_STEP * 1000


def test_full_size_force_coupling_fp32():
    """The benchmark configuration at full size, in the launch configuration
    the benchmark times: 256^3 two-rate MRT, FP32 storage, 10^4 bonded
    particles with the multiple time-step split; every output compared with
    the oracle after 3 steps."""
    c = _chains_case("c2_full", 256, 100, 100, 3, storage=1)
    check(c, TOL32)


def test_mts_chains_fp32():
    check(_chains_case("mts32", 48, 2, 20, 100, storage=1), TOL32)


def test_ib_shells_fp32():
    check(_ib_case("ib32", 4, storage=1), TOL32)


@pytest.mark.parametrize("kernel", [2, 4])
def test_ib_shells_carried_across_nodes_fp64(kernel):
    """Shells carried by a uniform flow of 0.05 sites per step: each step some
    markers' stencils move onto nodes the previous spread did not flag, so the
    interpolation lists them and the shells' workgroups redo them in the
    tether-force launch before the forces are taken."""
    T = I.icosphere(1, 3.0)
    cen = np.array([[6.3, 7.1, 8.2], [17.6, 15.4, 19.9]])
    X = np.vstack([c + T for c in cen])
    c = Case(name=f"ib_carried_k{kernel}", nx=24, ny=24, nz=28, tau=0.8, steps=40, coupling=3,
             kernel=kernel, u_noise=0.0, pos=X, nshell=2, template=T, tether_k=0.05)
    c.extra["u0"] = np.array([0.05, -0.02, 0.04])
    check(c, TOL64)


# ------------------------------------------------------------- totals
def test_totals_match_oracle():
    c = _soft_alg3_case("totals", 20)
    o = run_oracle(c)
    g = run_gpu(c)
    scale = np.abs(o["totals"]).max()
    assert np.abs(g["totals"] - o["totals"]).max() <= 1e-12 * scale


def test_full_size_ib_shell_channel_fp32():
    """The immersed-boundary channel at full size, in the configuration the
    benchmark's IB workload uses: 128x128x256 with y walls, body force along z,
    64 shells of 642 markers (R = 6), 4-point kernel, FP32 storage; every output
    compared with the oracle after 3 steps."""
    box = (128, 128, 256)
    T = I.icosphere(3, 6.0)
    cen = I.shell_centres(64, 6.0, box, True, 4.0, 3.0, seed=3)
    X = np.vstack([c + T for c in cen])
    c = Case(name="c3_full", nx=128, ny=128, nz=256, tau=0.8, steps=3, wall_y=1,
             fext=(0.0, 0.0, 1e-6), coupling=3, kernel=4, storage=1, u_noise=0.0, pos=X,
             nshell=64, template=T, tether_k=0.05)
    check(c, TOL32)


@pytest.mark.parametrize("kernel", [2, 3, 4])
def test_ib_markers_crossing_tiles_and_seam(kernel):
    """IB markers (bonded in pairs) placed just below 8-site tile faces and at
    the periodic seam, carried by a uniform flow across cell faces: exercises
    the LDS-staged interpolation/spreading and its direct fallback for markers
    that leave their staged region."""
    rng = np.random.default_rng(12)
    base = np.array([[7.999, 3.2, 5.5], [15.9995, 8.0, 7.999], [23.9999, 0.0005, 15.9999],
                     [0.0001, 23.9999, 8.4], [11.5, 7.9999, 23.9995], [4.0, 16.0, 0.0]])
    pos = np.vstack([base, base + rng.uniform(-0.6, 0.6, base.shape)])
    pos = pos % 24.0
    n = len(base)
    bonds = np.array([[i, i + n] for i in range(n)])
    u0 = np.array([0.05, -0.03, 0.04])
    c = Case(name=f"ib_tiles_k{kernel}", nx=24, ny=24, nz=24, tau=0.7, steps=40, coupling=3,
             kernel=kernel, u_noise=0.0, pos=pos, bonds=bonds, bond_k=0.05, bond_r0=0.5,
             fext=(1e-6, 0.0, -1e-6))
    c.extra["u0"] = u0
    check(c, TOL64)


@pytest.mark.parametrize("kernel,rebin,steps",
                         [(4, 0, 30), (3, 0, 30), (4, 8, 30), (4, 100000, 110)])
def test_ib_markers_spread_over_many_tiles(kernel, rebin, steps):
    """IB markers (bonded in pairs) scattered over a 40x32x48 channel (5 x 4 x 6
    spreading tiles, y walls) and at its periodic seams, carried by a uniform
    flow.  With the default binning every tile gathers from its neighbouring
    bins; rebinned every 8 steps, four binnings in the run; binned only once
    (rebin 100000), the markers travel more than six sites from their bins,
    and the spreads after that take the fallback."""
    rng = np.random.default_rng(33)
    n = 60
    a = rng.uniform(0.0, 1.0, (n, 3)) * np.array([40.0, 30.0, 48.0]) + np.array([0.0, 1.0, 0.0])
    a[:6, 0] = [0.0002, 39.9998, 7.9999, 8.0, 31.9999, 24.0001]
    a[6:12, 2] = [0.0003, 47.9997, 15.9999, 16.0, 39.9999, 40.0]
    b = a + rng.uniform(-0.5, 0.5, (n, 3))
    b[:, 1] = np.clip(b[:, 1], 1.0, 30.0)
    pos = np.vstack([a, b]) % np.array([40.0, 32.0, 48.0])
    bonds = np.array([[i, i + n] for i in range(n)])
    c = Case(name=f"ib_many_tiles_k{kernel}_r{rebin}", nx=40, ny=32, nz=48, tau=0.7, steps=steps,
             wall_y=1, coupling=3, kernel=kernel, u_noise=0.0, pos=pos, bonds=bonds, bond_k=0.05,
             bond_r0=0.5, fext=(1e-6, 0.0, -1e-6))
    c.extra["u0"] = np.array([0.07, 0.0, -0.06])
    c.extra["ib_rebin"] = rebin
    g = run_gpu(c)
    o = run_oracle(c)
    compare(c, g, o, TOL64)
    if rebin > steps:  # binned once: the markers must have left their bins' neighbourhood
        d = o["pos"] - pos
        d -= np.array([40.0, 32.0, 48.0]) * np.round(d / np.array([40.0, 32.0, 48.0]))
        assert np.abs(d[:, 0]).max() > 7.0, "the markers did not leave their bins' neighbourhood"


@pytest.mark.parametrize("kernel,storage", [(4, 0), (3, 0), (4, 1)])
def test_ib_dense_tile_overflows_spread_accumulator(kernel, storage):
    """400 IB markers (bonded in pairs) packed into one 8^3 tile: their
    stencils cover most of the 13^3 region, more sites than the spreading
    workgroup accumulates in LDS, so the sites listed beyond that add to the
    global field directly; every interpolation row stays staged.  A uniform
    flow carries the markers across the tile's upper faces."""
    rng = np.random.default_rng(21)
    n = 200
    a = rng.uniform(8.0, 16.0, (n, 3))
    b = a + rng.uniform(-0.4, 0.4, (n, 3))
    pos = np.vstack([a, b]) % 24.0
    bonds = np.array([[i, i + n] for i in range(n)])
    c = Case(name=f"ib_dense_k{kernel}_s{storage}", nx=24, ny=24, nz=24, tau=0.7, steps=12,
             coupling=3, kernel=kernel, storage=storage, u_noise=0.0, pos=pos, bonds=bonds,
             bond_k=0.05, bond_r0=0.4, fext=(1e-6, 0.0, -1e-6))
    c.extra["u0"] = np.array([0.03, 0.02, -0.025])
    check(c, TOL64 if storage == 0 else TOL32)


def test_timing_stride_counts_timed_passes():
    """Timing brackets the first lattice pass and then one in every `stride`,
    up to the number of event pairs armed; the stepping itself is unchanged
    (the timed and untimed runs give bit-identical states)."""
    from paper_1406_2211_amd import lbc as L
    import torch
    res = []
    for stride in (1, 3, 8):
        lat = L.Lattice(16, 16, 16, tau=0.8, storage=L.LB_F32, body_force=(1e-5, 0.0, 2e-6))
        lat.lb_init_fluid()
        lat.lb_timing(100, stride)
        lat.lb_step(20)
        ms, n = lat.lb_timing_read()
        assert n == (20 + stride - 1) // stride and ms > 0.0
        lat.lb_timing(2, stride)
        lat.lb_step(20)
        _, n2 = lat.lb_timing_read()
        assert n2 == 2
        res.append(lat.lb_populations().cpu().numpy())
        with pytest.raises(L.LbcError):
            lat.lb_timing(1, 0)
        lat.lb_destroy()
    torch.cuda.synchronize()
    assert np.array_equal(res[0], res[1]) and np.array_equal(res[0], res[2])
