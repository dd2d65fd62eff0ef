"""FP64 CPU oracle of the operator-split lattice Boltzmann step with
fluid-particle coupling (Schiller, arXiv:1406.2211).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark may import this package.  It wraps ``liblbo.so``
(built from ``lbo.c`` by ``oracle/build.py``) with ctypes and numpy and shares
no code with the GPU library.

Array conventions: populations are deviations ``df[19, nz, ny, nx]`` from
``w_i * rho0``; vector fields are ``[3, nz, ny, nx]``; particles ``[np, 3]``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbo.so")
_lib = None

BGK, TRT, MRT = 0, 1, 2
NONE, FC, EBF, IB = 0, 1, 2, 3
HARMONIC, FENE = 0, 1
Q = 19

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


class _Cfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("wall_y", C.c_int),
        ("tau", C.c_double), ("rho0", C.c_double), ("fext", C.c_double * 3),
        ("collision", C.c_int), ("magic", C.c_double),
        ("coupling", C.c_int), ("gamma", C.c_double), ("kernel", C.c_int),
        ("mts_n", C.c_int),
        ("nbond", C.c_int), ("bond_pairs", C.c_void_p), ("bond_k", C.c_double),
        ("bond_r0", C.c_double), ("bond_type", C.c_int),
        ("nshell", C.c_int), ("shell_size", C.c_int), ("shell_template", C.c_void_p),
        ("tether_k", C.c_double),
        ("csc", C.c_int),
        ("mts_inside", C.c_int),
        ("kT", C.c_double), ("seed", C.c_uint64), ("step0", C.c_int64),
        ("mrt_rates", C.c_double * 5),
        ("order", C.c_int),
    ]


def lib():
    """Load liblbo.so, building it first if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    L = C.CDLL(_LIB_PATH)
    P = C.POINTER(_Cfg)
    vp = C.c_void_p
    sig = {
        "lbo_d3q19": (C.c_int, [_ip, _dp, _ip]),
        "lbo_feq_dev": (None, [C.c_double, C.c_double, _dp, _dp]),
        "lbo_force_term": (None, [_dp, _dp, _dp]),
        "lbo_mrt_basis": (None, [_dp, _dp]),
        "lbo_group_basis": (None, [_dp, _dp]),
        "lbo_rates": (None, [P, _dp]),
        "lbo_collide_site": (None, [P, _dp]),
        "lbo_init_fluid": (None, [P, _dp, vp, vp]),
        "lbo_moments": (None, [P, _dp, _dp, _dp]),
        "lbo_force_half": (None, [P, _dp, vp]),
        "lbo_collide": (None, [P, _dp]),
        "lbo_collide_half": (None, [P, _dp]),
        "lbo_stress": (None, [P, _dp, _dp]),
        "lbo_stream": (None, [P, _dp, _dp]),
        "lbo_phi": (C.c_double, [C.c_int, C.c_double]),
        "lbo_interp": (None, [P, C.c_int, _dp, _dp, _dp, _dp, _dp]),
        "lbo_spread": (None, [P, C.c_int, _dp, _dp, _dp]),
        "lbo_fc_force": (None, [C.c_double] * 4 + [_dp, _dp, _dp, _dp]),
        "lbo_ebf_update": (None, [C.c_double] * 4 + [_dp, _dp, _dp, _dp, _dp]),
        "lbo_bond_forces": (None, [P, C.c_int, _dp, _dp]),
        "lbo_tether_forces": (None, [P, _dp, _dp, vp]),
        "lbo_intrinsic": (None, [P, C.c_int, _dp, _dp]),
        "lbo_run": (C.c_int, [P, C.c_int, _dp, C.c_int, vp, vp, vp]),
        "lbo_totals": (None, [P, _dp, C.c_int, vp, vp, _dp]),
        "lbo_threads": (C.c_int, []),
        "lbo_philox": (None, [_u32p, _u32p, _u32p]),
        "lbo_normals4": (None, [_u32p, _u32p, _dp]),
        "lbo_site_normals": (None, [P, C.c_int64, C.c_uint32, _dp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def lattice():
    """(c[19,3], w[19], opp[19]) of the oracle's D3Q19 lattice."""
    c = np.zeros(Q * 3, np.int32)
    w = np.zeros(Q)
    opp = np.zeros(Q, np.int32)
    lib().lbo_d3q19(c, w, opp)
    return c.reshape(Q, 3), w, opp


def feq_dev(rho, rho0, u):
    """f^eq(rho, u) - w rho0."""
    out = np.zeros(Q)
    lib().lbo_feq_dev(float(rho) - float(rho0), float(rho), _f64(u), out)
    return out


def force_term(u, F):
    G = np.zeros(Q)
    lib().lbo_force_term(_f64(u), _f64(F), G)
    return G


def mrt_basis():
    E = np.zeros(Q * Q)
    b = np.zeros(Q)
    lib().lbo_mrt_basis(E, b)
    return E.reshape(Q, Q), b


def group_basis():
    """Rows E[k, i] and norms b[k] of the general MRT basis (moment groups)."""
    E = np.zeros(Q * Q)
    b = np.zeros(Q)
    lib().lbo_group_basis(E, b)
    return E.reshape(Q, Q), b


def phi(kernel, r):
    return lib().lbo_phi(int(kernel), float(r))


def philox(ctr, key):
    """Philox4x32-10 block of the 4-word counter ctr under the 2-word key."""
    out = np.zeros(4, np.uint32)
    lib().lbo_philox(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def normals4(ctr, key):
    """Four standard normal deviates (Box-Muller) from one Philox block."""
    g = np.zeros(4)
    lib().lbo_normals4(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), g)
    return g


def fc_force(gamma, m, rho_p, hh, v, u_p, Fint):
    Fh = np.zeros(3)
    lib().lbo_fc_force(gamma, m, rho_p, hh, _f64(v), _f64(u_p), _f64(Fint), Fh)
    return Fh


def ebf_update(gamma, m, rho_p, hh, v, u_p, Fint):
    Fh = np.zeros(3)
    vn = np.zeros(3)
    lib().lbo_ebf_update(gamma, m, rho_p, hh, _f64(v), _f64(u_p), _f64(Fint), Fh, vn)
    return Fh, vn


class Oracle:
    """One configuration of the oracle.  Keys of ``cfg`` (defaults in brackets):
    nx, ny, nz, wall_y [0], tau, rho0 [1], fext [(0,0,0)], collision [BGK],
    magic [3/16], coupling [NONE], gamma [0], kernel [2], mts_n [0],
    bonds [None: int32 [nb,2]], bond_k, bond_r0, bond_type [HARMONIC],
    nshell [0], shell_template [None: [M,3]], tether_k, csc [0: the C S form; 1: C^1/2 S C^1/2],
    mts_inside [0: coupling outside the sub-steps; 1: inside every sub-step], kT [0: no
    fluctuations], seed [0], step0 [0: index of the first step in the random streams],
    mrt_rates [5 x 1.0: bulk, vector ghosts, pseudo-vector ghosts, scalar and tensor ghosts;
    collision MRT], order [0: the second-order splitting; test-only alternatives: 1 the
    first-order P S C F sequence, 2 a planted misordering (see lbo.h)]."""

    def __init__(self, **cfg):
        self.nx, self.ny, self.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg["nz"])
        c = _Cfg()
        c.nx, c.ny, c.nz = self.nx, self.ny, self.nz
        c.wall_y = int(cfg.get("wall_y", 0))
        c.tau = float(cfg["tau"])
        c.rho0 = float(cfg.get("rho0", 1.0))
        for a, v in enumerate(cfg.get("fext", (0.0, 0.0, 0.0))):
            c.fext[a] = float(v)
        c.collision = int(cfg.get("collision", BGK))
        c.magic = float(cfg.get("magic", 3.0 / 16.0))
        c.coupling = int(cfg.get("coupling", NONE))
        c.gamma = float(cfg.get("gamma", 0.0))
        c.kernel = int(cfg.get("kernel", 2))
        c.mts_n = int(cfg.get("mts_n", 0))
        bonds = cfg.get("bonds")
        self._bonds = None
        if bonds is not None and len(bonds):
            self._bonds = np.ascontiguousarray(bonds, dtype=np.int32).reshape(-1, 2)
            c.nbond = self._bonds.shape[0]
            c.bond_pairs = self._bonds.ctypes.data
        c.bond_k = float(cfg.get("bond_k", 0.0))
        c.bond_r0 = float(cfg.get("bond_r0", 0.0))
        c.bond_type = int(cfg.get("bond_type", HARMONIC))
        tmpl = cfg.get("shell_template")
        self._tmpl = None
        if tmpl is not None and int(cfg.get("nshell", 0)) > 0:
            self._tmpl = _f64(tmpl).reshape(-1, 3)
            c.nshell = int(cfg["nshell"])
            c.shell_size = self._tmpl.shape[0]
            c.shell_template = self._tmpl.ctypes.data
        c.tether_k = float(cfg.get("tether_k", 0.0))
        c.csc = int(cfg.get("csc", 0))
        c.mts_inside = int(cfg.get("mts_inside", 0))
        c.kT = float(cfg.get("kT", 0.0))
        c.seed = int(cfg.get("seed", 0))
        c.step0 = int(cfg.get("step0", 0))
        for k, r in enumerate(cfg.get("mrt_rates", (1.0,) * 5)):
            c.mrt_rates[k] = float(r)
        c.order = int(cfg.get("order", 0))
        self.cfg = c
        self.N = self.nx * self.ny * self.nz
        self.shape = (self.nz, self.ny, self.nx)

    # -- fields ---------------------------------------------------------
    def init_fluid(self, rho=None, u=None):
        df = np.zeros((Q,) + self.shape)
        r = None if rho is None else _f64(rho, self.shape)
        uu = None if u is None else _f64(u, (3,) + self.shape)
        lib().lbo_init_fluid(C.byref(self.cfg), df, _ptr(r), _ptr(uu))
        return df

    def moments(self, df):
        rho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        lib().lbo_moments(C.byref(self.cfg), _f64(df), rho, u)
        return rho, u

    def force_half(self, df, Fc=None):
        df = _f64(df).copy()
        F = None if Fc is None else _f64(Fc, (3,) + self.shape)
        lib().lbo_force_half(C.byref(self.cfg), df, _ptr(F))
        return df

    def collide(self, df):
        df = _f64(df).copy()
        lib().lbo_collide(C.byref(self.cfg), df)
        return df

    def collide_half(self, df):
        df = _f64(df).copy()
        lib().lbo_collide_half(C.byref(self.cfg), df)
        return df

    def site_normals(self, step, site):
        """The 19 normal deviates of one site in one step, g[i] for velocity c_i."""
        g = np.zeros(Q)
        lib().lbo_site_normals(C.byref(self.cfg), int(step), int(site), g)
        return g

    def stress(self, df):
        """Pi_ab = sum_i (f_i - f^eq_i) c_ia c_ib, [6] + shape: xx yy zz xy xz yz."""
        pi = np.zeros((6,) + self.shape)
        lib().lbo_stress(C.byref(self.cfg), _f64(df), pi)
        return pi

    def collide_site(self, f):
        f = _f64(f).copy()
        lib().lbo_collide_site(C.byref(self.cfg), f)
        return f

    def rates(self):
        lam = np.zeros(Q)
        lib().lbo_rates(C.byref(self.cfg), lam)
        return lam

    def stream(self, df):
        src = _f64(df)
        dst = np.zeros_like(src)
        lib().lbo_stream(C.byref(self.cfg), src, dst)
        return dst

    # -- particles ------------------------------------------------------
    def interp(self, pos, rho, u):
        pos = _f64(pos, (-1, 3))
        n = pos.shape[0]
        rp = np.zeros(n)
        up = np.zeros((n, 3))
        lib().lbo_interp(C.byref(self.cfg), n, pos, _f64(rho, self.shape),
                         _f64(u, (3,) + self.shape), rp, up)
        return rp, up

    def spread(self, pos, Fp, Fgrid=None):
        pos = _f64(pos, (-1, 3))
        out = np.zeros((3,) + self.shape) if Fgrid is None else _f64(Fgrid).copy()
        lib().lbo_spread(C.byref(self.cfg), pos.shape[0], pos, _f64(Fp, (-1, 3)), out)
        return out

    def bond_forces(self, pos):
        pos = _f64(pos, (-1, 3))
        F = np.zeros_like(pos)
        lib().lbo_bond_forces(C.byref(self.cfg), pos.shape[0], pos, F)
        return F

    def tether_forces(self, pos, want_rot=False):
        pos = _f64(pos, (-1, 3))
        F = np.zeros_like(pos)
        rot = np.zeros((max(self.cfg.nshell, 1), 3, 3)) if want_rot else None
        lib().lbo_tether_forces(C.byref(self.cfg), pos, F, _ptr(rot))
        return (F, rot) if want_rot else F

    def intrinsic(self, pos):
        pos = _f64(pos, (-1, 3))
        F = np.zeros_like(pos)
        lib().lbo_intrinsic(C.byref(self.cfg), pos.shape[0], pos, F)
        return F

    # -- time stepping --------------------------------------------------
    def run(self, df, nsteps, pos=None, vel=None, mass=None):
        """Advance (df, pos, vel) in place by nsteps full time steps."""
        assert df.dtype == np.float64 and df.flags.c_contiguous
        n = 0 if pos is None else pos.shape[0]
        for a in (pos, vel):
            assert a is None or (a.dtype == np.float64 and a.flags.c_contiguous)
        m = None if mass is None else _f64(mass)
        rc = lib().lbo_run(C.byref(self.cfg), int(nsteps), df, n, _ptr(pos), _ptr(vel), _ptr(m))
        if rc != 0:
            raise ValueError(f"oracle rejected the configuration (code {rc})")

    def totals(self, df, vel=None, mass=None):
        out = np.zeros(7)
        n = 0 if vel is None else vel.shape[0]
        m = None if mass is None else _f64(mass)
        v = None if vel is None else _f64(vel)
        lib().lbo_totals(C.byref(self.cfg), _f64(df), n, _ptr(v), _ptr(m), out)
        return out


def threads():
    return lib().lbo_threads()
