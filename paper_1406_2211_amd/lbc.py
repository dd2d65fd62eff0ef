"""ctypes binding of ``liblbc.so`` (the C ABI declared in ``include/lbc.h``).

Argument marshalling only: every step of the method runs in the HIP kernels.
PyTorch provides device memory and the stream.  There is no fallback: if the
library has not been built, using it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbc.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EBUSY, LB_EDEVICE, LB_ESTATE = range(6)
LB_BGK, LB_TRT, LB_MRT = 0, 1, 2
LB_FORCING_SPLIT2 = 0
LB_COUPLE_NONE, LB_COUPLE_FC, LB_COUPLE_EBF, LB_COUPLE_IB = 0, 1, 2, 3
LB_PHI2, LB_PHI3, LB_PHI4 = 2, 3, 4
LB_F64, LB_F32, LB_F16, LB_BF16 = 0, 1, 2, 3
LB_HARMONIC, LB_FENE = 0, 1

EXPORTS = ["lb_lattice_velocities", "lb_workspace_size", "lb_create", "lb_init_fluid",
           "lb_set_particles", "lb_set_bonds", "lb_set_shells", "lb_step", "lb_moments",
           "lb_populations", "lb_stress", "lb_stress_sweep", "lb_get_particles", "lb_totals", "lb_timing",
           "lb_timing_read", "lb_info", "lb_create_static", "lb_destroy",
           "lb_last_error", "lb_status_string", "lb_ensemble_footprint", "lb_ensemble_create",
           "lb_ensemble_stream", "lb_ensemble_admit", "lb_ensemble_step", "lb_ensemble_query",
           "lb_ensemble_retire", "lb_ensemble_autotune", "lb_ensemble_destroy",
           "lb_ensemble_last_error"]


class lb_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("wall_y", C.c_int32)]


class lb_params(C.Structure):
    _fields_ = [("tau", C.c_double), ("rho0", C.c_double), ("body_force", C.c_double * 3),
                ("collision", C.c_int32), ("trt_magic", C.c_double), ("forcing", C.c_int32),
                ("coupling", C.c_int32), ("gamma", C.c_double), ("kernel", C.c_int32),
                ("storage", C.c_int32), ("f16_scale_log2", C.c_int32),
                ("mts_substeps", C.c_int32), ("deterministic", C.c_int32),
                ("comoving", C.c_int32), ("csc", C.c_int32), ("mts_inside", C.c_int32),
                ("kT", C.c_double), ("seed", C.c_uint64), ("mrt_rates", C.c_double * 5),
                ("ib_rebin", C.c_int32)]


class lb_limits(C.Structure):
    _fields_ = [("max_particles", C.c_int64), ("max_bonds", C.c_int64),
                ("max_shells", C.c_int32), ("max_shell_size", C.c_int32)]


class LbcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lbc status {status}: {msg}")
        self.status = status


_lib = None


def load():
    """Load liblbc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1406_2211_amd/build.py "
                           "(or __graft_entry__.build())")
    # PyTorch's HIP runtime must be the process's runtime: it carries the same
    # soname as the one liblbc.so was linked against, so loading torch first
    # makes the dynamic loader bind liblbc.so to it (one runtime, one device
    # view).  Loading liblbc.so first would bring in a second runtime.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    G, P, M = C.POINTER(lb_grid), C.POINTER(lb_params), C.POINTER(lb_limits)
    sig = {
        "lb_lattice_velocities": (i32, [C.POINTER(i32)]),
        "lb_workspace_size": (i32, [G, P, M, C.POINTER(C.c_size_t)]),
        "lb_create": (i32, [G, P, M, vp, C.c_size_t, vp, C.POINTER(vp)]),
        "lb_create_static": (i32, [G, P, M, vp, C.POINTER(vp)]),
        "lb_init_fluid": (i32, [vp, vp, vp]),
        "lb_set_particles": (i32, [vp, i64, vp, vp, vp]),
        "lb_set_bonds": (i32, [vp, i64, vp, dbl, dbl, i32]),
        "lb_set_shells": (i32, [vp, i32, i32, vp, dbl]),
        "lb_step": (i32, [vp, i64]),
        "lb_moments": (i32, [vp, vp, vp]),
        "lb_populations": (i32, [vp, vp]),
        "lb_stress": (i32, [vp, vp]),
        "lb_stress_sweep": (i32, [vp, vp]),
        "lb_get_particles": (i32, [vp, vp, vp]),
        "lb_totals": (i32, [vp, C.POINTER(dbl)]),
        "lb_timing": (i32, [vp, i32, i32]),
        "lb_timing_read": (i32, [vp, C.POINTER(dbl), C.POINTER(i64)]),
        "lb_info": (i32, [vp, C.POINTER(i64), C.POINTER(i64)]),
        "lb_destroy": (i32, [vp]),
        "lb_last_error": (C.c_char_p, [vp]),
        "lb_status_string": (C.c_char_p, [i32]),
        "lb_ensemble_footprint": (i32, [G, P, M, C.POINTER(C.c_size_t)]),
        "lb_ensemble_create": (i32, [vp, C.c_size_t, i32, i32, i32, i32, vp, C.POINTER(vp)]),
        "lb_ensemble_stream": (i32, [vp, C.POINTER(vp)]),
        "lb_ensemble_admit": (i32, [vp, G, P, M, i64, C.POINTER(i32), C.POINTER(vp)]),
        "lb_ensemble_step": (i32, [vp, i64]),
        "lb_ensemble_query": (i32, [vp, i32, C.POINTER(i64), C.POINTER(i32)]),
        "lb_ensemble_retire": (i32, [vp, i32]),
        "lb_ensemble_autotune": (i32, [vp, i32, C.POINTER(i32), C.POINTER(i32)]),
        "lb_ensemble_destroy": (i32, [vp]),
        "lb_ensemble_last_error": (C.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status, ctx=None):
    if status != LB_OK:
        msg = load().lb_last_error(ctx).decode()
        raise LbcError(status, msg)


def lattice_velocities():
    c = (C.c_int32 * 57)()
    q = load().lb_lattice_velocities(c)
    return np.array(c[:], dtype=np.int64).reshape(q, 3)


def make_params(tau, rho0=1.0, body_force=(0.0, 0.0, 0.0), collision=LB_BGK, trt_magic=3.0 / 16.0,
                coupling=LB_COUPLE_NONE, gamma=0.0, kernel=LB_PHI2, storage=LB_F64,
                f16_scale_log2=0, mts_substeps=0, comoving=0, csc=0, mts_inside=0, kT=0.0,
                seed=0, mrt_rates=(1.0, 1.0, 1.0, 1.0, 1.0), deterministic=0, ib_rebin=0):
    p = lb_params()
    p.tau, p.rho0 = float(tau), float(rho0)
    for a in range(3):
        p.body_force[a] = float(body_force[a])
    p.collision, p.trt_magic, p.forcing = int(collision), float(trt_magic), LB_FORCING_SPLIT2
    p.coupling, p.gamma, p.kernel = int(coupling), float(gamma), int(kernel)
    p.storage, p.f16_scale_log2 = int(storage), int(f16_scale_log2)
    p.mts_substeps, p.deterministic = int(mts_substeps), int(deterministic)
    p.comoving, p.csc, p.mts_inside = int(comoving), int(csc), int(mts_inside)
    p.kT, p.seed = float(kT), int(seed)
    for k in range(5):
        p.mrt_rates[k] = float(mrt_rates[k])
    p.ib_rebin = int(ib_rebin)
    return p


def workspace_size(grid, params, limits):
    n = C.c_size_t()
    _check(load().lb_workspace_size(C.byref(grid), C.byref(params), C.byref(limits), C.byref(n)))
    return n.value


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Lattice:
    """One lattice context.  Device memory (the workspace) is a torch uint8
    tensor owned by this object; all calls are enqueued on ``stream`` (a
    torch.cuda.Stream; default: the current stream at construction).  With
    static_workspace=True the context is made by lb_create_static instead and
    takes its workspace from the library's static device array (no device
    memory is allocated; one such context per device at a time)."""

    def __init__(self, nx, ny, nz, wall_y=0, max_particles=0, max_bonds=0, max_shells=0,
                 max_shell_size=0, stream=None, device="cuda", _ctx=None, static_workspace=False,
                 **params):
        import torch
        self.torch = torch
        if _ctx is not None:  # a slot of an ensemble: the ensemble owns memory and stream
            self.grid = lb_grid(int(nx), int(ny), int(nz), int(wall_y))
            self.params = make_params(**params)
            self.device = torch.device(device)
            self.stream = stream
            self.workspace = None
            self.ctx = _ctx
            self.shape = (int(nz), int(ny), int(nx))
            self.N = int(nx) * int(ny) * int(nz)
            self.np = 0
            self._owned = False
            return
        self._owned = True
        self.grid = lb_grid(int(nx), int(ny), int(nz), int(wall_y))
        self.params = make_params(**params)
        self.limits = lb_limits(int(max_particles), int(max_bonds), int(max_shells),
                                int(max_shell_size))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.shape = (int(nz), int(ny), int(nx))
        self.N = int(nx) * int(ny) * int(nz)
        self.np = 0
        if static_workspace:
            self.workspace = None
            self.ctx = C.c_void_p()
            _check(load().lb_create_static(C.byref(self.grid), C.byref(self.params),
                                           C.byref(self.limits),
                                           C.c_void_p(self.stream.cuda_stream), C.byref(self.ctx)))
            return
        nbytes = workspace_size(self.grid, self.params, self.limits)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr = base + off
        self.ctx = C.c_void_p()
        _check(load().lb_create(C.byref(self.grid), C.byref(self.params), C.byref(self.limits),
                                C.c_void_p(self._ws_ptr), nbytes, C.c_void_p(self.stream.cuda_stream),
                                C.byref(self.ctx)))
        self.shape = (int(nz), int(ny), int(nx))
        self.N = int(nx) * int(ny) * int(nz)
        self.np = 0

    # -- helpers ------------------------------------------------------------
    def _f64(self, t, shape):
        t = self.torch.as_tensor(t, dtype=self.torch.float64, device=self.device)
        return t.reshape(shape).contiguous()

    def _call(self, name, *args):
        _check(getattr(load(), name)(self.ctx, *args), self.ctx)

    # -- ABI ----------------------------------------------------------------
    def lb_init_fluid(self, rho=None, u=None):
        r = None if rho is None else self._f64(rho, self.shape)
        v = None if u is None else self._f64(u, (3,) + self.shape)
        self.torch.cuda.synchronize(self.device)
        self._call("lb_init_fluid", _ptr(r), _ptr(v))
        self._keep = (r, v)

    def lb_set_particles(self, pos, vel=None, mass=None):
        p = self._f64(pos, (-1, 3))
        n = p.shape[0]
        v = None if vel is None else self._f64(vel, (n, 3))
        m = None if mass is None else self._f64(mass, (n,))
        self.torch.cuda.synchronize(self.device)
        self._call("lb_set_particles", n, _ptr(p), _ptr(v), _ptr(m))
        self._keep_p = (p, v, m)
        self.np = n

    def lb_set_bonds(self, pairs, k, r0, type=LB_HARMONIC):
        pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        self._call("lb_set_bonds", pr.shape[0], pr.ctypes.data_as(C.c_void_p), float(k),
                   float(r0), int(type))

    def lb_set_shells(self, nshell, template, k_tether):
        t = np.ascontiguousarray(template, dtype=np.float64).reshape(-1, 3)
        self._call("lb_set_shells", int(nshell), t.shape[0], t.ctypes.data_as(C.c_void_p),
                   float(k_tether))

    def lb_step(self, nsteps=1):
        self._call("lb_step", int(nsteps))

    def lb_moments(self):
        rho = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
        u = self.torch.empty((3,) + self.shape, dtype=self.torch.float64, device=self.device)
        self._call("lb_moments", _ptr(rho), _ptr(u))
        return rho, u

    def lb_populations(self):
        df = self.torch.empty((19,) + self.shape, dtype=self.torch.float64, device=self.device)
        self._call("lb_populations", _ptr(df))
        return df

    def lb_stress(self):
        sigma = self.torch.empty((6,) + self.shape, dtype=self.torch.float64, device=self.device)
        self._call("lb_stress", _ptr(sigma))
        return sigma

    def lb_stress_sweep(self, attach=True):
        """Attach (or detach) a [6, nz, ny, nx] tensor that every following
        lattice pass fills with the viscous stress of the state it starts
        from; FP64 with FP64 storage, FP32 otherwise.  Returns the tensor."""
        if not attach:
            self._call("lb_stress_sweep", None)
            self._sweep = None
            return None
        dt = self.torch.float64 if self.params.storage == LB_F64 else self.torch.float32
        self._sweep = self.torch.zeros((6,) + self.shape, dtype=dt, device=self.device)
        self.torch.cuda.synchronize(self.device)
        self._call("lb_stress_sweep", _ptr(self._sweep))
        return self._sweep

    def lb_get_particles(self):
        pos = self.torch.empty((self.np, 3), dtype=self.torch.float64, device=self.device)
        vel = self.torch.empty((self.np, 3), dtype=self.torch.float64, device=self.device)
        if self.np:
            self._call("lb_get_particles", _ptr(pos), _ptr(vel))
        return pos, vel

    def lb_totals(self):
        out = (C.c_double * 7)()
        self._call("lb_totals", out)
        return np.array(out[:])

    def lb_timing(self, max_passes, stride=1):
        self._call("lb_timing", int(max_passes), int(stride))

    def lb_timing_read(self):
        ms, n = C.c_double(), C.c_int64()
        self._call("lb_timing_read", C.byref(ms), C.byref(n))
        return ms.value, n.value

    def lb_info(self):
        n, s = C.c_int64(), C.c_int64()
        self._call("lb_info", C.byref(n), C.byref(s))
        return n.value, s.value

    def lb_destroy(self):
        if self.ctx and getattr(self, "_owned", True):
            load().lb_destroy(self.ctx)
        self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.lb_destroy()
        except Exception:
            pass


def _echeck(status, ens=None):
    if status != LB_OK:
        raise LbcError(status, load().lb_ensemble_last_error(ens).decode())


def ensemble_footprint(nx, ny, nz, max_particles=0, **params):
    n = C.c_size_t()
    g = lb_grid(int(nx), int(ny), int(nz), 0)
    p = make_params(**params)
    m = lb_limits(int(max_particles), 0, 0, 0)
    _check(load().lb_ensemble_footprint(C.byref(g), C.byref(p), C.byref(m), C.byref(n)))
    return n.value


class Ensemble:
    """Many periodic boxes resident in one device pool (a torch uint8 tensor)
    and stepped together by batched launches replayed from HIP graphs, all
    ordered on ``stream`` (a torch.cuda.Stream the library borrows).  Without
    one the library makes its own blocking default-priority stream (the legacy
    null stream cannot be captured), which orders with work on torch's default
    stream."""

    def __init__(self, pool_bytes, max_slots, storage=LB_F32, kernel=LB_PHI2, device="cuda",
                 stream=None, deterministic=0):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream
        self.pool = torch.empty(int(pool_bytes) + 256, dtype=torch.uint8, device=self.device)
        base = self.pool.data_ptr()
        ptr = base + ((-base) % 256)
        self.storage, self.kernel = int(storage), int(kernel)
        self.deterministic = int(deterministic)
        self.ens = C.c_void_p()
        torch.cuda.synchronize(self.device)
        _echeck(load().lb_ensemble_create(C.c_void_p(ptr), int(pool_bytes), int(max_slots),
                                          self.storage, self.kernel, self.deterministic,
                                          None if stream is None else C.c_void_p(stream.cuda_stream),
                                          C.byref(self.ens)))
        st = C.c_void_p()
        _echeck(load().lb_ensemble_stream(self.ens, C.byref(st)), self.ens)
        self.stream_ptr = st.value
        self.slots = {}

    def admit(self, nx, ny, nz, nsteps, max_particles=0, **params):
        """Returns (slot, Lattice view of the slot) or None when the pool or the
        slot table is full (LB_EBUSY)."""
        g = lb_grid(int(nx), int(ny), int(nz), 0)
        params.setdefault("storage", self.storage)
        params.setdefault("kernel", self.kernel)
        params.setdefault("deterministic", self.deterministic)
        p = make_params(**params)
        m = lb_limits(int(max_particles), 0, 0, 0)
        slot, ctx = C.c_int32(), C.c_void_p()
        st = load().lb_ensemble_admit(self.ens, C.byref(g), C.byref(p), C.byref(m), int(nsteps),
                                      C.byref(slot), C.byref(ctx))
        if st == LB_EBUSY:
            return None
        _echeck(st, self.ens)
        lat = Lattice(nx, ny, nz, stream=None, device=self.device, _ctx=ctx, **params)
        self.slots[slot.value] = lat
        return slot.value, lat

    def step(self, nsteps):
        _echeck(load().lb_ensemble_step(self.ens, int(nsteps)), self.ens)

    def query(self, slot):
        sd, done = C.c_int64(), C.c_int32()
        _echeck(load().lb_ensemble_query(self.ens, int(slot), C.byref(sd), C.byref(done)), self.ens)
        return sd.value, bool(done.value)

    def retire(self, slot):
        _echeck(load().lb_ensemble_retire(self.ens, int(slot)), self.ens)
        lat = self.slots.pop(slot, None)
        if lat is not None:
            lat.ctx = C.c_void_p()

    def autotune(self, steps_per_candidate=2):
        lg, pg = C.c_int32(), C.c_int32()
        _echeck(load().lb_ensemble_autotune(self.ens, int(steps_per_candidate), C.byref(lg),
                                            C.byref(pg)), self.ens)
        return lg.value, pg.value

    def synchronize(self):
        self.torch.cuda.synchronize(self.device)

    def destroy(self):
        if self.ens:
            for lat in self.slots.values():
                lat.ctx = C.c_void_p()
            self.slots = {}
            load().lb_ensemble_destroy(self.ens)
            self.ens = C.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
