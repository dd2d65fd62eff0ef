/*
 * lbc.h -- C ABI of the MI355X (gfx950) lattice Boltzmann library with
 * operator-split second-order forcing and fluid-particle coupling, after
 * Schiller, "A unified operator splitting approach for multi-scale
 * fluid-particle coupling in the lattice Boltzmann method" (arXiv:1406.2211).
 *
 * Conventions shared by every call
 *   - Lattice units: time step h = 1, lattice spacing a = 1.  D3Q19.
 *   - Every call returns an lb_status; no exception crosses the ABI.  On a
 *     failure lb_last_error(ctx) holds a message (lb_last_error(NULL) holds
 *     the message of a failed lb_create / lb_workspace_size).
 *   - Pointers named d_* are device pointers, h_* host pointers, both owned
 *     by the caller.  The library never allocates device memory: all of its
 *     device state lives in the caller's workspace (lb_workspace_size).
 *   - Every device operation is enqueued on the stream given to lb_create and
 *     is asynchronous unless stated otherwise.  Parameter errors are detected
 *     on the host before anything is enqueued.
 *   - Field layouts: scalar fields [nz][ny][nx] (x fastest); vector fields
 *     [3][nz][ny][nx]; populations [19][nz][ny][nx] in the order returned by
 *     lb_lattice_velocities; particle vectors [n][3].  Exchange precision is
 *     FP64 regardless of the storage precision.
 *   - tau is the lattice relaxation time: the Crank-Nicolson collision of
 *     Sec. 3.2 (Eq. collision-operator) with BGK time tau_paper relaxes at
 *     lambda = h/(tau_paper + h/2); this ABI takes tau = tau_paper + h/2 > 1/2.
 *
 * One time step (Eq. LB-splitting and Eq. fc-splitting) is
 *   P^1/2  F^1/2  C  S  F^1/2  P^1/2
 * where F^1/2 is the midpoint half force (Sec. 3.3) applied to the lattice
 * together with the coupling half step, C the full collision (which equals
 * C^1/2 C^1/2 of Eq. LB-splitting up to the end half-collisions, Eq.
 * LB-splitting-combined) and S streaming (Sec. 3.1).  The library stores the
 * post-collision populations and folds the second half force of one step and
 * the first half force of the next into a single exact equilibrium shift of
 * one fused lattice pass; the physical state is defined at every step
 * boundary and is what lb_moments / lb_populations / lb_totals return.
 */
#ifndef LBC_H
#define LBC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lb_status {
  LB_OK = 0,
  LB_EINVAL = 1,  /* invalid argument or configuration */
  LB_ENOMEM = 2,  /* workspace too small or capacity exceeded */
  LB_EBUSY = 3,   /* ensemble has no free slot or memory for a request */
  LB_EDEVICE = 4, /* a HIP runtime call failed */
  LB_ESTATE = 5   /* call not valid in the current state */
} lb_status;

enum lb_collision { LB_BGK = 0, LB_TRT = 1, LB_MRT = 2 };
enum lb_forcing { LB_FORCING_SPLIT2 = 0 };
enum lb_coupling { LB_COUPLE_NONE = 0, LB_COUPLE_FC = 1, LB_COUPLE_EBF = 2, LB_COUPLE_IB = 3 };
enum lb_kernel { LB_PHI2 = 2, LB_PHI3 = 3, LB_PHI4 = 4 };
enum lb_storage { LB_F64 = 0, LB_F32 = 1, LB_F16 = 2, LB_BF16 = 3 };
enum lb_bond_type { LB_HARMONIC = 0, LB_FENE = 1 };

typedef struct lb_grid {
  int32_t nx, ny, nz;
  int32_t wall_y; /* 0: periodic in y; 1: halfway bounce-back walls at y=-1/2, ny-1/2 */
} lb_grid;

typedef struct lb_params {
  double tau;            /* lattice relaxation time (> 1/2), see above */
  double rho0;           /* reference density; populations are stored as f - w rho0 */
  double body_force[3];  /* constant body-force density F_ext */
  int32_t collision;     /* LB_BGK; LB_TRT: MRT with the two rates of Eq. mrt-coll; LB_MRT:
                            Eq. mrt-coll with a rate per moment group (mrt_rates) */
  double trt_magic;      /* (1/l+ - 1/2)(1/l- - 1/2) for LB_TRT; 3/16 if <= 0 */
  int32_t forcing;       /* LB_FORCING_SPLIT2: midpoint half forces around C S */
  int32_t coupling;      /* LB_COUPLE_* (Sec. 5.1 IB, 5.2 FC, 5.3 modified EBF) */
  double gamma;          /* friction of FC / EBF (Eq. viscous-coupling) */
  int32_t kernel;        /* LB_PHI2, LB_PHI3, LB_PHI4 (Appendix A) */
  int32_t storage;       /* LB_F64 (FP64 compute), LB_F32/LB_F16/LB_BF16 (FP32 compute) */
  int32_t f16_scale_log2;/* LB_F16/LB_BF16: stored value is 2^p (f - w rho0) */
  int32_t mts_substeps;  /* 0: Alg. 3 ordering; n > 0: Sec. 6 split with the coupling
                            outside and n velocity-Verlet sub-steps on each side */
  int32_t deterministic; /* 0: spreading (Eq. IBM-spreading, the adjoint of interpolation) adds
                            each contribution W F to its site with a floating-point atomic, so
                            the order of the additions, and the rounding of the sum, varies
                            from run to run.  1: the sum at each site is formed exactly in
                            128-bit fixed point (resolution 2^-96, contributions below 2^20)
                            with integer atomics and then rounded once, so every run gives
                            bitwise the same result, alone or in an ensemble mix.  Slower
                            (two extra launches per spread, 48 B of accumulator per site). */
  int32_t comoving;      /* 0: store f - w rho0; 1: store f - f^eq(rho0, U_ref) with U_ref
                            advancing by F_ext/rho0 per step (the mean velocity a uniform body
                            force gives the fluid); an exact change of variables that keeps
                            stored values small in 16-bit storage */
  int32_t csc;           /* 0: the standard state; 1: the collide-stream-collide form of
                            Sec. 4 (Eq. csc): the state at a step boundary is the half
                            collision C^1/2 of the standard one (Eq. LB-splitting-combined),
                            with 1 - lambda_1/2 = sqrt(1 - lambda) per rate (Sec. 3.2), so
                            every rate must be <= 1 (tau >= 1; for LB_TRT also
                            trt_magic >= (tau - 1/2)/2), else LB_EINVAL.  Dynamics, moments,
                            particles and stress are those of the standard form. */
  int32_t mts_inside;    /* with mts_substeps = n > 0: 0 the coupling outside the sub-steps
                            (Sec. 6, second decomposition: F_h^1/2 [P F_int P]^n (C S)
                            [P F_int P]^n F_h^1/2); 1 the coupling inside every sub-step
                            (Eq. multistep: [P^(1/4n) F^(1/2n) P^(1/4n)]^n (C S) [...]^n, F
                            holding every force; 2n coupling evaluations per step).
                            LB_EINVAL without sub-steps.  Unless deterministic is set, the
                            workspace also holds min(n - 1, 4) extra force fields (16 B per
                            site each, 32 B in FP64) and a second copy of the particle
                            state. */
  double kT;             /* thermal energy k_B T (lattice units); 0: deterministic.  > 0: the
                            fluctuating collision of Eq. mrt-fluct (noise sqrt(rho) phi_k r_k
                            on every non-conserved moment, phi_k = sqrt(mu b_k lambda_k
                            (2 - lambda_k)), mu = k_B T / c_s^2) and, for LB_COUPLE_FC, the
                            random force zeta of Eq. viscous-coupling (variance
                            2 k_B T gamma / h' per component over a coupling step h').  Not
                            with csc or comoving (LB_EINVAL) nor in ensembles. */
  uint64_t seed;         /* key of the Philox4x32-10 streams; the random numbers of a step
                            depend only on (seed, step index, site or particle), not on the
                            launch configuration */
  double mrt_rates[5];   /* LB_MRT: relaxation rates in (0, 2) of the moment groups of the
                            D3Q19 basis of Duenweg, Schiller and Ladd (2007), each invariant
                            under the cubic symmetry: [0] bulk stress c^2 - 1 (bulk viscosity
                            (2/3) rho c_s^2 (1/rate - 1/2)), [1] vector ghosts c_a(3c^2 - 5),
                            [2] pseudo-vector ghosts cx(cy^2 - cz^2) and cyclic, [3] scalar
                            ghost 3c^4 - 6c^2 + 1, [4] tensor ghosts (2c^2 - 3)(3cx^2 - c^2),
                            (2c^2 - 3)(cy^2 - cz^2).  The shear stress relaxes at 1/tau.  Not
                            with csc or comoving, nor in ensembles (LB_EINVAL). */
  int32_t ib_rebin;      /* LB_COUPLE_IB with LB_PHI3/LB_PHI4 (markers binned into 8^3 tiles
                            for spreading): steps between two binnings, 0 for the default 32.
                            Any value gives the same results: a marker whose stencil leaves
                            its bin's neighbourhood switches that spread to a slower path. */
} lb_params;

typedef struct lb_limits {
  int64_t max_particles;  /* capacity for lb_set_particles */
  int64_t max_bonds;      /* capacity for lb_set_bonds */
  int32_t max_shells;     /* capacity for lb_set_shells */
  int32_t max_shell_size;
} lb_limits;

typedef struct lb_ctx lb_ctx;

/* D3Q19 velocity set (the discrete velocities c_i of Sec. 2, Eq.
 * discrete-Boltzmann; the paper fixes no particular set) in library order,
 * c[i*3 + a] into a caller array of 57; returns 19.  No error. */
int32_t lb_lattice_velocities(int32_t c[57]);

/* Device bytes needed for a context of this size (a pure function of the
 * arguments): the two population buffers of the pull stream (Sec. 3.1), the
 * coupling force fields of the two half steps (Sec. 5), particle state and
 * tables.  The caller allocates them (alignment 256 B) and passes them to
 * lb_create.  Errors: LB_EINVAL for invalid arguments (checked on the host). */
lb_status lb_workspace_size(const lb_grid* g, const lb_params* p, const lb_limits* lim,
                            size_t* bytes);

/* Creates a context on the current HIP device: the lattice of Sec. 3 (Eq.
 * split-lb) with the relaxation time and collision of Sec. 3.2 (Eq.
 * collision-operator, Eq. mrt-coll), the forcing of Sec. 3.3 and the coupling
 * scheme of Sec. 5 chosen in lb_params.  The workspace and the stream (a
 * hipStream_t, or NULL for the null stream) are borrowed: the caller keeps
 * them alive until lb_destroy.  Initialises the fluid at rest,
 * f = f^eq(rho0, 0), with no particles.  Errors: LB_EINVAL (bad grid or
 * parameters, e.g. tau <= 1/2), LB_ENOMEM (workspace smaller than
 * lb_workspace_size), LB_EDEVICE. */
lb_status lb_create(const lb_grid* g, const lb_params* p, const lb_limits* lim,
                    void* d_workspace, size_t bytes, void* hip_stream, lb_ctx** out);

/* Sets the physical state f = f^eq(rho, u) (moments of Sec. 2).  d_rho
 * [nz][ny][nx] and d_u [3][nz][ny][nx] are FP64 device arrays; NULL means
 * rho0 and 0. */
lb_status lb_init_fluid(lb_ctx* ctx, const double* d_rho, const double* d_u);

/* Copies n particles into the context: for FC/EBF the positions r_i,
 * velocities v_i and masses m_i > 0 of the particle equations of motion
 * (Sec. 5.2, Eq. fc-vel and the equations before Eq. fc-splitting); for IB
 * the Lagrangian marker positions X_i of Sec. 5.1 (velocities and masses are
 * ignored and may be NULL; markers move with the interpolated fluid).  FP64
 * device arrays [n][3], [n][3], [n], read (copied) on the context stream.
 * Positions in periodic directions are wrapped into [0, L).  Errors:
 * LB_ENOMEM if n exceeds max_particles, LB_EINVAL for n < 0 or a NULL array
 * that is needed. */
lb_status lb_set_particles(lb_ctx* ctx, int64_t n, const double* d_pos, const double* d_vel,
                           const double* d_mass);

/* Bonds between particles (intrinsic forces, "CalculateForces" of Alg. 3
 * and Alg. 2; the paper leaves their model open): harmonic
 * U = k/2 (|d| - r0)^2 or FENE U = -k r0^2/2 ln(1 - |d|^2/r0^2) with d the
 * minimum-image separation.  A FENE bond stretched to |d| >= r0 has infinite
 * energy: its force is NaN, which propagates into the particles and the
 * fluid (the run is not stopped; lb_totals then reports non-finite sums).
 * h_pairs [nb][2] host int32 particle indices, copied.  Bonded clusters must
 * not exceed 1024 particles.  Errors: LB_ENOMEM beyond max_bonds, LB_EINVAL
 * for an unknown type, non-finite k or r0, or FENE with r0 <= 0.
 * Synchronous. */
lb_status lb_set_bonds(lb_ctx* ctx, int64_t nb, const int32_t* h_pairs, double k, double r0,
                       int32_t type);

/* Rigid shells for IB (intrinsic forces of Alg. 2): markers
 * s*shell_size .. (s+1)*shell_size-1 form shell s and are tethered with
 * stiffness k_tether to a copy of h_template ([shell_size][3] host FP64,
 * centred on the origin) placed at the shell centroid with the least-squares
 * rotation.  Synchronous. */
lb_status lb_set_shells(lb_ctx* ctx, int32_t nshell, int32_t shell_size,
                        const double* h_template, double k_tether);

/* Advances nsteps full time steps (see the top of this file; Alg. 2 for IB,
 * Alg. 3 or the Sec. 6 split for FC/EBF).  Asynchronous. */
lb_status lb_step(lb_ctx* ctx, int64_t nsteps);

/* Physical density and velocity at every site (rho u = sum_i f_i c_i of the
 * physical populations, i.e. including the second half force; the
 * redefined velocity of Sec. 4).  FP64 device outputs d_rho [nz][ny][nx]
 * (may be NULL) and d_u [3][nz][ny][nx]. */
lb_status lb_moments(lb_ctx* ctx, double* d_rho, double* d_u);

/* Physical populations as deviations f_i - w_i rho0, FP64 [19][nz][ny][nx].
 * With csc = 1 these are the collide-stream-collide populations (Eq. csc):
 * f^eq(rho, u) + sqrt(1 - lambda) (f - f^eq(rho, u)) per relaxation mode of
 * the standard physical populations f, which have the same rho and u. */
lb_status lb_populations(lb_ctx* ctx, double* d_df);

/* Local viscous stress (Eq. viscstress) at every site, FP64 device output
 * d_sigma [6][nz][ny][nx] in the order xx, yy, zz, xy, xz, yz:
 * sigma = (1 - lambda_+/2) sum_i (f_i - f^eq_i(rho, u)) c_i c_i of the
 * standard physical populations, lambda_+ = 1/tau the rate of the stress
 * modes (with LB_MRT the trace part takes (1 - lambda_bulk/2) instead).  This equals (1/2)((1 - lambda_1/2)^-1 + (1 - lambda_1/2)) times the
 * same sum over the collide-stream-collide populations, and -rho nu
 * (grad u + grad u^T) with nu = (tau - 1/2)/3 up to second-order terms.  The
 * same physical quantity in both forms; the half forces are equilibrium
 * shifts and do not enter it.  Asynchronous. */
lb_status lb_stress(lb_ctx* ctx, double* d_sigma);

/* Viscous stress in the sweep (Sec. 4: in the collide-stream-collide form the
 * stress is available locally at every step): with d_sigma non-NULL, every
 * fused lattice pass that follows also writes, at every site, the viscous
 * stress of Eq. viscstress (the quantity lb_stress returns) of the physical
 * state the pass starts from, i.e. lb_step(1) leaves in d_sigma the stress of
 * the state it was called on, at the cost of the stores only (no extra read
 * pass).  d_sigma is [6][nz][ny][nx] (xx, yy, zz, xy, xz, yz) in the compute
 * precision: FP64 with LB_F64 storage, FP32 otherwise; owned by the caller,
 * who keeps it alive while attached.  NULL detaches.  Errors: LB_EINVAL with
 * LB_MRT or kT > 0 (not supported), LB_ESTATE on an ensemble slot. */
lb_status lb_stress_sweep(lb_ctx* ctx, void* d_sigma);

/* Current particle positions and velocities (r_i, v_i of Sec. 5.2; for IB the
 * marker positions X_i of Sec. 5.1 and zero velocities) at the step boundary,
 * copied on the context stream into FP64 device arrays [n][3] owned by the
 * caller (either may be NULL).  Asynchronous; no error beyond a NULL context. */
lb_status lb_get_particles(lb_ctx* ctx, double* d_pos, double* d_vel);

/* Conserved totals in FP64, reduced on the device in a fixed order: mass,
 * conserved by collision and streaming (Sec. 3.1, 3.2), and momentum, which
 * the coupling exchanges between fluid and particles with equal and opposite
 * forces (Sec. 5.2, the force on the fluid is -I* F^h).
 * h_out[0] = sum_x rho - N rho0, h_out[1..3] = fluid momentum sum_x rho u of
 * the physical state (Sec. 4), h_out[4..6] = particle momentum sum_p m_p v_p
 * (0 for IB).  h_out is a host array of 7.  Synchronous (waits for the
 * context stream). */
lb_status lb_totals(lb_ctx* ctx, double h_out[7]);

/* Kernel timing for measurement: with max_passes > 0, of the fused lattice
 * passes that follow, the first and then one in every `stride` (>= 1) is
 * bracketed by a pair of HIP events recorded on the context stream, up to
 * max_passes timed passes (host-side event objects; no device memory); 0
 * disables.  Each event pair costs a few microseconds of idle pipeline, so a
 * stride above 1 keeps the measurement from slowing the run it measures.
 * lb_timing_read waits for the stream and returns the summed event time of
 * the timed passes (ms) and their number, then resets the count.  EINVAL for
 * a negative or huge max_passes or a stride outside [1, 2^20]. */
lb_status lb_timing(lb_ctx* ctx, int32_t max_passes, int32_t stride);
lb_status lb_timing_read(lb_ctx* ctx, double* lattice_ms, int64_t* passes);

/* Number of particles and time steps taken so far (host-side counters, no
 * device work). */
lb_status lb_info(const lb_ctx* ctx, int64_t* nparticles, int64_t* steps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lb_create
 * with the workspace taken from a static device array of the library instead
 * of the caller, 64 MiB per GPU (held by each GPU the library runs on until
 * the process ends).  Allocates no device memory.  At most one context made
 * this way is alive per device at a time (they would share the array):
 * another call on the same device returns LB_EBUSY until lb_destroy of the
 * first; contexts made by lb_create are unaffected.  The array keeps the
 * last context's contents; the call initialises everything the context reads
 * (as lb_create does).  The caller must not use the context from two threads
 * or streams at once (calls that overlap on one device race on the array).
 * Errors: LB_ENOMEM when lb_workspace_size of this box exceeds 64 MiB,
 * LB_EBUSY as above, LB_EINVAL and LB_EDEVICE as lb_create.  Every other
 * call works on the context as on one made by lb_create. */
lb_status lb_create_static(const lb_grid* g, const lb_params* p, const lb_limits* lim,
                           void* hip_stream, lb_ctx** out);

/* Frees the host-side context (the workspace and stream stay the caller's;
 * a lb_create_static context releases the device's static array). */
lb_status lb_destroy(lb_ctx* ctx);
/* Message of the last failed call on ctx (NULL: of a failed creation). */
const char* lb_last_error(const lb_ctx* ctx);
/* Text of a status code. */
const char* lb_status_string(lb_status s);

/* ------------------------------------------------------------------------
 * Ensembles: many independent periodic boxes (the same time step as above,
 * Alg. 3 ordering, force coupling / modified EBF / no coupling, free
 * particles) resident in one caller-owned pool and advanced together.  Each
 * step is one batched lattice launch over every live box plus one batched
 * launch per coupling half, replayed from captured HIP graphs.  Boxes have
 * their own grid, tau, body force, particles and step budget; a box stops
 * when its budget is spent while the others continue.
 * ------------------------------------------------------------------------ */
typedef struct lb_ensemble lb_ensemble;

/* Device bytes one box occupies in the pool (its admission footprint): the
 * same workspace as lb_workspace_size. */
lb_status lb_ensemble_footprint(const lb_grid* g, const lb_params* p, const lb_limits* lim,
                                size_t* bytes);

/* Creates an ensemble (the batching form: independent runs of the method of
 * Sec. 5.2 stepped together) over the borrowed device pool d_pool (256-byte
 * aligned, kept alive by the caller until lb_ensemble_destroy) for at most
 * max_slots boxes, all with the given storage precision and delta kernel and
 * the given spreading mode (deterministic 0 or 1, which every admitted box's
 * lb_params.deterministic must match, see there).
 * Every operation on the ensemble and on its slots is ordered on hip_stream
 * (a hipStream_t the caller keeps alive until lb_ensemble_destroy; the batched
 * steps are captured from it into HIP graphs, so it must not be the legacy
 * null stream).  With hip_stream NULL the ensemble creates its own blocking
 * default-priority stream and destroys it with the ensemble.
 * lb_ensemble_stream returns the stream in use.  Errors: LB_EINVAL (pool
 * misaligned, max_slots outside [1, 65536], unknown storage or kernel),
 * LB_ENOMEM (pool smaller than the slot tables), LB_EDEVICE. */
lb_status lb_ensemble_create(void* d_pool, size_t bytes, int32_t max_slots, int32_t storage,
                             int32_t kernel, int32_t deterministic, void* hip_stream,
                             lb_ensemble** out);
/* The stream the ensemble's work is ordered on (the caller's, or its own). */
lb_status lb_ensemble_stream(lb_ensemble* e, void** stream);

/* Admits a box with a budget of nsteps time steps.  Returns its slot and a
 * context handle for the slot (lb_init_fluid, lb_set_particles, lb_moments,
 * lb_populations, lb_get_particles, lb_totals work on it; particles must be
 * set before the slot's first ensemble step; lb_step is not valid on it).
 * The box starts at rest.  Errors: LB_EBUSY when no slot is free or its
 * footprint does not fit in the free pool memory (the caller may retry after a
 * retirement); LB_EINVAL for walls, IB, sub-stepping, bonds, shells, or a
 * storage / kernel different from the ensemble's. */
lb_status lb_ensemble_admit(lb_ensemble* e, const lb_grid* g, const lb_params* p,
                            const lb_limits* lim, int64_t nsteps, int32_t* slot, lb_ctx** ctx);

/* Advances every live box by nsteps time steps of Eq. fc-splitting in the
 * ordering of Alg. 3 (boxes whose budget is spent do not move).  Asynchronous
 * on the ensemble stream.  Errors: LB_EINVAL for nsteps < 0, LB_EDEVICE. */
lb_status lb_ensemble_step(lb_ensemble* e, int64_t nsteps);

/* Waits for the ensemble stream and reports the steps a slot has taken and
 * whether its budget is spent; also brings the slot's context up to date for
 * lb_moments and the other queries.  Synchronous. */
lb_status lb_ensemble_query(lb_ensemble* e, int32_t slot, int64_t* steps_done, int32_t* done);

/* Frees a slot and its pool memory (its context handle becomes invalid).
 * Errors: LB_EINVAL for a slot that is not live. */
lb_status lb_ensemble_retire(lb_ensemble* e, int32_t slot);

/* Times steps_per_candidate real steps of the live mix under each candidate
 * persistent-grid shape of the batched particle launches, keeps the fastest
 * and returns it (lat_grid: the lattice launch, one block per 256-site work
 * item, reported as it is).  The tuning steps count against the boxes'
 * budgets. */
lb_status lb_ensemble_autotune(lb_ensemble* e, int32_t steps_per_candidate, int32_t* lat_grid,
                               int32_t* part_grid);

/* Waits for the ensemble stream, frees every slot and the host-side state
 * (the pool and a borrowed stream stay the caller's). */
lb_status lb_ensemble_destroy(lb_ensemble* e);
/* Message of the last failed call on e (NULL: of a failed lb_ensemble_create). */
const char* lb_ensemble_last_error(const lb_ensemble* e);

#ifdef __cplusplus
}
#endif
#endif /* LBC_H */
