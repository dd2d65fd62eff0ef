// lbc_internal.h -- argument blocks and launchers shared by the host runtime
// (lbc_api.hip) and the kernels (lbc_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbc.h"

namespace lbc {

// Lattice geometry passed to every kernel.
struct Geo {
  int nx, ny, nz;
  int wall;  // halfway bounce-back walls in y
  int wpr;   // 64-bit force-mask words per row
  long long N;
  long long ps;  // population stride: N rounded up to a multiple of 128 sites, so that
                 // every population array starts on a 256-byte boundary
};

struct BondArgs {
  Geo g;
  const int32_t* perm;   // particles ordered by group
  const int32_t* loc;    // slot of each particle inside its group
  const int32_t* goff;   // group offsets into perm
  const int32_t* start;  // CSR of bond partners (global particle indices)
  const int32_t* nbr;
  double* pos;
  double* vel;
  const double* mass;
  double* fint;
  double k, r0;
  int type;
};

// Fused lattice pass (stream, both pending half forces, collide).
struct LatArgs {
  Geo g;
  const void* fin;  // f* of the previous pass
  void* fout;       // f* of this pass
  void* FA;         // first-half coupling force of this step (vec4 per site)
  void* FB;         // second-half coupling force of the previous step
  uint64_t* mask;   // per-site flag: FA or FB nonzero
  double rho0;
  double Fx, Fy, Fz;  // body force times the number of pending halves (1 or 2)
  double omp, omm;    // 1 - lambda for even / odd non-conserved moments
  float scale, inv;   // 16-bit storage scale 2^p and its inverse (1 otherwise)
  double uin[3];      // storage reference velocity of fin (comoving frame; 0 otherwise)
  double uout[3];     // storage reference velocity of fout
  double cm[40];      // comoving reference terms of the pass (comoving_terms)
  float cmf[40];      // the same in FP32
  double rnx, rny;    // 1/nx, 1/ny (linear-site pass)
  int clear_mask;     // clear the force mask after reading it (every kMaskKeep steps)
  int ib_copy;        // immersed boundary: FA becomes the pending FB (same spread)
  // fluctuating collision (noise != 0): S sqrt(mu lambda (2 - lambda)) for the
  // even / odd moments, generator key, step index
  int noise;
  double ap, am;
  uint32_t key0, key1, t0, t1;
  // general MRT (mrt != 0): rate of each moment group (bulk, shear, vector
  // ghosts, pseudo-vector ghosts, scalar ghost, tensor ghosts) and the noise
  // amplitude S sqrt(mu lambda (2 - lambda)) of each group
  int mrt;
  double lg[6], ag[6];
  int occ_lds;  // dynamic LDS bytes reserved per workgroup (occupancy cap), 0: none
  // Intrinsic-force sub-steps run by extra workgroups of the same launch
  // (bond_groups > 0), each doing bond_nsub velocity-Verlet sub-steps of
  // bond_dt for one bond group.  Row-mapped pass: the workgroups of the first
  // z slab (blockIdx.z == 0) take group blockIdx.y * gridDim.x + blockIdx.x
  // and the lattice rows are at blockIdx.z - 1; linear-site pass: workgroup b
  // < bond_groups takes group b and the sites start at workgroup bond_groups.
  // They touch only particle state, the pass only fluid state.
  // Viscous stress output (non-null): sigma [6][N] in the compute precision,
  // (1 - lambda_+/2) sum_i (f_i - f^eq_i) c_i c_i of the pulled state, sp = 1 - lambda_+/2
  void* sigma;
  double sp;
  BondArgs bond;
  int bond_groups, bond_nsub;
  int bond_cap;  // particles per bond group at most (needs that many lanes and 24 B of LDS each)
  double bond_dt;
};

struct InitArgs {
  Geo g;
  void* f;
  const double* rho;
  const double* u;
  double rho0;
  float scale;
};

// Read access to the stored state for moments at a site.
struct SiteArgs {
  Geo g;
  const void* f;
  const void* FB;
  double rho0;
  double pfx, pfy, pfz;  // pending body force (0 before the first step, F_ext after)
  float inv;
  double uref[3];  // storage reference velocity of f (comoving frame; 0 otherwise)
};

struct PartArgs {
  SiteArgs s;
  void* FA;
  void* FB;  // writable alias of s.FB
  uint64_t* mask;
  int K;  // delta kernel points (2, 3, 4)
  long long n;
  double* pos;
  double* vel;
  const double* mass;
  double* fint;
  double* aux;  // IB predictor positions
  double gamma;
  double fext[3];   // body-force density the fluid feels over the coupling step; it
                    // enters the implicit force-coupling solve as +(beta/2) F_ext
  int coupling;
  int use_fint;     // F_int enters the coupling force and the kick (Alg. 3)
  int phys;         // interpolate the physical velocity (with pending FB)
  int target;       // spread into FA (0) or FB (1)
  int drift_before;  // first P^1/2 of Alg. 3 (when no intrinsic forces sit between)
  int drift_after;   // final P^1/2 of Alg. 3
  // random force of the force coupling (kT > 0): generator key, step index and
  // the index of this coupling step within the step
  double kT;
  uint32_t key0, key1, t0, t1;
  int jc;
  double hh;         // coupling step length: h/2 (half steps) or h/2n (coupled sub-steps)
  double hd;         // length of drift_before / drift_after
  int fa_rd;         // the interpolated momentum also takes (h/2) FA (earlier sub-steps)
  double sw;         // scale of the lattice force written: 1, or 2 hh for sub-steps
  double* defer;     // non-null: store the lattice force per particle [n][3] here for a
                     // separate (deterministic) spread
  // Moment cache: the second coupling half stores, per particle and stencil
  // node, the moments it gathered; the next step's first half reads the same
  // populations (no lattice pass in between) and reuses them when the
  // particle's first stencil node is unchanged.
  double4* mcache;  // [n][L] (drho, j) of each node, before the pending force
  int4* mbase;      // [n] first stencil node (x, y, z) of the cached entries
  int cache_use;    // first half: cached entries are current
  int cache_fill;   // second half: store the gathered moments
};

// A coupled sub-step of the multiple time-step split with the coupling inside
// (Eq. multistep) as one launch.  The particle state is read from one buffer
// pair and written to the other, so that a particle takes its bond partners'
// midpoint positions from their start-of-sub-step state while they advance.
// The lattice force of a sub-step that later sub-steps of the same side read
// goes into a field of its own (gout), and the interpolation adds the target
// field and the fields of the earlier sub-steps (gin): a sub-step never sees
// its own spreads.  A fold launch moves those fields into the target field
// at the flagged sites.
constexpr int kMtsFields = 4;  // sub-step fields held before a fold
constexpr int kSubPartners = 3;  // bond partners a sub-step holds in registers

struct SubArgs {
  const double* pin;
  const double* vin;
  double* pout;
  double* vout;
  const void* gin[kMtsFields];  // fields of the earlier sub-steps of this side
  int ngin;
  void* gout;    // null: spread into the target field
  int bonds;     // F_int from the bond partners at the midpoints
  const int4* pn;  // per particle: up to kSubPartners partners (x, y, z) and the
                   // partner count (w); more partners: the CSR list in b
  BondArgs b;
};

struct ShellArgs {
  Geo g;
  const double* pos;
  const double* tmpl;
  double* fint;
  double* rot;
  int M;
  double k;
};

// Binning of markers into 8^3 tiles (counting sort) for LDS-staged
// interpolation and spreading.
struct TileArgs {
  Geo g;
  int tx, ty, tz, ntiles;
  int* count;   // [ntiles]
  int* start;   // [ntiles + 1]
  int* cursor;  // [ntiles]
  int* occ;     // occupied tiles in increasing order
  int* nocc;    // [1]
  int* ptile;   // tile of every marker
  int* sorted;  // markers grouped by tile
  uint64_t* mask;
};

hipError_t launch_bin(const TileArgs& t, const double* pos, long long n, hipStream_t st);
// Interpolation from the velocity of the flagged sites; redo = false leaves
// the listed markers to launch_shell_redo_forces (a marker set of whole
// shells), which redoes them and then computes the tether forces.
hipError_t launch_flag_interp(int storage, int K, const SiteArgs& s, const uint64_t* mask,
                              void* U, uint32_t stamp, const double* at, double* pos, double* aux,
                              int mode, long long n, int* miss, bool all_miss, bool redo,
                              hipStream_t st);
hipError_t launch_shell_redo_forces(int storage, int K, const ShellArgs& sa, int nshell,
                                    const SiteArgs& s, const void* U, uint32_t stamp,
                                    const double* at, double* pos, double* aux, int mode,
                                    int* miss, hipStream_t st);
hipError_t launch_tile_spread(int storage, int K, const TileArgs& t, const double* at,
                              const double* F, void* field, long long n, hipStream_t st);

// One ensemble member as the batched kernels see it (device memory).  The
// fields cur, pend and steps_done are advanced on the device only.
struct EnsSlot {
  Geo g;  // wpr == 0: linear force mask
  double rnx, rny;  // 1/nx, 1/ny for the site decomposition
  void* f[2];
  void* FA;
  void* FB;
  uint64_t* mask;
  double* pos;
  double* vel;
  const double* mass;
  long long np;
  double rho0, fx, fy, fz;
  double omp, omm, gamma;
  float scale, inv;
  int collision, coupling;
  int cur, pend;
  long long steps_done, steps_target;
  int live;
  int comoving;
  double uref[3];  // storage reference velocity of f[cur]
  double4* mcache;  // coupling moment cache (see PartArgs)
  int4* mbase;
  int mvalid;       // the cache holds the state of f[cur]
  double cm[40];    // comoving reference terms of the next pass (comoving_terms)
  float cmf[40];    // the same in FP32
  int det_on;       // deterministic spreading: lattice forces stored in aux, summed in det
  double* aux;      // [np][3]
  uint64_t* det;    // [N][3][2] fixed-point accumulator
};

struct EnsArgs {
  EnsSlot* slots;
  int nslots;
  const int2* litems;  // (slot, 256-site chunk)
  const int* nlitems;
  const int2* pitems;  // (slot, first particle of a 256-lane group block)
  const int* npitems;
};

// det: the deterministic spreading kernels run after each coupling half
hipError_t launch_ens_step(int storage, int K, const EnsArgs& e, int lat_grid, int part_grid,
                           int det, hipStream_t st);

hipError_t launch_stream_collide(int storage, bool comoving, const LatArgs& a, hipStream_t st);
hipError_t launch_init(int storage, const InitArgs& a, hipStream_t st);
hipError_t launch_moments(int storage, const SiteArgs& a, double* rho, double* u, hipStream_t st);
// gp, gm: factors of the even and odd non-equilibrium parts (1, 1: the
// physical populations; sqrt(1 - lambda+-): the collide-stream-collide state).
hipError_t launch_populations(int storage, const SiteArgs& a, double* out, double gp, double gm,
                              hipStream_t st);
// pref: factor of the traceless part; prefb: factor of the trace part
hipError_t launch_stress(int storage, const SiteArgs& a, double* out, double pref, double prefb,
                         hipStream_t st);
hipError_t launch_totals(int storage, const SiteArgs& a, double* partial, int nblk,
                         const double* vel, const double* mass, long long np, double* out,
                         hipStream_t st);
hipError_t launch_drift(const Geo& g, long long n, double* pos, const double* vel, double dt,
                        hipStream_t st);
hipError_t launch_wrap(const Geo& g, long long n, double* pos, hipStream_t st);
// Zeroes bytes (a multiple of 8) at p with a fill kernel.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_couple_half(int storage, const PartArgs& a, hipStream_t st);
// One coupled sub-step (SubArgs); and the fold: the nf fields u.gin moved
// into the target field of a (a.target) at the flagged sites and left zero.
hipError_t launch_mts_substep(int storage, const PartArgs& a, const SubArgs& u, hipStream_t st);
hipError_t launch_mts_fold(int storage, const PartArgs& a, const SubArgs& u, int nf,
                           hipStream_t st);
// Deterministic spreading: W F of every particle (positions X, lattice forces
// F [n][3]) into the 128-bit fixed-point accumulator acc [N][3][2], flagging
// the sites (and the closing drift if a.drift_after); then field += the sums
// at every flagged site and acc back to zero there.
hipError_t launch_spread_det(const PartArgs& a, const double* X, const double* F, uint64_t* acc,
                             hipStream_t st);
hipError_t launch_det_finalize(int storage, const Geo& g, const uint64_t* mask, uint64_t* acc,
                               void* field, hipStream_t st);
hipError_t launch_ib_predict(int storage, const PartArgs& a, hipStream_t st);
hipError_t launch_ib_advect(int storage, const PartArgs& a, int spread_fint, hipStream_t st);
hipError_t launch_bond_groups(const BondArgs& b, int ngroups, int gcap, int mode, int acc,
                              int nsub, double dt, hipStream_t st);
hipError_t launch_shell_forces(const ShellArgs& s, int nshell, hipStream_t st);

constexpr int kTotalsBlocks = 1024;

}  // namespace lbc
