// lbc_api.hip -- host runtime behind include/lbc.h: parameter checks, the
// workspace layout (all device memory belongs to the caller), bonded-group
// construction, and the per-step kernel sequence of each coupling scheme.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "lbc_device.h"
#include "lbc_internal.h"

using namespace lbc;

namespace {

thread_local std::string g_last_error;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int storage_bytes(int s) { return s == LB_F64 ? 8 : (s == LB_F32 ? 4 : 2); }
int force_vec_bytes(int s) { return s == LB_F64 ? 32 : 16; }

// Sequential carving of the workspace; with base == nullptr only sizes.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t bytes) {
    T* p = base ? (T*)(base + off) : nullptr;
    off = align256(off + bytes);
    return p;
  }
};

struct Layout {
  void* f[2];
  void *FA, *FB;
  uint64_t* mask;
  double *pos, *vel, *mass, *fint, *aux;
  int32_t *perm, *loc, *goff, *bstart, *bnbr;
  double *tmpl, *rot, *partial, *tot;
  int *tcount, *tstart, *tcursor, *tocc, *tnocc, *ptile, *psorted;
  double4* mcache;
  int4* mbase;
  uint64_t* det;  // fixed-point spreading accumulator [N][3][2] (deterministic mode)
  void* U;        // velocity at the flagged sites [N][4] (binned immersed boundary)
  int* miss;      // markers left to the gathering interpolation: 2 counters, then the list
  // coupling-inside sub-steps: second state buffer pair and the lattice-force
  // fields of the sub-steps before a fold
  double *pos2, *vel2;
  int4* pn;  // packed bond partners (SubArgs::pn)
  void* G[kMtsFields];
  size_t bytes;
};

int kernel_lanes(int K) { return K == 2 ? 8 : (K == 3 ? 32 : 64); }

// 64-bit force-mask words allocated for a box (enough for both layouts).
size_t mask_words(const lb_grid& g) { return (size_t)g.nz * g.ny * ((g.nx + 63) / 64); }

int tiles_along(int n) { return (n + 7) / 8; }

// Sites between consecutive population arrays: N rounded up to 128 sites, so
// that each array starts 256-byte aligned in every storage precision and a
// wavefront of 64 consecutive sites never straddles two cache lines for lack
// of alignment of the array itself.
long long pop_stride(long long N) { return (N + 127) / 128 * 128; }

Layout carve(const lb_grid& g, const lb_params& p, const lb_limits& lim, void* base) {
  Carver c{(char*)base};
  Layout L{};
  const long long N = (long long)g.nx * g.ny * g.nz;
  const size_t fb = (size_t)19 * pop_stride(N) * storage_bytes(p.storage);
  L.f[0] = c.take<void>(fb);
  L.f[1] = c.take<void>(fb);
  L.FA = c.take<void>((size_t)N * force_vec_bytes(p.storage));
  L.FB = c.take<void>((size_t)N * force_vec_bytes(p.storage));
  L.mask = c.take<uint64_t>(mask_words(g) * 8);
  const size_t np = (size_t)std::max<int64_t>(lim.max_particles, 1);
  L.pos = c.take<double>(np * 24);
  L.vel = c.take<double>(np * 24);
  L.mass = c.take<double>(np * 8);
  L.fint = c.take<double>(np * 24);
  L.aux = c.take<double>(np * 24);
  L.perm = c.take<int32_t>(np * 4);
  L.loc = c.take<int32_t>(np * 4);
  L.goff = c.take<int32_t>((np + 1) * 4);
  L.bstart = c.take<int32_t>((np + 1) * 4);
  L.bnbr = c.take<int32_t>((size_t)std::max<int64_t>(2 * lim.max_bonds, 1) * 4);
  L.tmpl = c.take<double>((size_t)std::max(lim.max_shell_size, 1) * 24);
  L.rot = c.take<double>((size_t)std::max(lim.max_shells, 1) * 72);
  L.partial = c.take<double>((size_t)kTotalsBlocks * 4 * 8);
  L.tot = c.take<double>(8 * 8);
  const size_t nt = (size_t)tiles_along(g.nx) * tiles_along(g.ny) * tiles_along(g.nz);
  L.tcount = c.take<int>(nt * 4);
  L.tstart = c.take<int>((nt + 1) * 4);
  L.tcursor = c.take<int>(nt * 4);
  L.tocc = c.take<int>(nt * 4);
  L.tnocc = c.take<int>(64);
  L.ptile = c.take<int>(np * 4);
  L.psorted = c.take<int>(np * 4);
  const bool cached = p.coupling == LB_COUPLE_FC || p.coupling == LB_COUPLE_EBF;
  L.mcache = c.take<double4>(cached ? np * kernel_lanes(p.kernel) * 32 : 32);
  L.mbase = c.take<int4>(cached ? np * 16 : 16);
  L.det = c.take<uint64_t>(p.deterministic ? (size_t)N * 48 : 64);
  const bool binned = p.coupling == LB_COUPLE_IB && p.kernel >= 3;
  L.U = c.take<void>(binned ? (size_t)N * 4 * (p.storage == LB_F64 ? 8 : 4) : 64);
  L.miss = c.take<int>(binned ? (np + 2) * 4 : 64);
  const bool sub = p.mts_inside && p.mts_substeps > 0 && !p.deterministic;
  const int nf = sub ? std::min(p.mts_substeps - 1, kMtsFields) : 0;
  L.pos2 = c.take<double>(sub ? np * 24 : 64);
  L.vel2 = c.take<double>(sub ? np * 24 : 64);
  L.pn = c.take<int4>(sub ? np * 16 : 64);
  for (int f = 0; f < kMtsFields; ++f)
    L.G[f] = f < nf ? c.take<void>((size_t)N * force_vec_bytes(p.storage)) : nullptr;
  L.bytes = c.off;
  return L;
}

bool check_params(const lb_grid* g, const lb_params* p, const lb_limits* lim, std::string& err) {
  if (!g || !p || !lim) return err = "null argument", false;
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return err = "grid dimensions must be >= 1", false;
  if ((long long)g->nx * g->ny * g->nz >= (1ll << 32))
    return err = "grid too large (at most 2^32 - 1 sites)", false;
  if (g->wall_y != 0 && g->wall_y != 1) return err = "wall_y must be 0 or 1", false;
  if (g->wall_y && g->ny < 2) return err = "a walled channel needs ny >= 2", false;
  if (!(p->tau > 0.5) || !std::isfinite(p->tau))
    return err = "tau (lattice relaxation time) must be > 1/2", false;
  if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return err = "rho0 must be > 0", false;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->body_force[a])) return err = "body force must be finite", false;
  if (p->collision != LB_BGK && p->collision != LB_TRT && p->collision != LB_MRT)
    return err = "unknown collision", false;
  if (p->collision == LB_MRT) {
    for (int k = 0; k < 5; ++k)
      if (!(p->mrt_rates[k] > 0.0 && p->mrt_rates[k] < 2.0))
        return err = "mrt_rates must lie in (0, 2)", false;
    if (p->csc) return err = "the collide-stream-collide output takes the two-rate collision", false;
    if (p->comoving) return err = "the comoving storage frame takes the two-rate collision", false;
  }
  if (p->forcing != LB_FORCING_SPLIT2) return err = "unknown forcing scheme", false;
  if (p->coupling < LB_COUPLE_NONE || p->coupling > LB_COUPLE_IB)
    return err = "unknown coupling", false;
  if ((p->coupling == LB_COUPLE_FC || p->coupling == LB_COUPLE_EBF) &&
      (!(p->gamma > 0.0) || !std::isfinite(p->gamma)))
    return err = "force coupling needs gamma > 0", false;
  if (p->kernel < 2 || p->kernel > 4) return err = "kernel must be 2, 3 or 4", false;
  if (p->storage < LB_F64 || p->storage > LB_BF16) return err = "unknown storage", false;
  if (p->f16_scale_log2 < -40 || p->f16_scale_log2 > 40)
    return err = "f16_scale_log2 out of range", false;
  if (p->mts_substeps < 0 || p->mts_substeps > 256) return err = "mts_substeps out of range", false;
  if (p->ib_rebin < 0) return err = "ib_rebin must be >= 0", false;
  if (p->mts_substeps > 0 && p->coupling == LB_COUPLE_IB)
    return err = "multiple time stepping applies to force coupling only", false;
  if (p->mts_inside != 0 && p->mts_inside != 1) return err = "mts_inside must be 0 or 1", false;
  if (!(p->kT >= 0.0) || !std::isfinite(p->kT)) return err = "kT must be finite and >= 0", false;
  if (p->kT > 0.0 && p->csc)
    return err = "the collide-stream-collide output is not defined for a fluctuating fluid", false;
  if (p->kT > 0.0 && p->comoving)
    return err = "the comoving storage frame is not combined with thermal fluctuations", false;
  if (p->mts_inside && p->mts_substeps < 1)
    return err = "mts_inside needs mts_substeps >= 1", false;
  if (p->deterministic != 0 && p->deterministic != 1) return err = "deterministic must be 0 or 1", false;
  if (p->comoving != 0 && p->comoving != 1) return err = "comoving must be 0 or 1", false;
  if (p->comoving && g->wall_y)
    return err = "the comoving storage frame needs a periodic box (walls break uniform flow)", false;
  if (p->csc != 0 && p->csc != 1) return err = "csc must be 0 or 1", false;
  if (p->csc) {  // the exact half collision sqrt(1 - lambda) needs every rate <= 1
    const double magic = p->trt_magic > 0 ? p->trt_magic : 3.0 / 16.0;
    if (p->tau < 1.0) return err = "the collide-stream-collide form needs tau >= 1", false;
    if (p->collision == LB_TRT && 0.5 + magic / (p->tau - 0.5) < 1.0)
      return err = "the collide-stream-collide form needs trt_magic >= (tau - 1/2)/2", false;
  }
  if (lim->max_particles < 0 || lim->max_particles > (1ll << 30) || lim->max_bonds < 0 ||
      lim->max_bonds > (1ll << 29) || lim->max_shells < 0 || lim->max_shell_size < 0)
    return err = "invalid limits", false;
  return true;
}

// Steps between two binnings of IB markers into tiles.
constexpr int64_t kRebin = 32;  // default steps between two marker binnings

}  // namespace

struct lb_ctx {
  lb_grid g;
  lb_params p;
  lb_limits lim;
  hipStream_t st;
  Geo geo;
  Layout L;
  int cur = 0;
  int pend = 0;
  int64_t steps = 0;
  int64_t np = 0;
  int64_t nbond = 0;
  std::vector<int32_t> bonds;
  double bond_k = 0, bond_r0 = 1;
  int bond_type = LB_HARMONIC;
  bool groups_dirty = true;
  int ngroups = 0, gcap = 64;
  bool tiled = false;   // binned LDS-staged particle path (dense IB markers)
  int64_t binned_at = -1;  // step of the last marker binning (-1: markers changed since)
  bool adv_pending = false;  // tiled IB: the final half advection of the last step is due
  uint32_t ustamp = 0;  // tiled IB: stamp of the last velocity pass over the flagged sites
  bool flags_follow = false;  // tiled IB: the force mask holds the markers' last stencils
  bool member = false;  // slot of an ensemble: stepped only by lb_ensemble_step
  bool running = false;  // ensemble slot whose device record has been uploaded
  bool mvalid = false;   // coupling moment cache holds the state of f[cur]
  int lds_cu = 0;        // LDS bytes per compute unit (for the lattice-pass occupancy cap)
  int nshell = 0, shell_size = 0;
  double k_tether = 0;
  double omp = 0, omm = 0;
  float scale = 1.f, inv = 1.f;
  double uref[3] = {0, 0, 0};  // storage reference velocity of f[cur] (comoving frame)
  std::vector<hipEvent_t> ev;  // timing event pairs
  int32_t ev_used = 0;
  int32_t ev_stride = 1;   // time one pass in every ev_stride
  int64_t ev_seen = 0;     // passes since timing was armed
  int static_dev = -1;     // device whose static array holds the workspace (lb_create_static)
  void* sweep = nullptr;   // lb_stress_sweep output: stress of each pass's starting state
  std::string err;
};

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);                  \
      return LB_EDEVICE;                                                               \
    }                                                                                  \
  } while (0)

static lb_status fail(lb_ctx* ctx, lb_status s, const std::string& m) {
  if (ctx)
    ctx->err = m;
  else
    g_last_error = m;
  return s;
}

static SiteArgs site_args(const lb_ctx* c) {
  SiteArgs s;
  s.g = c->geo;
  s.f = c->L.f[c->cur];
  s.FB = c->L.FB;
  s.rho0 = c->p.rho0;
  s.pfx = c->pend * c->p.body_force[0];
  s.pfy = c->pend * c->p.body_force[1];
  s.pfz = c->pend * c->p.body_force[2];
  s.inv = c->inv;
  for (int k = 0; k < 3; ++k) s.uref[k] = c->uref[k];
  return s;
}

static PartArgs part_args(const lb_ctx* c) {
  PartArgs a;
  a.s = site_args(c);
  a.FA = c->L.FA;
  a.FB = c->L.FB;
  a.mask = c->L.mask;
  a.K = c->p.kernel;
  a.n = c->np;
  a.pos = c->L.pos;
  a.vel = c->L.vel;
  a.mass = c->L.mass;
  a.fint = c->L.fint;
  a.aux = c->L.aux;
  a.gamma = c->p.gamma;
  for (int k = 0; k < 3; ++k) a.fext[k] = c->p.body_force[k];
  a.coupling = c->p.coupling;
  a.use_fint = 0;
  a.phys = 1;
  a.target = 0;
  a.drift_before = 0;
  a.drift_after = 0;
  a.mcache = c->L.mcache;
  a.mbase = c->L.mbase;
  a.cache_use = 0;
  a.cache_fill = 0;
  a.kT = c->p.coupling == LB_COUPLE_FC ? c->p.kT : 0.0;
  a.key0 = (uint32_t)c->p.seed;
  a.key1 = (uint32_t)(c->p.seed >> 32);
  a.t0 = (uint32_t)c->steps;
  a.t1 = (uint32_t)((uint64_t)c->steps >> 32);
  a.jc = 0;
  a.hh = 0.5;
  a.hd = 0.5;
  a.fa_rd = 0;
  a.sw = 1.0;
  a.defer = nullptr;
  return a;
}

static TileArgs tile_args(const lb_ctx* c) {
  TileArgs t;
  t.g = c->geo;
  t.tx = tiles_along(c->geo.nx);
  t.ty = tiles_along(c->geo.ny);
  t.tz = tiles_along(c->geo.nz);
  t.ntiles = t.tx * t.ty * t.tz;
  t.count = c->L.tcount;
  t.start = c->L.tstart;
  t.cursor = c->L.tcursor;
  t.occ = c->L.tocc;
  t.nocc = c->L.tnocc;
  t.ptile = c->L.ptile;
  t.sorted = c->L.psorted;
  t.mask = c->L.mask;
  return t;
}

static BondArgs bond_args(const lb_ctx* c, double* pos) {
  BondArgs b;
  b.g = c->geo;
  b.perm = c->L.perm;
  b.loc = c->L.loc;
  b.goff = c->L.goff;
  b.start = c->L.bstart;
  b.nbr = c->L.bnbr;
  b.pos = pos;
  b.vel = c->L.vel;
  b.mass = c->L.mass;
  b.fint = c->L.fint;
  b.k = c->bond_k;
  b.r0 = c->bond_r0;
  b.type = c->bond_type;
  return b;
}

// Groups of whole bonded clusters (union-find), packed into blocks of at most
// gcap particles, plus a CSR list of bond partners.
static lb_status build_groups(lb_ctx* c) {
  const int64_t n = c->np;
  std::vector<int32_t> parent(n);
  std::iota(parent.begin(), parent.end(), 0);
  auto find = [&](int32_t x) {
    while (parent[x] != x) x = parent[x] = parent[parent[x]];
    return x;
  };
  std::vector<int32_t> deg(n + 1, 0);
  for (int64_t b = 0; b < c->nbond; ++b) {
    const int32_t i = c->bonds[2 * b], j = c->bonds[2 * b + 1];
    if (i < 0 || j < 0 || i >= n || j >= n)
      return fail(c, LB_EINVAL, "bond index outside the particle range");
    parent[find(i)] = find(j);
    deg[i]++;
    deg[j]++;
  }
  std::vector<int32_t> start(n + 1, 0);
  for (int64_t p = 0; p < n; ++p) start[p + 1] = start[p] + deg[p];
  std::vector<int32_t> nbr(std::max<int64_t>(2 * c->nbond, 1)), fill(start.begin(), start.end() - 1);
  for (int64_t b = 0; b < c->nbond; ++b) {
    const int32_t i = c->bonds[2 * b], j = c->bonds[2 * b + 1];
    nbr[fill[i]++] = j;
    nbr[fill[j]++] = i;
  }
  // members of each cluster in index order
  std::vector<int32_t> root(n), order(n);
  for (int64_t p = 0; p < n; ++p) root[p] = find((int32_t)p);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return root[a] < root[b]; });
  std::vector<std::pair<int32_t, int32_t>> clusters;  // (offset in order, size)
  for (int64_t k = 0; k < n;) {
    int64_t e = k;
    while (e < n && root[order[e]] == root[order[k]]) ++e;
    clusters.push_back({(int32_t)k, (int32_t)(e - k)});
    k = e;
  }
  int maxc = 1;
  for (auto& cl : clusters) maxc = std::max(maxc, cl.second);
  if (maxc > 1024) return fail(c, LB_EINVAL, "a bonded cluster has more than 1024 particles");
  const int gcap = std::max(128, ((maxc + 63) / 64) * 64);
  std::vector<int32_t> perm, loc(n), goff{0};
  std::vector<int4> pn;
  int fillg = 0;
  for (auto& cl : clusters) {
    if (fillg + cl.second > gcap) {
      goff.push_back((int32_t)perm.size());
      fillg = 0;
    }
    for (int k = 0; k < cl.second; ++k) {
      const int32_t p = order[cl.first + k];
      loc[p] = fillg + k;
      perm.push_back(p);
    }
    fillg += cl.second;
  }
  if (fillg > 0) goff.push_back((int32_t)perm.size());
  c->ngroups = (int)goff.size() - 1;
  c->gcap = gcap;
  if (n > 0) {
    HIPCHK(c, hipMemcpyAsync(c->L.perm, perm.data(), n * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->L.loc, loc.data(), n * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->L.goff, goff.data(), goff.size() * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->L.bstart, start.data(), (n + 1) * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->L.bnbr, nbr.data(), nbr.size() * 4, hipMemcpyHostToDevice, c->st));
    if (c->p.mts_inside && !c->p.deterministic) {  // the first partners in list order
      pn.assign(n, int4{0, 0, 0, 0});
      for (int64_t p = 0; p < n; ++p) {
        int32_t q[kSubPartners] = {0, 0, 0};
        for (int k = 0; k < kSubPartners && k < deg[p]; ++k) q[k] = nbr[start[p] + k];
        pn[p] = int4{q[0], q[1], q[2], deg[p]};
      }
      HIPCHK(c, hipMemcpyAsync(c->L.pn, pn.data(), n * 16, hipMemcpyHostToDevice, c->st));
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
  }
  c->groups_dirty = false;
  return LB_OK;
}

// F_int at the given positions: shell tethers and bonds (shells_done: the
// tether forces are already in fint).
static lb_status enqueue_fint(lb_ctx* c, double* pos, bool& any, bool shells_done = false) {
  any = shells_done;
  if (c->nshell > 0 && !shells_done) {
    const int64_t nm = (int64_t)c->nshell * c->shell_size;
    if (nm < c->np)
      HIPCHK(c, launch_zero(c->L.fint + 3 * nm, (size_t)(c->np - nm) * 24, c->st));
    ShellArgs s{c->geo, pos, c->L.tmpl, c->L.fint, c->L.rot, c->shell_size, c->k_tether};
    HIPCHK(c, launch_shell_forces(s, c->nshell, c->st));
    any = true;
  }
  if (c->nbond > 0) {
    HIPCHK(c, launch_bond_groups(bond_args(c, pos), c->ngroups, c->gcap, 0, any ? 1 : 0, 0, 0.0,
                                 c->st));
    any = true;
  }
  return LB_OK;
}

// P^(hd): r <- wrap(r + hd v) for every particle, then F_int at the new
// positions.  With bonds and no shells both run in one launch of the bond
// groups (every particle belongs to a group), else as a drift and enqueue_fint.
static lb_status drift_and_fint(lb_ctx* c, double hd, bool& any) {
  if (c->nshell == 0 && c->nbond > 0 && c->ngroups > 0) {
    HIPCHK(c, launch_bond_groups(bond_args(c, c->L.pos), c->ngroups, c->gcap, 2, 0, 0, hd, c->st));
    any = true;
    return LB_OK;
  }
  HIPCHK(c, launch_drift(c->geo, c->np, c->L.pos, c->L.vel, hd, c->st));
  return enqueue_fint(c, c->L.pos, any);
}

// Whether the 2n intrinsic-force sub-steps of the multiple time-step split can
// run as extra workgroups of the lattice launch: a bond group fits a
// workgroup, and on the row-mapped pass the groups fit one z slab of
// workgroups.
static bool bonds_in_pass(const lb_ctx* c) {
  if (c->ngroups <= 0) return false;
  if (c->geo.wpr == 0) return c->gcap <= 256;  // linear-site pass: 256-lane workgroups
  const int bx = std::min(256, (c->geo.nx + 63) / 64 * 64);
  const long long slab = (long long)((c->geo.nx + bx - 1) / bx) * c->geo.ny;
  return c->gcap <= bx && c->ngroups <= slab;
}

// bond_nsub > 0: the launch also runs bond_nsub sub-steps of bond_dt of every
// bond group (bonds_in_pass must hold).
static lb_status lattice_pass(lb_ctx* c, int bond_nsub = 0, double bond_dt = 0.0) {
  LatArgs a{};
  a.g = c->geo;
  a.fin = c->L.f[c->cur];
  a.fout = c->L.f[1 - c->cur];
  a.FA = c->L.FA;
  a.FB = c->L.FB;
  a.mask = c->L.mask;
  a.rho0 = c->p.rho0;
  const double fac = 1.0 + c->pend;
  a.Fx = fac * c->p.body_force[0];
  a.Fy = fac * c->p.body_force[1];
  a.Fz = fac * c->p.body_force[2];
  a.omp = c->omp;
  a.omm = c->omm;
  a.scale = c->scale;
  a.inv = c->inv;
  a.rnx = 1.0 / c->geo.nx;
  a.rny = 1.0 / c->geo.ny;
  a.clear_mask = c->steps % kMaskKeep == 0 ? 1 : 0;
  a.ib_copy = (c->p.coupling == LB_COUPLE_IB && c->np > 0) ? 1 : 0;
  a.noise = c->p.kT > 0.0 ? 1 : 0;
  {  // S sqrt(mu lambda (2 - lambda)), mu = k_B T / c_s^2 = 3 k_B T
    const double lp = 1.0 - c->omp, lm = 1.0 - c->omm, mu = 3.0 * c->p.kT;
    a.ap = c->scale * std::sqrt(mu * lp * (2.0 - lp));
    a.am = c->scale * std::sqrt(mu * lm * (2.0 - lm));
  }
  a.key0 = (uint32_t)c->p.seed;
  a.key1 = (uint32_t)(c->p.seed >> 32);
  a.t0 = (uint32_t)c->steps;
  a.t1 = (uint32_t)((uint64_t)c->steps >> 32);
  // Occupancy cap of the pass.  Fewer resident wavefronts per CU keep fewer
  // of the 19 population streams open at once, which raised the streaming
  // rate of the deterministic pass: 20 waves per CU for FP32 (256^3: 452 ->
  // 435 us; 250^3 on the linear-site pass: 427 -> 408 us), 24 for 16-bit
  // storage (256^3 FP16: 229 -> 225 us).  Narrow rows stream best with fewer
  // still (FP32, 2^22 sites): 12 waves for 128-wide rows (122.4 -> 116.7 us
  // per step) and 8 for 64-wide rows (122.2 -> 114.6 us); 256-wide rows lose
  // 8 % below 20.  The cap is an unused dynamic LDS reservation per
  // workgroup.  Not for FP64 (no gain measured) nor with thermal noise (its
  // arithmetic needs the occupancy).
  a.occ_lds = 0;
  if (c->lds_cu > 0 && c->p.kT == 0.0 && c->p.storage != LB_F64) {
    const int bx = c->geo.wpr == 0 ? 256 : std::min(256, (c->geo.nx + 63) / 64 * 64);
    int waves_cu = c->p.storage == LB_F32 ? 20 : 24;
    if (c->p.storage == LB_F32 && bx == 64) waves_cu = 8;
    if (c->p.storage == LB_F32 && bx == 128) waves_cu = 12;
    const int groups = std::max(1, waves_cu / (bx / 64));
    a.occ_lds = (c->lds_cu / groups) & ~1023;
  }
  a.mrt = c->p.collision == LB_MRT ? 1 : 0;
  {  // group rates: bulk, shear, vector, pseudo-vector, scalar and tensor ghosts
    const double* r = c->p.mrt_rates;
    const double lg[6] = {r[0], 1.0 - c->omp, r[1], r[2], r[3], r[4]};
    for (int g = 0; g < 6; ++g) {
      a.lg[g] = lg[g];
      a.ag[g] = c->scale * std::sqrt(3.0 * c->p.kT * lg[g] * (2.0 - lg[g]));
    }
  }
  for (int k = 0; k < 3; ++k) {
    a.uin[k] = c->uref[k];
    a.uout[k] = c->uref[k] + (c->p.comoving ? c->p.body_force[k] / c->p.rho0 : 0.0);
  }
  comoving_terms(c->scale, c->p.rho0, a.uin, a.uout, a.cm, a.cmf);
  a.sigma = c->sweep;
  a.sp = 0.5 * (1.0 + c->omp);  // 1 - lambda_+/2
  if (bond_nsub > 0) {
    a.bond = bond_args(c, c->L.pos);
    a.bond_groups = c->ngroups;
    a.bond_nsub = bond_nsub;
    a.bond_dt = bond_dt;
    a.bond_cap = c->gcap;
    a.occ_lds = std::max(a.occ_lds, c->gcap * 3 * (int)sizeof(double));
  }
  const bool timed =
      2 * (size_t)c->ev_used + 1 < c->ev.size() && c->ev_seen++ % c->ev_stride == 0;
  if (timed) HIPCHK(c, hipEventRecord(c->ev[2 * c->ev_used], c->st));
  HIPCHK(c, launch_stream_collide(c->p.storage, c->p.comoving != 0, a, c->st));
  if (timed) HIPCHK(c, hipEventRecord(c->ev[2 * c->ev_used++ + 1], c->st));
  c->cur = 1 - c->cur;
  c->pend = 1;
  for (int k = 0; k < 3; ++k) c->uref[k] = a.uout[k];
  return LB_OK;
}

// Interpolation of the tiled IB path (modes of launch_flag_interp): the
// velocity pass over the flagged sites under a new stamp, then the markers.
// The field is cleared before a stamp is reused (every 2^32 - 1 calls), so
// that an entry carries the current stamp only if this call wrote it.
// redo = false: the listed markers are left to shell_forces_redo, which must
// follow with the same call's arguments.
static lb_status flag_interp(lb_ctx* c, const double* at, double* pos, double* aux, int mode,
                             bool redo = true) {
  if (++c->ustamp == 0xffffffffu) {
    HIPCHK(c, launch_zero(c->L.U, (size_t)c->geo.N * 4 * (c->p.storage == LB_F64 ? 8 : 4), c->st));
    c->ustamp = 1;
  }
  HIPCHK(c, launch_flag_interp(c->p.storage, c->p.kernel, site_args(c), c->L.mask, c->L.U,
                               c->ustamp, at, pos, aux, mode, c->np, c->L.miss, !c->flags_follow,
                               redo, c->st));
  return LB_OK;
}

// Whether the markers listed by a flag_interp call of the tiled path can be
// redone by the shells' workgroups: the markers are whole shells and the
// flags follow them (right after the fluid or the markers were set every
// marker is listed, which the grid of k_marker_slow handles better).
static bool redo_in_shells(const lb_ctx* c) {
  return c->nshell > 0 && (int64_t)c->nshell * c->shell_size == c->np && c->flags_follow;
}

// The listed markers of the last flag_interp call (same arguments) redone,
// then the tether forces at the positions pos_f (launch_shell_redo_forces).
static lb_status shell_forces_redo(lb_ctx* c, const double* at, double* pos, double* aux,
                                   int mode, double* pos_f) {
  ShellArgs s{c->geo, pos_f, c->L.tmpl, c->L.fint, c->L.rot, c->shell_size, c->k_tether};
  HIPCHK(c, launch_shell_redo_forces(c->p.storage, c->p.kernel, s, c->nshell, site_args(c),
                                     c->L.U, c->ustamp, at, pos, aux, mode, c->L.miss, c->st));
  return LB_OK;
}

// Complete a deferred final half advection of the tiled IB path, so that
// lb_step returns at a step boundary.
static lb_status finish_step(lb_ctx* c) {
  if (!c->adv_pending) return LB_OK;
  const lb_status s = flag_interp(c, c->L.aux, c->L.pos, c->L.aux, 1);
  if (s != LB_OK) return s;
  c->adv_pending = false;
  return LB_OK;
}

// One coupling step (k_couple_half).  In the deterministic mode the kernel
// stores each particle's lattice force instead of spreading it (into aux,
// unused by force coupling), and the fixed-point spread (with the closing
// drift, if any) and its finalize into the target field follow.
static lb_status couple(lb_ctx* c, const PartArgs& a) {
  if (!c->p.deterministic) {
    HIPCHK(c, launch_couple_half(c->p.storage, a, c->st));
    return LB_OK;
  }
  PartArgs b = a;
  b.defer = c->L.aux;
  b.drift_after = 0;
  HIPCHK(c, launch_couple_half(c->p.storage, b, c->st));
  PartArgs d = a;
  d.defer = nullptr;
  HIPCHK(c, launch_spread_det(d, c->L.pos, c->L.aux, c->L.det, c->st));
  HIPCHK(c, launch_det_finalize(c->p.storage, c->geo, c->L.mask, c->L.det,
                                a.target ? c->L.FB : c->L.FA, c->st));
  return LB_OK;
}

// Deterministic spread of the intrinsic forces at the IB predictor positions
// X~ (aux) into FA.
static lb_status spread_fint_det(lb_ctx* c) {
  PartArgs a = part_args(c);
  a.drift_after = 0;
  HIPCHK(c, launch_spread_det(a, c->L.aux, c->L.fint, c->L.det, c->st));
  HIPCHK(c, launch_det_finalize(c->p.storage, c->geo, c->L.mask, c->L.det, c->L.FA, c->st));
  return LB_OK;
}

// Multiple time stepping with the coupling inside (Eq. multistep): n coupled
// sub-steps of dt = h/2n on each side of the lattice pass.  A sub-step drifts
// dt/2, takes the intrinsic force at the midpoint, couples over dt (F^h, kick,
// lattice force) and drifts dt/2.  Its lattice force goes into FA (before the
// pass) or FB (after), scaled by 2 dt, so each field holds the impulse of its
// n sub-steps as a half-step force and the pass is unchanged.  The fluid
// velocity a sub-step sees is that of the populations with every force
// applied so far: the pending fields of the earlier sub-steps and k dt of the
// body force; after the pass the first sub-step sees the post-stream velocity
// (as the second half of Alg. 3).  Each sub-step is one launch (SubArgs):
// the first of a side spreads into the side's field, the later ones into
// fields of their own that the next interpolations add, folded into the
// side's field when kMtsFields are in use and at the end of the side.  The
// deterministic mode takes step_mts_inside_det.
static lb_status step_mts_inside_det(lb_ctx* c);

static lb_status step_mts_inside(lb_ctx* c) {
  if (c->p.deterministic) return step_mts_inside_det(c);
  const int n = c->p.mts_substeps;
  const double dt = 1.0 / (2.0 * n);
  double* const P[2] = {c->L.pos, c->L.pos2};
  double* const V[2] = {c->L.vel, c->L.vel2};
  lb_status s;
  for (int side = 0; side < 2; ++side) {
    if (side == 1 && (s = lattice_pass(c)) != LB_OK) return s;
    SubArgs u{};
    u.bonds = c->nbond > 0 ? 1 : 0;
    u.pn = c->L.pn;
    u.b = bond_args(c, c->L.pos);
    int used = 0;  // sub-step fields written since the last fold
    PartArgs a;
    for (int k = 0; k < n; ++k) {
      a = part_args(c);
      a.hh = dt;
      a.hd = 0.5 * dt;
      a.sw = 2.0 * dt;
      a.jc = side * n + k;
      a.use_fint = u.bonds;
      a.target = side;
      const double ext = (side == 0 ? c->pend : 0) + 2.0 * k * dt;  // body force applied, x h/2
      a.s.pfx = ext * c->p.body_force[0];
      a.s.pfy = ext * c->p.body_force[1];
      a.s.pfz = ext * c->p.body_force[2];
      a.phys = (side == 0 || k > 0) ? 1 : 0;  // side 1, k > 0: FB holds the earlier sub-steps
      a.fa_rd = (side == 0 && k > 0) ? 1 : 0;
      a.cache_fill = (side == 1 && k == 0) ? 1 : 0;
      a.cache_use = (side == 1 && k > 0) || (side == 0 && c->mvalid) ? 1 : 0;
      if (k > 0 && used == kMtsFields) {
        HIPCHK(c, launch_mts_fold(c->p.storage, a, u, used, c->st));
        used = 0;
      }
      const int i = side * n + k;  // 2n sub-steps: the state ends where it started
      u.pin = P[i & 1];
      u.vin = V[i & 1];
      u.pout = P[(i + 1) & 1];
      u.vout = V[(i + 1) & 1];
      for (int f = 0; f < kMtsFields; ++f) u.gin[f] = c->L.G[f];
      u.ngin = used;
      u.gout = k > 0 ? c->L.G[used] : nullptr;
      HIPCHK(c, launch_mts_substep(c->p.storage, a, u, c->st));
      if (k > 0) ++used;
    }
    if (used > 0) HIPCHK(c, launch_mts_fold(c->p.storage, a, u, used, c->st));
  }
  c->mvalid = true;
  return LB_OK;
}

// The deterministic mode: each sub-step as a launch of the bond forces, a
// coupling launch and the fixed-point spread of the lattice forces.
static lb_status step_mts_inside_det(lb_ctx* c) {
  const int n = c->p.mts_substeps;
  const double dt = 1.0 / (2.0 * n);
  const bool fint = c->nshell > 0 || c->nbond > 0;
  lb_status s;
  for (int side = 0; side < 2; ++side) {
    if (side == 1 && (s = lattice_pass(c)) != LB_OK) return s;
    for (int k = 0; k < n; ++k) {
      bool any = false;
      if (fint && (s = drift_and_fint(c, 0.5 * dt, any)) != LB_OK) return s;
      PartArgs a = part_args(c);
      a.hh = dt;
      a.hd = 0.5 * dt;
      a.sw = 2.0 * dt;
      a.jc = side * n + k;
      a.use_fint = any ? 1 : 0;
      a.drift_before = fint ? 0 : 1;
      a.drift_after = 1;
      a.target = side;
      const double ext = (side == 0 ? c->pend : 0) + 2.0 * k * dt;  // body force applied, x h/2
      a.s.pfx = ext * c->p.body_force[0];
      a.s.pfy = ext * c->p.body_force[1];
      a.s.pfz = ext * c->p.body_force[2];
      a.phys = (side == 0 || k > 0) ? 1 : 0;  // side 1, k > 0: FB holds the earlier sub-steps
      a.fa_rd = (side == 0 && k > 0) ? 1 : 0;
      a.cache_fill = (side == 1 && k == 0) ? 1 : 0;
      a.cache_use = (side == 1 && k > 0) || (side == 0 && c->mvalid) ? 1 : 0;
      if ((s = couple(c, a)) != LB_OK) return s;
    }
  }
  c->mvalid = true;
  return LB_OK;
}

static lb_status step_once(lb_ctx* c) {
  const bool parts = c->p.coupling != LB_COUPLE_NONE && c->np > 0;
  lb_status s;
  if (!parts) {
    c->mvalid = false;
    return lattice_pass(c);
  }
  if (c->p.coupling == LB_COUPLE_IB && c->tiled) {
    // dense markers: interpolation from the velocity of the flagged sites,
    // binned LDS-accumulated spreading
    const TileArgs t = tile_args(c);
    const int S = c->p.storage, K = c->p.kernel;
    // The binning only decides which workgroup accumulates a marker's force;
    // a marker whose stencil has left its tile's region adds to the field
    // directly, so results do not depend on how fresh the binning is.
    // Markers move far less than a site per step: rebin every kRebin steps.
    const int64_t rebin = c->p.ib_rebin > 0 ? c->p.ib_rebin : kRebin;
    if (c->binned_at < 0 || c->steps - c->binned_at >= rebin) {
      HIPCHK(c, launch_bin(t, c->L.pos, c->np, c->st));
      c->binned_at = c->steps;
    }
    // X~ = X + h/2 I[X]u(t), then X <- X + h/2 I[X~]u(t), from one velocity
    // pass.  The final advection of the previous step, X <- X + h/2 I[X~]u(t),
    // reads the same state and is done first (mode 3).
    // Markers listed by the interpolation are redone by their shells'
    // workgroups in the tether-force launch where the markers are whole shells.
    const bool fused = redo_in_shells(c);
    const double* at = c->adv_pending ? c->L.aux : c->L.pos;
    const int mode = c->adv_pending ? 3 : 2;
    if ((s = flag_interp(c, at, c->L.pos, c->L.aux, mode, !fused)) != LB_OK) return s;
    if (fused && (s = shell_forces_redo(c, at, c->L.pos, c->L.aux, mode, c->L.aux)) != LB_OK)
      return s;
    bool any;
    if ((s = enqueue_fint(c, c->L.aux, any, fused)) != LB_OK) return s;
    if (!any) HIPCHK(c, launch_zero(c->L.fint, (size_t)c->np * 24, c->st));
    if (c->p.deterministic) {
      if ((s = spread_fint_det(c)) != LB_OK) return s;
    } else {
      HIPCHK(c, launch_tile_spread(S, K, t, c->L.aux, c->L.fint, c->L.FA, c->np, c->st));
    }
    // The second half force is the same spread of the same F_int at X~: the
    // lattice pass keeps the first-half field as the pending one (ib_copy).
    if ((s = lattice_pass(c)) != LB_OK) return s;
    c->adv_pending = true;  // X <- X + h/2 I[X~]u(t+h): with the next step, or finish_step
    c->flags_follow = true;  // the mask now holds the stencils at X~
    return LB_OK;
  }
  if (c->p.coupling == LB_COUPLE_IB) {
    PartArgs a = part_args(c);
    HIPCHK(c, launch_ib_predict(c->p.storage, a, c->st));
    bool any;
    if ((s = enqueue_fint(c, c->L.aux, any)) != LB_OK) return s;
    if (!any) HIPCHK(c, launch_zero(c->L.fint, (size_t)c->np * 24, c->st));
    HIPCHK(c, launch_ib_advect(c->p.storage, a, c->p.deterministic ? 0 : 1, c->st));
    if (c->p.deterministic && (s = spread_fint_det(c)) != LB_OK) return s;
    if ((s = lattice_pass(c)) != LB_OK) return s;  // FB <- FA (ib_copy)
    a = part_args(c);
    HIPCHK(c, launch_ib_advect(c->p.storage, a, 0, c->st));
    return LB_OK;
  }
  if (c->p.mts_substeps > 0 && c->p.mts_inside) return step_mts_inside(c);
  if (c->p.mts_substeps > 0) {
    const int n = c->p.mts_substeps;
    const double dt = 1.0 / (2.0 * n);
    PartArgs a = part_args(c);
    a.target = 0;
    a.cache_use = c->mvalid ? 1 : 0;
    if ((s = couple(c, a)) != LB_OK) return s;
    // The 2n intrinsic-force sub-steps between the two coupling halves touch
    // only particle state and the lattice pass only fluid state, so all 2n
    // run together (bitwise the same as n, pass, n): as extra workgroups of
    // the lattice launch where they fit (they then cost the pass about one
    // percent of its CU time instead of a launch of their own), else as one
    // launch before the pass.  Running them on a second stream beside the
    // pass was measured slower.
    if (bonds_in_pass(c)) {
      if ((s = lattice_pass(c, 2 * n, dt)) != LB_OK) return s;
    } else {
      HIPCHK(c, launch_bond_groups(bond_args(c, c->L.pos), c->ngroups, c->gcap, 1, 0, 2 * n, dt,
                                   c->st));
      if ((s = lattice_pass(c)) != LB_OK) return s;
    }
    a = part_args(c);
    a.phys = 0;
    a.target = 1;
    a.cache_fill = 1;
    a.jc = 1;
    if ((s = couple(c, a)) != LB_OK) return s;
    c->mvalid = true;
    return LB_OK;
  }
  // Alg. 3: P^1/2, F_int, coupling half (+ spread A), LB, coupling half (+ spread B), P^1/2.
  // Without intrinsic forces the first P^1/2 is done by the coupling kernel.
  const bool fint = c->nshell > 0 || c->nbond > 0;
  bool any = false;
  if (fint && (s = drift_and_fint(c, 0.5, any)) != LB_OK) return s;
  PartArgs a = part_args(c);
  a.use_fint = any ? 1 : 0;
  a.drift_before = fint ? 0 : 1;
  a.target = 0;
  a.cache_use = c->mvalid ? 1 : 0;
  if ((s = couple(c, a)) != LB_OK) return s;
  if ((s = lattice_pass(c)) != LB_OK) return s;
  a = part_args(c);
  a.use_fint = any ? 1 : 0;
  a.phys = 0;
  a.target = 1;
  a.drift_after = 1;
  a.cache_fill = 1;
  a.jc = 1;
  if ((s = couple(c, a)) != LB_OK) return s;
  c->mvalid = true;
  return LB_OK;
}

extern "C" {

int32_t lb_lattice_velocities(int32_t c[57]) {
  for (int i = 0; i < Q; ++i) {
    c[3 * i] = CX[i];
    c[3 * i + 1] = CY[i];
    c[3 * i + 2] = CZ[i];
  }
  return Q;
}

lb_status lb_workspace_size(const lb_grid* g, const lb_params* p, const lb_limits* lim,
                            size_t* bytes) {
  std::string err;
  if (!bytes) return fail(nullptr, LB_EINVAL, "null output");
  if (!check_params(g, p, lim, err)) return fail(nullptr, LB_EINVAL, err);
  *bytes = carve(*g, *p, *lim, nullptr).bytes;
  return LB_OK;
}

static lb_status create_ctx(const lb_grid* g, const lb_params* p, const lb_limits* lim,
                            void* d_workspace, size_t bytes, void* hip_stream, bool linear_mask,
                            lb_ctx** out);

lb_status lb_create(const lb_grid* g, const lb_params* p, const lb_limits* lim, void* d_workspace,
                    size_t bytes, void* hip_stream, lb_ctx** out) {
  return create_ctx(g, p, lim, d_workspace, bytes, hip_stream, false, out);
}

}  // extern "C"

static lb_status create_ctx(const lb_grid* g, const lb_params* p, const lb_limits* lim,
                            void* d_workspace, size_t bytes, void* hip_stream, bool linear_mask,
                            lb_ctx** out) {
  std::string err;
  if (!out) return fail(nullptr, LB_EINVAL, "null output");
  *out = nullptr;
  if (!check_params(g, p, lim, err)) return fail(nullptr, LB_EINVAL, err);
  const size_t need = carve(*g, *p, *lim, nullptr).bytes;
  if (!d_workspace || bytes < need)
    return fail(nullptr, LB_ENOMEM, "workspace smaller than lb_workspace_size");
  if (((uintptr_t)d_workspace & 255) != 0)
    return fail(nullptr, LB_EINVAL, "workspace must be 256-byte aligned");
  lb_ctx* c = new lb_ctx();
  c->g = *g;
  c->p = *p;
  if (!(c->p.trt_magic > 0)) c->p.trt_magic = 3.0 / 16.0;
  c->lim = *lim;
  c->st = (hipStream_t)hip_stream;
  c->geo.nx = g->nx;
  c->geo.ny = g->ny;
  c->geo.nz = g->nz;
  c->geo.wall = g->wall_y;
  // Row-aligned mask words (and the row-per-workgroup lattice pass) when x is
  // a multiple of 64; otherwise one word per 64 consecutive linear sites and
  // the linear-site pass.
  c->geo.wpr = (linear_mask || g->nx % 64 != 0) ? 0 : g->nx / 64;
  c->member = linear_mask;
  c->geo.N = (long long)g->nx * g->ny * g->nz;
  c->geo.ps = pop_stride(c->geo.N);
  c->L = carve(*g, *p, *lim, d_workspace);
  c->tiled = p->coupling == LB_COUPLE_IB && p->kernel >= 3;
  const double lp = 1.0 / c->p.tau;
  const double lm = c->p.collision == LB_TRT ? 1.0 / (0.5 + c->p.trt_magic / (c->p.tau - 0.5)) : lp;
  c->omp = 1.0 - lp;
  c->omm = 1.0 - lm;
  if (p->storage == LB_F16 || p->storage == LB_BF16) {
    c->scale = std::ldexp(1.0f, p->f16_scale_log2);
    c->inv = std::ldexp(1.0f, -p->f16_scale_log2);
  }
  {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
            hipSuccess)
      c->lds_cu = v;
  }
  lb_status s = lb_init_fluid(c, nullptr, nullptr);
  if (s != LB_OK) {
    g_last_error = c->err;
    delete c;
    return s;
  }
  *out = c;
  return LB_OK;
}

extern "C" {

lb_status lb_init_fluid(lb_ctx* c, const double* d_rho, const double* d_u) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (c->running) return fail(c, LB_ESTATE, "an ensemble slot is initialised before its first step");
  InitArgs a{c->geo, c->L.f[0], d_rho, d_u, c->p.rho0, c->scale};
  c->cur = 0;
  HIPCHK(c, launch_init(c->p.storage, a, c->st));
  const size_t vb = (size_t)c->geo.N * force_vec_bytes(c->p.storage);
  HIPCHK(c, launch_zero(c->L.FA, vb, c->st));
  HIPCHK(c, launch_zero(c->L.FB, vb, c->st));
  HIPCHK(c, launch_zero(c->L.mask, mask_words(c->g) * 8, c->st));
  for (int f = 0; f < kMtsFields; ++f)
    if (c->L.G[f]) HIPCHK(c, launch_zero(c->L.G[f], vb, c->st));
  if (c->p.deterministic) HIPCHK(c, launch_zero(c->L.det, (size_t)c->geo.N * 48, c->st));
  if (c->tiled) {
    HIPCHK(c, launch_zero(c->L.U, (size_t)c->geo.N * 4 * (c->p.storage == LB_F64 ? 8 : 4), c->st));
    HIPCHK(c, launch_zero(c->L.miss, 8, c->st));
    c->ustamp = 0;
    c->flags_follow = false;
  }
  c->pend = 0;
  c->mvalid = false;
  c->uref[0] = c->uref[1] = c->uref[2] = 0.0;
  return LB_OK;
}

lb_status lb_set_particles(lb_ctx* c, int64_t n, const double* d_pos, const double* d_vel,
                           const double* d_mass) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (c->running) return fail(c, LB_ESTATE, "an ensemble slot is given particles before its first step");
  if (n < 0) return fail(c, LB_EINVAL, "negative particle count");
  if (n > c->lim.max_particles) return fail(c, LB_ENOMEM, "more particles than max_particles");
  const bool massive = c->p.coupling == LB_COUPLE_FC || c->p.coupling == LB_COUPLE_EBF;
  if (n > 0 && !d_pos) return fail(c, LB_EINVAL, "null positions");
  if (n > 0 && massive && (!d_vel || !d_mass))
    return fail(c, LB_EINVAL, "force coupling needs velocities and masses");
  if (n > 0) {
    HIPCHK(c, hipMemcpyAsync(c->L.pos, d_pos, n * 24, hipMemcpyDeviceToDevice, c->st));
    if (d_vel)
      HIPCHK(c, hipMemcpyAsync(c->L.vel, d_vel, n * 24, hipMemcpyDeviceToDevice, c->st));
    else
      HIPCHK(c, launch_zero(c->L.vel, n * 24, c->st));
    if (d_mass) {
      HIPCHK(c, hipMemcpyAsync(c->L.mass, d_mass, n * 8, hipMemcpyDeviceToDevice, c->st));
    } else {
      std::vector<double> ones(n, 1.0);
      HIPCHK(c, hipMemcpyAsync(c->L.mass, ones.data(), n * 8, hipMemcpyHostToDevice, c->st));
      HIPCHK(c, hipStreamSynchronize(c->st));
    }
    HIPCHK(c, launch_wrap(c->geo, n, c->L.pos, c->st));
  }
  c->np = n;
  c->groups_dirty = true;
  c->binned_at = -1;
  c->flags_follow = false;
  c->mvalid = false;
  return LB_OK;
}

lb_status lb_set_bonds(lb_ctx* c, int64_t nb, const int32_t* h_pairs, double k, double r0,
                       int32_t type) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (nb < 0 || (nb > 0 && !h_pairs)) return fail(c, LB_EINVAL, "invalid bond list");
  if (nb > c->lim.max_bonds) return fail(c, LB_ENOMEM, "more bonds than max_bonds");
  if (type != LB_HARMONIC && type != LB_FENE) return fail(c, LB_EINVAL, "unknown bond type");
  if (!std::isfinite(k) || !std::isfinite(r0) || (type == LB_FENE && !(r0 > 0)))
    return fail(c, LB_EINVAL, "invalid bond parameters");
  c->bonds.assign(h_pairs, h_pairs + 2 * nb);
  c->nbond = nb;
  c->bond_k = k;
  c->bond_r0 = r0;
  c->bond_type = type;
  c->groups_dirty = true;
  return LB_OK;
}

lb_status lb_set_shells(lb_ctx* c, int32_t nshell, int32_t shell_size, const double* h_template,
                        double k_tether) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (nshell < 0 || shell_size < 0 || (nshell > 0 && (shell_size < 3 || !h_template)))
    return fail(c, LB_EINVAL, "invalid shell description");
  if (nshell > c->lim.max_shells || shell_size > c->lim.max_shell_size)
    return fail(c, LB_ENOMEM, "shells exceed the limits");
  if (nshell > 0 && c->p.mts_substeps > 0)
    return fail(c, LB_EINVAL, "shells are not supported with multiple time stepping");
  if (nshell > 0) {
    HIPCHK(c, hipMemcpyAsync(c->L.tmpl, h_template, (size_t)shell_size * 24,
                             hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
  }
  c->nshell = nshell;
  c->shell_size = shell_size;
  c->k_tether = k_tether;
  return LB_OK;
}

lb_status lb_step(lb_ctx* c, int64_t nsteps) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (c->member) return fail(c, LB_ESTATE, "an ensemble slot is stepped by lb_ensemble_step");
  if (nsteps < 0) return fail(c, LB_EINVAL, "negative step count");
  if ((int64_t)c->nshell * c->shell_size > c->np)
    return fail(c, LB_ESTATE, "shells need nshell*shell_size particles");
  const bool need_groups =
      c->np > 0 && c->p.coupling != LB_COUPLE_NONE && (c->nbond > 0 || c->p.mts_substeps > 0);
  if (need_groups && c->groups_dirty) {
    lb_status s = build_groups(c);
    if (s != LB_OK) return s;
  }
  for (int64_t t = 0; t < nsteps; ++t) {
    lb_status s = step_once(c);
    if (s != LB_OK) return s;
    c->steps++;
  }
  return finish_step(c);
}

lb_status lb_moments(lb_ctx* c, double* d_rho, double* d_u) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (!d_u) return fail(c, LB_EINVAL, "null velocity output");
  HIPCHK(c, launch_moments(c->p.storage, site_args(c), d_rho, d_u, c->st));
  return LB_OK;
}

lb_status lb_populations(lb_ctx* c, double* d_df) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (!d_df) return fail(c, LB_EINVAL, "null output");
  const double gp = c->p.csc ? std::sqrt(c->omp) : 1.0, gm = c->p.csc ? std::sqrt(c->omm) : 1.0;
  HIPCHK(c, launch_populations(c->p.storage, site_args(c), d_df, gp, gm, c->st));
  return LB_OK;
}

lb_status lb_stress(lb_ctx* c, double* d_sigma) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (!d_sigma) return fail(c, LB_EINVAL, "null output");
  // 1 - lambda+/2 with 1 - lambda+ = omp; the trace part relaxes at the bulk rate for LB_MRT
  const double ps = 0.5 * (1.0 + c->omp);
  const double pb = c->p.collision == LB_MRT ? 1.0 - 0.5 * c->p.mrt_rates[0] : ps;
  HIPCHK(c, launch_stress(c->p.storage, site_args(c), d_sigma, ps, pb, c->st));
  return LB_OK;
}

lb_status lb_stress_sweep(lb_ctx* c, void* d_sigma) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (c->member) return fail(c, LB_ESTATE, "ensemble slots have no stress sweep");
  if (d_sigma && (c->p.collision == LB_MRT || c->p.kT > 0.0))
    return fail(c, LB_EINVAL, "the stress sweep takes the BGK or two-rate collision without noise");
  c->sweep = d_sigma;
  return LB_OK;
}

lb_status lb_get_particles(lb_ctx* c, double* d_pos, double* d_vel) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (c->np > 0 && d_pos)
    HIPCHK(c, hipMemcpyAsync(d_pos, c->L.pos, c->np * 24, hipMemcpyDeviceToDevice, c->st));
  if (c->np > 0 && d_vel)
    HIPCHK(c, hipMemcpyAsync(d_vel, c->L.vel, c->np * 24, hipMemcpyDeviceToDevice, c->st));
  return LB_OK;
}

lb_status lb_totals(lb_ctx* c, double h_out[7]) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (!h_out) return fail(c, LB_EINVAL, "null output");
  const bool massive = c->p.coupling == LB_COUPLE_FC || c->p.coupling == LB_COUPLE_EBF;
  HIPCHK(c, launch_totals(c->p.storage, site_args(c), c->L.partial, kTotalsBlocks,
                          massive ? c->L.vel : nullptr, massive ? c->L.mass : nullptr, c->np,
                          c->L.tot, c->st));
  double tmp[8];
  HIPCHK(c, hipMemcpyAsync(tmp, c->L.tot, 8 * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (int k = 0; k < 7; ++k) h_out[k] = tmp[k];
  return LB_OK;
}

static void free_events(lb_ctx* c) {
  for (auto e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  c->ev_used = 0;
  c->ev_seen = 0;
}

lb_status lb_timing(lb_ctx* c, int32_t max_passes, int32_t stride) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (max_passes < 0 || max_passes > (1 << 20)) return fail(c, LB_EINVAL, "invalid pass count");
  if (stride < 1 || stride > (1 << 20)) return fail(c, LB_EINVAL, "invalid timing stride");
  HIPCHK(c, hipStreamSynchronize(c->st));
  free_events(c);
  for (int32_t k = 0; k < 2 * max_passes; ++k) {
    hipEvent_t e;
    HIPCHK(c, hipEventCreate(&e));
    c->ev.push_back(e);
  }
  c->ev_stride = stride;
  return LB_OK;
}

lb_status lb_timing_read(lb_ctx* c, double* lattice_ms, int64_t* passes) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  HIPCHK(c, hipStreamSynchronize(c->st));
  double tot = 0;
  for (int32_t k = 0; k < c->ev_used; ++k) {
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
    tot += ms;
  }
  if (lattice_ms) *lattice_ms = tot;
  if (passes) *passes = c->ev_used;
  c->ev_used = 0;
  return LB_OK;
}

lb_status lb_info(const lb_ctx* c, int64_t* nparticles, int64_t* steps) {
  if (!c) return fail(nullptr, LB_EINVAL, "null context");
  if (nparticles) *nparticles = c->np;
  if (steps) *steps = c->steps;
  return LB_OK;
}

static void release_static(lb_ctx* c);

lb_status lb_destroy(lb_ctx* c) {
  if (!c) return LB_OK;
  free_events(c);
  release_static(c);
  delete c;
  return LB_OK;
}

const char* lb_last_error(const lb_ctx* c) { return c ? c->err.c_str() : g_last_error.c_str(); }

const char* lb_status_string(lb_status s) {
  switch (s) {
    case LB_OK: return "ok";
    case LB_EINVAL: return "invalid argument";
    case LB_ENOMEM: return "insufficient workspace or capacity";
    case LB_EBUSY: return "busy";
    case LB_EDEVICE: return "device error";
    case LB_ESTATE: return "invalid state";
  }
  return "unknown status";
}

}  // extern "C"

// ===========================================================================
// A context without caller memory: its workspace is a file-scope device array
// of the library (one copy per GPU, held until the process ends).
// ===========================================================================
namespace {

constexpr size_t kStaticBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

struct StaticSlot {
  void* ptr = nullptr;     // device address of this GPU's copy of `scratch`
  lb_ctx* owner = nullptr; // the live context whose workspace it is
};
std::mutex g_static_mu;
StaticSlot g_static[kMaxDevices];

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

static void release_static(lb_ctx* c) {
  if (c->static_dev < 0) return;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (g_static[c->static_dev].owner == c) g_static[c->static_dev].owner = nullptr;
  c->static_dev = -1;
}

extern "C" lb_status lb_create_static(const lb_grid* g, const lb_params* p, const lb_limits* lim,
                                      void* hip_stream, lb_ctx** out) {
  std::string err;
  if (!out) return fail(nullptr, LB_EINVAL, "null output");
  *out = nullptr;
  if (!check_params(g, p, lim, err)) return fail(nullptr, LB_EINVAL, err);
  const size_t need = carve(*g, *p, *lim, nullptr).bytes;
  if (need > kStaticBytes)
    return fail(nullptr, LB_ENOMEM,
                "the box needs " + std::to_string(need) + " bytes of device memory; "
                "lb_create_static holds at most " + std::to_string(kStaticBytes) +
                " bytes (use lb_create with a caller workspace)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, LB_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, LB_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_static_mu);
  StaticSlot& sl = g_static[dev];
  if (sl.owner)
    return fail(nullptr, LB_EBUSY,
                "a context made by lb_create_static is alive on this device; destroy it first");
  if (!sl.ptr) {  // first use on this device (which is current): resolve its copy of the array
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(nullptr, LB_EDEVICE,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    sl.ptr = ptr;
  }
  lb_ctx* c = nullptr;
  lb_status st = create_ctx(g, p, lim, sl.ptr, kStaticBytes, hip_stream, false, &c);
  if (st != LB_OK) return st;
  c->static_dev = dev;
  sl.owner = c;
  *out = c;
  return LB_OK;
}

// ===========================================================================
// Ensembles: many boxes resident in one caller-owned pool, stepped together.
// ===========================================================================
namespace {

struct EnsHost {
  bool live = false;
  bool fresh = false;  // admitted, host fields authoritative until the next refresh
  lb_ctx* ctx = nullptr;
  size_t off = 0, bytes = 0;
  int64_t target = 0;
};

constexpr int kGraphSteps = 8;

}  // namespace

struct lb_ensemble {
  char* pool = nullptr;
  size_t bytes = 0, head = 0;
  hipStream_t st = nullptr;
  bool own_stream = false;  // created by lb_ensemble_create (no stream was given)
  int max_slots = 0, storage = LB_F32, kernel = 2;
  int det = 0;  // deterministic spreading in every slot
  EnsSlot* d_slots = nullptr;
  int2* d_litems = nullptr;
  int2* d_pitems = nullptr;
  int* d_counts = nullptr;  // [0] lattice items, [1] particle items
  size_t max_items = 0;
  std::vector<EnsHost> slots;
  std::vector<std::pair<size_t, size_t>> used;  // (offset, bytes), sorted
  bool dirty = true;
  int cus = 256;
  int lat_grid = 0, part_grid = 512;  // lattice: one block per item (ens_refresh)
  int part_items = 1024;  // particle work items, rounded up (an autotuner candidate)
  hipGraphExec_t exec[2] = {nullptr, nullptr};  // kGraphSteps steps, one step
  bool graphs_ok = false;
  std::string err;
};

#define EHIPCHK(e, call)                                                              \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      (e)->err = std::string(#call) + ": " + hipGetErrorString(e_);                   \
      return LB_EDEVICE;                                                              \
    }                                                                                 \
  } while (0)

static lb_status efail(lb_ensemble* e, lb_status s, const std::string& m) {
  if (e)
    e->err = m;
  else
    g_last_error = m;
  return s;
}

static EnsArgs ens_args(const lb_ensemble* e) {
  EnsArgs a;
  a.slots = e->d_slots;
  a.nslots = e->max_slots;
  a.litems = e->d_litems;
  a.nlitems = e->d_counts;
  a.pitems = e->d_pitems;
  a.npitems = e->d_counts + 1;
  return a;
}

static EnsSlot slot_from_ctx(const lb_ctx* c) {
  EnsSlot s{};
  s.g = c->geo;
  s.rnx = 1.0 / c->geo.nx;
  s.rny = 1.0 / c->geo.ny;
  s.f[0] = c->L.f[0];
  s.f[1] = c->L.f[1];
  s.FA = c->L.FA;
  s.FB = c->L.FB;
  s.mask = c->L.mask;
  s.pos = c->L.pos;
  s.vel = c->L.vel;
  s.mass = c->L.mass;
  s.np = c->np;
  s.rho0 = c->p.rho0;
  s.fx = c->p.body_force[0];
  s.fy = c->p.body_force[1];
  s.fz = c->p.body_force[2];
  s.omp = c->omp;
  s.omm = c->omm;
  s.gamma = c->p.gamma;
  s.det_on = c->p.deterministic;
  s.aux = c->L.aux;
  s.det = c->L.det;
  s.scale = c->scale;
  s.inv = c->inv;
  s.collision = c->p.collision;
  s.coupling = c->p.coupling;
  s.cur = c->cur;
  s.pend = c->pend;
  s.steps_done = 0;
  s.live = 1;
  s.comoving = c->p.comoving;
  for (int k = 0; k < 3; ++k) s.uref[k] = c->uref[k];
  s.mcache = c->L.mcache;
  s.mbase = c->L.mbase;
  s.mvalid = 0;
  double uo[3];
  for (int k = 0; k < 3; ++k)
    uo[k] = c->uref[k] + (c->p.comoving ? c->p.body_force[k] / c->p.rho0 : 0.0);
  comoving_terms(c->scale, c->p.rho0, c->uref, uo, s.cm, s.cmf);
  return s;
}

// Download the device slot table, take the device-advanced fields of running
// slots, write host fields of freshly admitted ones, upload, rebuild the work
// lists.
static void ens_drop_graphs(lb_ensemble* e);

static lb_status ens_refresh(lb_ensemble* e) {
  std::vector<EnsSlot> hs(e->max_slots);
  EHIPCHK(e, hipStreamSynchronize(e->st));
  EHIPCHK(e, hipMemcpy(hs.data(), e->d_slots, hs.size() * sizeof(EnsSlot), hipMemcpyDeviceToHost));
  std::vector<int2> li, pi;
  const int L = e->kernel == 2 ? 8 : (e->kernel == 3 ? 32 : 64);
  const int ppb = 256 / L;
  for (int i = 0; i < e->max_slots; ++i) {
    EnsHost& h = e->slots[i];
    if (!h.live) {
      hs[i].live = 0;
      continue;
    }
    if (h.fresh) {
      hs[i] = slot_from_ctx(h.ctx);
      hs[i].steps_target = h.target;
      h.fresh = false;
      h.ctx->running = true;
    }
    const long long nch = (h.ctx->geo.N + 255) / 256;
    for (long long k = 0; k < nch; ++k) li.push_back(make_int2(i, (int)k));
    for (long long p = 0; p < h.ctx->np; p += ppb) pi.push_back(make_int2(i, (int)p));
  }
  if (li.size() > e->max_items || pi.size() > e->max_items)
    return efail(e, LB_ENOMEM, "ensemble work list exceeds its capacity");
  const int counts[2] = {(int)li.size(), (int)pi.size()};
  // One workgroup per lattice item: a persistent grid striding over the items
  // streamed 15-20 % slower (FP16: 32 x 96^3 4.92 -> 5.88 TB/s, one 250^3 box
  // 4.62 -> 5.48, 8 x 128^3 4.70 -> 5.16).  The grid is the item count rounded
  // up to 4096; workgroups beyond the count leave at once, and the captured
  // graphs are rebuilt only when that size grows or falls below half.
  const int cap = std::max(4096, ((int)li.size() + 4095) / 4096 * 4096);
  if (cap > e->lat_grid || 2 * cap < e->lat_grid) {
    e->lat_grid = cap;
    ens_drop_graphs(e);
  }
  e->part_items = std::max(1024, ((int)pi.size() + 1023) / 1024 * 1024);
  EHIPCHK(e, hipMemcpy(e->d_slots, hs.data(), hs.size() * sizeof(EnsSlot), hipMemcpyHostToDevice));
  if (!li.empty())
    EHIPCHK(e, hipMemcpy(e->d_litems, li.data(), li.size() * sizeof(int2), hipMemcpyHostToDevice));
  if (!pi.empty())
    EHIPCHK(e, hipMemcpy(e->d_pitems, pi.data(), pi.size() * sizeof(int2), hipMemcpyHostToDevice));
  EHIPCHK(e, hipMemcpy(e->d_counts, counts, sizeof(counts), hipMemcpyHostToDevice));
  e->dirty = false;
  return LB_OK;
}

static void ens_drop_graphs(lb_ensemble* e) {
  for (auto& x : e->exec)
    if (x) {
      (void)hipGraphExecDestroy(x);
      x = nullptr;
    }
  e->graphs_ok = false;
}

// Capture kGraphSteps steps and one step into graphs (kernels only).
static lb_status ens_build_graphs(lb_ensemble* e) {
  ens_drop_graphs(e);
  const EnsArgs a = ens_args(e);
  for (int g = 0; g < 2; ++g) {
    const int n = g == 0 ? kGraphSteps : 1;
    hipGraph_t graph;
    EHIPCHK(e, hipStreamBeginCapture(e->st, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < n; ++k) {
      hipError_t r = launch_ens_step(e->storage, e->kernel, a, e->lat_grid, e->part_grid, e->det, e->st);
      if (r != hipSuccess) {
        (void)hipStreamEndCapture(e->st, &graph);
        e->err = std::string("capture: ") + hipGetErrorString(r);
        return LB_EDEVICE;
      }
    }
    EHIPCHK(e, hipStreamEndCapture(e->st, &graph));
    EHIPCHK(e, hipGraphInstantiate(&e->exec[g], graph, nullptr, nullptr, 0));
    EHIPCHK(e, hipGraphDestroy(graph));
  }
  e->graphs_ok = true;
  return LB_OK;
}

static bool ens_place(lb_ensemble* e, size_t need, size_t& off) {
  size_t cur = e->head;
  for (const auto& u : e->used) {
    if (u.first >= cur + need) break;
    cur = std::max(cur, align256(u.first + u.second));
  }
  if (cur + need > e->bytes) return false;
  off = cur;
  e->used.push_back({off, need});
  std::sort(e->used.begin(), e->used.end());
  return true;
}

extern "C" {

lb_status lb_ensemble_footprint(const lb_grid* g, const lb_params* p, const lb_limits* lim,
                                size_t* bytes) {
  return lb_workspace_size(g, p, lim, bytes);
}

lb_status lb_ensemble_create(void* d_pool, size_t bytes, int32_t max_slots, int32_t storage,
                             int32_t kernel, int32_t deterministic, void* hip_stream,
                             lb_ensemble** out) {
  if (!out) return efail(nullptr, LB_EINVAL, "null output");
  *out = nullptr;
  if (!d_pool || ((uintptr_t)d_pool & 255)) return efail(nullptr, LB_EINVAL, "pool must be 256-byte aligned");
  if (max_slots < 1 || max_slots > 65536) return efail(nullptr, LB_EINVAL, "max_slots out of range");
  if (storage != LB_F32 && storage != LB_F16 && storage != LB_BF16 && storage != LB_F64)
    return efail(nullptr, LB_EINVAL, "unknown storage");
  if (kernel < 2 || kernel > 4) return efail(nullptr, LB_EINVAL, "kernel must be 2, 3 or 4");
  if (deterministic != 0 && deterministic != 1)
    return efail(nullptr, LB_EINVAL, "deterministic must be 0 or 1");
  lb_ensemble* e = new lb_ensemble();
  e->det = deterministic;
  e->pool = (char*)d_pool;
  e->bytes = bytes;
  e->max_slots = max_slots;
  e->storage = storage;
  e->kernel = kernel;
  e->max_items = std::max<size_t>(bytes / 16384, 4096);
  Carver c{e->pool};
  e->d_slots = c.take<EnsSlot>(sizeof(EnsSlot) * max_slots);
  e->d_litems = c.take<int2>(sizeof(int2) * e->max_items);
  e->d_pitems = c.take<int2>(sizeof(int2) * e->max_items);
  e->d_counts = c.take<int>(64);
  e->head = c.off;
  if (e->head >= bytes) {
    delete e;
    return efail(nullptr, LB_ENOMEM, "pool too small for the ensemble tables");
  }
  e->slots.resize(max_slots);
  {
    // default persistent grid of the particle launches: two 256-lane blocks
    // per CU (the lattice grid follows the item count, see ens_refresh)
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      e->cus = prop.multiProcessorCount;
      e->part_grid = 2 * e->cus;
    }
  }
  if (hip_stream) {  // borrowed: the caller keeps it alive until lb_ensemble_destroy
    e->st = (hipStream_t)hip_stream;
    e->own_stream = false;
  } else {  // the legacy null stream cannot be captured: make a default-priority stream
    hipError_t r = hipStreamCreate(&e->st);
    if (r != hipSuccess) {
      delete e;
      return efail(nullptr, LB_EDEVICE, hipGetErrorString(r));
    }
    e->own_stream = true;
  }
  std::vector<EnsSlot> zero(max_slots);
  for (auto& z : zero) z.live = 0;
  const int counts[2] = {0, 0};
  if (hipMemcpy(e->d_slots, zero.data(), zero.size() * sizeof(EnsSlot), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(e->d_counts, counts, sizeof(counts), hipMemcpyHostToDevice) != hipSuccess) {
    if (e->own_stream) (void)hipStreamDestroy(e->st);
    delete e;
    return efail(nullptr, LB_EDEVICE, "cannot initialise the ensemble tables");
  }
  *out = e;
  return LB_OK;
}

lb_status lb_ensemble_stream(lb_ensemble* e, void** stream) {
  if (!e || !stream) return efail(e, LB_EINVAL, "null argument");
  *stream = (void*)e->st;
  return LB_OK;
}

lb_status lb_ensemble_admit(lb_ensemble* e, const lb_grid* g, const lb_params* p,
                            const lb_limits* lim, int64_t nsteps, int32_t* slot, lb_ctx** ctx) {
  if (!e || !g || !p || !lim || !slot) return efail(e, LB_EINVAL, "null argument");
  std::string err;
  if (!check_params(g, p, lim, err)) return efail(e, LB_EINVAL, err);
  if (g->wall_y) return efail(e, LB_EINVAL, "ensemble members are periodic boxes");
  if (p->coupling == LB_COUPLE_IB || p->mts_substeps != 0)
    return efail(e, LB_EINVAL, "ensemble members use FC, EBF or no coupling without sub-steps");
  if (p->kT != 0.0) return efail(e, LB_EINVAL, "ensemble members are deterministic (kT = 0)");
  if (p->deterministic != e->det)
    return efail(e, LB_EINVAL, "deterministic spreading must match the ensemble's");
  if (p->collision == LB_MRT)
    return efail(e, LB_EINVAL, "ensemble members use the BGK or two-rate collision");
  if (lim->max_bonds != 0 || lim->max_shells != 0)
    return efail(e, LB_EINVAL, "ensemble members carry free particles only");
  if (p->storage != e->storage || p->kernel != e->kernel)
    return efail(e, LB_EINVAL, "storage and kernel must match the ensemble");
  if (nsteps < 0) return efail(e, LB_EINVAL, "negative step budget");
  int idx = -1;
  for (int i = 0; i < e->max_slots; ++i)
    if (!e->slots[i].live) {
      idx = i;
      break;
    }
  if (idx < 0) return efail(e, LB_EBUSY, "no free slot");
  size_t need = carve(*g, *p, *lim, nullptr).bytes, off;
  if (!ens_place(e, need, off)) return efail(e, LB_EBUSY, "not enough free memory in the pool");
  lb_ctx* c = nullptr;
  lb_status s = create_ctx(g, p, lim, e->pool + off, need, (void*)e->st, true, &c);
  if (s != LB_OK) {
    e->used.erase(std::find(e->used.begin(), e->used.end(), std::make_pair(off, need)));
    return efail(e, s, g_last_error);
  }
  EnsHost& h = e->slots[idx];
  h.live = true;
  h.fresh = true;
  h.ctx = c;
  h.off = off;
  h.bytes = need;
  h.target = nsteps;
  e->dirty = true;
  *slot = idx;
  if (ctx) *ctx = c;
  return LB_OK;
}

lb_status lb_ensemble_step(lb_ensemble* e, int64_t nsteps) {
  if (!e) return efail(nullptr, LB_EINVAL, "null ensemble");
  if (nsteps < 0) return efail(e, LB_EINVAL, "negative step count");
  lb_status s;
  if (e->dirty && (s = ens_refresh(e)) != LB_OK) return s;
  if (!e->graphs_ok && (s = ens_build_graphs(e)) != LB_OK) return s;
  int64_t k = 0;
  for (; k + kGraphSteps <= nsteps; k += kGraphSteps) EHIPCHK(e, hipGraphLaunch(e->exec[0], e->st));
  for (; k < nsteps; ++k) EHIPCHK(e, hipGraphLaunch(e->exec[1], e->st));
  return LB_OK;
}

lb_status lb_ensemble_query(lb_ensemble* e, int32_t slot, int64_t* steps_done, int32_t* done) {
  if (!e) return efail(nullptr, LB_EINVAL, "null ensemble");
  if (slot < 0 || slot >= e->max_slots || !e->slots[slot].live)
    return efail(e, LB_EINVAL, "not a live slot");
  EnsHost& h = e->slots[slot];
  int64_t sd = 0;
  if (!h.fresh) {
    EnsSlot d;
    EHIPCHK(e, hipStreamSynchronize(e->st));
    EHIPCHK(e, hipMemcpy(&d, e->d_slots + slot, sizeof(EnsSlot), hipMemcpyDeviceToHost));
    h.ctx->cur = d.cur;
    h.ctx->pend = d.pend;
    h.ctx->steps = d.steps_done;
    for (int k = 0; k < 3; ++k) h.ctx->uref[k] = d.uref[k];
    sd = d.steps_done;
  }
  if (steps_done) *steps_done = sd;
  if (done) *done = sd >= h.target ? 1 : 0;
  return LB_OK;
}

lb_status lb_ensemble_retire(lb_ensemble* e, int32_t slot) {
  if (!e) return efail(nullptr, LB_EINVAL, "null ensemble");
  if (slot < 0 || slot >= e->max_slots || !e->slots[slot].live)
    return efail(e, LB_EINVAL, "not a live slot");
  EHIPCHK(e, hipStreamSynchronize(e->st));
  EnsHost& h = e->slots[slot];
  e->used.erase(std::find(e->used.begin(), e->used.end(), std::make_pair(h.off, h.bytes)));
  lb_destroy(h.ctx);
  h = EnsHost();
  e->dirty = true;
  return LB_OK;
}

// Project autotuner: time real steps of the current mix under each candidate
// persistent-grid shape of the particle launches and keep the fastest (every
// shape computes the same update, so tuning steps are ordinary steps of the
// live slots).  The lattice launch has one block per work item.
lb_status lb_ensemble_autotune(lb_ensemble* e, int32_t steps_per_candidate, int32_t* lat_grid,
                               int32_t* part_grid) {
  if (!e) return efail(nullptr, LB_EINVAL, "null ensemble");
  if (steps_per_candidate < 1) return efail(e, LB_EINVAL, "need at least one step per candidate");
  lb_status s;
  if (e->dirty && (s = ens_refresh(e)) != LB_OK) return s;
  const int cus = e->cus;
  const int lat_c[] = {e->lat_grid};
  const int part_c[] = {cus, cus * 2, cus * 4, e->part_items};
  hipEvent_t t0, t1;
  EHIPCHK(e, hipEventCreate(&t0));
  EHIPCHK(e, hipEventCreate(&t1));
  float best = 1e30f;
  int bl = e->lat_grid, bp = e->part_grid;
  const EnsArgs a = ens_args(e);
  for (int lg : lat_c)
    for (int pg : part_c) {
      EHIPCHK(e, hipEventRecord(t0, e->st));
      for (int k = 0; k < steps_per_candidate; ++k)
        EHIPCHK(e, launch_ens_step(e->storage, e->kernel, a, lg, pg, e->det, e->st));
      EHIPCHK(e, hipEventRecord(t1, e->st));
      EHIPCHK(e, hipEventSynchronize(t1));
      float ms;
      EHIPCHK(e, hipEventElapsedTime(&ms, t0, t1));
      if (ms < best) {
        best = ms;
        bl = lg;
        bp = pg;
      }
    }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (bl != e->lat_grid || bp != e->part_grid) {
    e->lat_grid = bl;
    e->part_grid = bp;
    ens_drop_graphs(e);
  }
  if (lat_grid) *lat_grid = bl;
  if (part_grid) *part_grid = bp;
  return LB_OK;
}

lb_status lb_ensemble_destroy(lb_ensemble* e) {
  if (!e) return LB_OK;
  (void)hipStreamSynchronize(e->st);
  for (auto& h : e->slots)
    if (h.live) lb_destroy(h.ctx);
  ens_drop_graphs(e);
  if (e->own_stream) (void)hipStreamDestroy(e->st);
  delete e;
  return LB_OK;
}

const char* lb_ensemble_last_error(const lb_ensemble* e) {
  return e ? e->err.c_str() : g_last_error.c_str();
}

}  // extern "C"
