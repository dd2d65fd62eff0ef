// lbc_kernels.hip -- gfx950 kernels of the split-forcing lattice Boltzmann
// step with fluid-particle coupling (Schiller, arXiv:1406.2211).
//
// Lattice state between steps: post-collision populations f* (deviation from
// w rho0, structure of arrays [19][nz][ny][nx]), a pending second half force
// FB (per-site vector, nonzero only at sites flagged in a per-site bit mask)
// and a flag telling whether the body force's second half is pending.  The
// physical populations at a step boundary are S f* shifted by the equilibrium
// difference of that pending half force (Sec. 3.3: a midpoint half force is an
// exact equilibrium shift).
#include "lbc_device.h"
#include "lbc_internal.h"

namespace lbc {

// ======================================================================
// Fused lattice pass: pull (streaming S, Sec. 3.1), moments, both pending
// half forces as one equilibrium shift (F^1/2 of the previous step and of
// this step, Sec. 3.3), collision C (Eq. collision-operator / Eq. mrt-coll),
// store.  One work-item per site; a 64-wide wavefront covers 64 consecutive
// x sites of one row, i.e. exactly one 64-bit word of the force mask.
// ======================================================================
//
// Addressing: a block covers (part of) one x row, so the y and z of the nine
// source rows are block-uniform and live in scalar registers together with
// the per-population base pointers; each work-item adds a 32-bit site offset.
// All 19 loads are issued before any arithmetic.  With y walls the
// bounce-back choice is also block-uniform (it depends on y only).
// Coupling forces of one site for the fused pass, from the two force fields
// where the mask word flags the site; both fields are zeroed after the read,
// and the owning lane clears the word when the pass clears the mask.
template <int S>
__device__ __forceinline__ void take_forces(uint64_t word, uint64_t* mp, size_t site, uint32_t lane,
                                            void* FAp, void* FBp, bool clear,
                                            typename Store<S>::R& Fx, typename Store<S>::R& Fy,
                                            typename Store<S>::R& Fz) {
  using V4 = typename Store<S>::V4;
  if ((word >> lane) & 1ull) {
    V4* FA = (V4*)FAp;
    V4* FB = (V4*)FBp;
    const V4 fa = FA[site], fb = FB[site];
    Fx += fa.x + fb.x;
    Fy += fa.y + fb.y;
    Fz += fa.z + fb.z;
    V4 zero;
    zero.x = zero.y = zero.z = zero.w = 0;
    FA[site] = zero;
    FB[site] = zero;
  }
  if (lane == 0 && clear) *mp = 0;
}

// Immersed boundary: the second half force of a step is the same spread of
// the same F_int as the first (Sec. 5.1), so the first-half field becomes the
// pending second half: FB <- FA, FA <- 0, and the owning lane rewrites the
// word to flag exactly the sites of the pending field (which the next pass
// must read).  Called by all lanes of a wavefront that owns the (nonzero)
// word.
template <int S>
__device__ __forceinline__ void take_forces_ib(uint64_t word, uint64_t* mp, size_t site,
                                               uint32_t lane, void* FAp, void* FBp,
                                               typename Store<S>::R& Fx, typename Store<S>::R& Fy,
                                               typename Store<S>::R& Fz) {
  using V4 = typename Store<S>::V4;
  bool live = false;
  if ((word >> lane) & 1ull) {
    V4* FA = (V4*)FAp;
    V4* FB = (V4*)FBp;
    const V4 fa = FA[site], fb = FB[site];
    Fx += fa.x + fb.x;
    Fy += fa.y + fb.y;
    Fz += fa.z + fb.z;
    V4 zero;
    zero.x = zero.y = zero.z = zero.w = 0;
    FA[site] = zero;
    FB[site] = fa;
    live = fa.x != 0 || fa.y != 0 || fa.z != 0;
  }
  const uint64_t keep = __ballot(live);
  if (lane == 0 && keep != word) *mp = keep;
}

// Intrinsic-force sub-steps of one bond group (defined with the particle
// kernels below); the lattice pass may run them in extra workgroups.
__device__ void bond_group(const BondArgs& b, int grp, int mode, int acc, int nsub, double dt,
                           double* lds);

template <int S, bool CM, bool WALL, bool NS = false, bool MRT = false, bool SG = false>
__global__ __launch_bounds__(256) void k_stream_collide(LatArgs a) {
  using St = Store<S>;
  using T = typename St::T;
  using R = typename St::R;
  // Intrinsic-force sub-steps (workgroup-uniform branch).
  if (a.bond_groups > 0 && blockIdx.z == 0) {
    const int grp = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if (grp < a.bond_groups) {
      extern __shared__ double bond_lds[];
      bond_group(a.bond, grp, 1, 0, a.bond_nsub, a.bond_dt, bond_lds);
    }
    return;
  }
  const uint32_t nx = (uint32_t)a.g.nx, ny = (uint32_t)a.g.ny, nz = (uint32_t)a.g.nz;
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t y = blockIdx.y, z = blockIdx.z - (a.bond_groups > 0 ? 1u : 0u);
  if (x >= nx) return;
  const uint32_t ys[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
  const uint32_t zs[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
  const uint32_t xs[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
  const uint32_t own = (z * ny + y) * nx + x;
  const size_t N = (size_t)a.g.ps;  // population stride
  const T* __restrict__ fin = (const T*)a.fin;
  uint64_t* mp = a.mask + ((size_t)z * ny + y) * a.g.wpr + (x >> 6);
  const uint64_t word = *mp;
  R f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    // source of population i: x - c_i
    const uint32_t row = (zs[1 - CZ[i]] * ny + ys[1 - CY[i]]) * nx;
    const T* base = fin + (size_t)i * N;
    uint32_t off = row + xs[1 - CX[i]];
    if (WALL && ((CY[i] == 1 && y == 0) || (CY[i] == -1 && y == ny - 1))) {
      base = fin + (size_t)OPP[i] * N;  // halfway bounce-back: opposite population, same site
      off = own;
    }
    // non-temporal loads measured faster for the FP32 pass (256^3: 441 -> 432 us)
    // and slower for 16-bit storage and with thermal noise
    f[i] = (S == LB_F32 && !NS) ? St::raw_nt(base + off) : St::raw(base + off);
  }
  R Fx = R(a.Fx), Fy = R(a.Fy), Fz = R(a.Fz);
  if (word) {
    if (a.ib_copy)
      take_forces_ib<S>(word, mp, own, x & 63, a.FA, a.FB, Fx, Fy, Fz);
    else
      take_forces<S>(word, mp, own, x & 63, a.FA, a.FB, a.clear_mask != 0, Fx, Fy, Fz);
  }
  PassK<R> k;
  k.rho0 = R(a.rho0);
  k.sc = R(a.scale);
  k.inv = R(a.inv);
  k.hp = R(0.5) * R(a.omp);
  k.hm = R(0.5) * R(a.omm);
  for (int c = 0; c < 3; ++c) k.ui[c] = R(a.uin[c]);
  k.cm = pick_terms<R>(a.cm, a.cmf);
  if (NS) {
    k.ap = R(a.ap);
    k.am = R(a.am);
    k.k0 = a.key0;
    k.k1 = a.key1;
    k.t0 = a.t0;
    k.t1 = a.t1;
  }
  if (MRT) {
    for (int c = 0; c < 6; ++c) {
      k.lg[c] = R(a.lg[c]);
      k.ag[c] = R(a.ag[c]);
    }
    fused_site_mrt<S, NS>(f, Fx, Fy, Fz, k, (T*)a.fout, N, own);
  } else {
    fused_site<S, CM, NS, SG>(f, Fx, Fy, Fz, k, (T*)a.fout, N, own, (R*)a.sigma, (size_t)a.g.N,
                              R(a.sp));
  }
}

// ======================================================================
// Initialisation: physical state f = f^eq(rho, u).  Written as the pre-image
// under the pull gather (push of each population to the slot it will be
// pulled from), so that the first lattice pass sees exactly f^eq.
// ======================================================================
template <int S>
__global__ void k_init(InitArgs a) {
  using St = Store<S>;
  using T = typename St::T;
  using R = typename St::R;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= a.g.nx) return;
  const long long s = site_index(a.g, x, y, z);
  const double rho = a.rho ? a.rho[s] : a.rho0;
  const double ux = a.u ? a.u[s] : 0.0, uy = a.u ? a.u[a.g.N + s] : 0.0,
               uz = a.u ? a.u[2 * a.g.N + s] : 0.0;
  const double usq = ux * ux + uy * uy + uz * uz;
  const double drho = rho - a.rho0;
  T* f = (T*)a.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double v = feq_dev<double>(i, drho, rho, ux, uy, uz, usq);
    const int ys = y - CY[i];
    long long dst;
    if (a.g.wall && (ys < 0 || ys >= a.g.ny)) {
      dst = (long long)OPP[i] * a.g.ps + s;
    } else {
      dst = (long long)i * a.g.ps +
            site_index(a.g, wrap_idx(x - CX[i], a.g.nx), wrap_idx(ys, a.g.ny),
                       wrap_idx(z - CZ[i], a.g.nz));
    }
    St::st(f + dst, (R)v, (R)a.scale);
  }
}

template <int S>
__global__ void k_moments(SiteArgs a, double* rho, double* u) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= a.g.nx) return;
  double fl[Q], drho, j[3];
  site_phys<S>(a, x, y, z, fl, drho, j, true);
  const long long s = site_index(a.g, x, y, z);
  const double r = a.rho0 + drho;
  if (rho) rho[s] = r;
  u[s] = j[0] / r;
  u[a.g.N + s] = j[1] / r;
  u[2 * a.g.N + s] = j[2] / r;
}

// Physical populations: the stored ones moved by the pending half force, an
// equilibrium shift f -> f + f^eq(rho, u_phys) - f^eq(rho, u).  With csc the
// non-equilibrium part f - f^eq(rho, u) is split into even and odd parts
// over opposite directions and scaled by gp, gm: the exact half collision of
// the two-rate operator (Sec. 3.2), which leaves rho and u unchanged.
template <int S>
__global__ void k_populations(SiteArgs a, double* out, double gp, double gm, int csc) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= a.g.nx) return;
  double fl[Q], drho, j[3], jb[3];
  site_phys<S>(a, x, y, z, fl, drho, jb, false);
  site_phys<S>(a, x, y, z, fl, drho, j, true);
  const long long s = site_index(a.g, x, y, z);
  const double r = a.rho0 + drho;
  const double ub[3] = {jb[0] / r, jb[1] / r, jb[2] / r}, up[3] = {j[0] / r, j[1] / r, j[2] / r};
  const double sb = ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2];
  const double sp = up[0] * up[0] + up[1] * up[1] + up[2] * up[2];
  if (!csc) {
#pragma unroll
    for (int i = 0; i < Q; ++i)
      out[(long long)i * a.g.N + s] = fl[i] + feq_dev<double>(i, drho, r, up[0], up[1], up[2], sp) -
                                      feq_dev<double>(i, drho, r, ub[0], ub[1], ub[2], sb);
    return;
  }
  double ne[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) ne[i] = fl[i] - feq_dev<double>(i, drho, r, ub[0], ub[1], ub[2], sb);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double e = 0.5 * (ne[i] + ne[OPP[i]]), o = 0.5 * (ne[i] - ne[OPP[i]]);
    out[(long long)i * a.g.N + s] =
        feq_dev<double>(i, drho, r, up[0], up[1], up[2], sp) + gp * e + gm * o;
  }
}

// Local viscous stress pref * sum_i (f_i - f^eq_i(rho, u)) c_i c_i (order xx,
// yy, zz, xy, xz, yz).  The pending half force is an equilibrium shift and
// drops out, so the stored populations and their own velocity give it.
template <int S>
__global__ void k_stress(SiteArgs a, double* out, double pref, double prefb) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= a.g.nx) return;
  double fl[Q], drho, j[3];
  site_phys<S>(a, x, y, z, fl, drho, j, false);
  const double r = a.rho0 + drho;
  const double u[3] = {j[0] / r, j[1] / r, j[2] / r};
  const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double p[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double ne = fl[i] - feq_dev<double>(i, drho, r, u[0], u[1], u[2], usq);
    p[0] += ne * (CX[i] * CX[i]);
    p[1] += ne * (CY[i] * CY[i]);
    p[2] += ne * (CZ[i] * CZ[i]);
    p[3] += ne * (CX[i] * CY[i]);
    p[4] += ne * (CX[i] * CZ[i]);
    p[5] += ne * (CY[i] * CZ[i]);
  }
  const long long s = site_index(a.g, x, y, z);
  if (prefb != pref) {  // general MRT: the trace part relaxes at its own rate
    const double tr = (p[0] + p[1] + p[2]) / 3.0;
    for (int q = 0; q < 3; ++q) p[q] = pref * (p[q] - tr) + prefb * tr;
    for (int q = 3; q < 6; ++q) p[q] *= pref;
    for (int q = 0; q < 6; ++q) out[(long long)q * a.g.N + s] = p[q];
    return;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) out[(long long)q * a.g.N + s] = pref * p[q];
}

// Block reduction of 4 doubles in a fixed order (deterministic).
__device__ __forceinline__ void block_sum4(double v[4], double* lds /*[4*16]*/) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
    for (int k = 0; k < 4; ++k) lds[4 * wv + k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k) {
      double t = 0;
      for (int w = 0; w < nw; ++w) t += lds[4 * w + k];
      v[k] = t;
    }
  }
  __syncthreads();
}

template <int S>
__global__ __launch_bounds__(256) void k_totals_sites(SiteArgs a, double* partial) {
  __shared__ double lds[64];
  double v[4] = {0, 0, 0, 0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < a.g.N; s += stride) {
    const int x = (int)(s % a.g.nx);
    const long long r = s / a.g.nx;
    const int y = (int)(r % a.g.ny), z = (int)(r / a.g.ny);
    double fl[Q], drho, j[3];
    site_phys<S>(a, x, y, z, fl, drho, j, true);
    v[0] += drho;
    v[1] += j[0];
    v[2] += j[1];
    v[3] += j[2];
  }
  block_sum4(v, lds);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) partial[4 * blockIdx.x + k] = v[k];
}

__global__ __launch_bounds__(256) void k_totals_final(const double* partial, int nblk,
                                                      const double* vel, const double* mass,
                                                      long long np, double* out) {
  __shared__ double lds[64];
  double v[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
    for (int k = 0; k < 4; ++k) v[k] += partial[4 * b + k];
  block_sum4(v, lds);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) out[k] = v[k];
  double p[4] = {0, 0, 0, 0};
  if (vel && mass)
    for (long long i = threadIdx.x; i < np; i += blockDim.x)
      for (int k = 0; k < 3; ++k) p[k] += mass[i] * vel[3 * i + k];
  block_sum4(p, lds);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) out[4 + k] = p[k];
}

// ======================================================================
// Particle side: interpolation I (Eq. IBM-interpolation), spreading I*
// (Eq. IBM-spreading), coupling forces (Eq. modified-force, Eq.
// modified-ebf), velocity kicks and position drifts (Alg. 2 and 3).
//
// Work mapping: an aligned group of L lanes (L = 8, 32, 64 for the 2-, 3- and
// 4-point kernels, L >= K^3) handles one particle, one lane per stencil site,
// so the site gathers and the spreading atomics of a particle are issued in
// parallel.  Weighted sums are reduced inside the group with butterfly
// shuffles (fixed order), after which every lane holds the interpolated
// values and evaluates the (cheap, FP64) coupling update redundantly.
// ======================================================================
struct SiteSlot {
  bool site;   // the node lies in the box (not beyond a wall)
  bool valid;  // ... and carries a nonzero weight
  double W;
  int x, y, z;  // wrapped node
  int j0[3];    // first stencil node, unwrapped
};

template <int K>
__device__ __forceinline__ SiteSlot slot_of(const Geo& g, const double X[3], int lane) {
  SiteSlot s{false, false, 0.0, 0, 0, 0, {0, 0, 0}};
  for (int a = 0; a < 3; ++a) s.j0[a] = first_node<K>(X[a]);
  if (lane >= K * K * K) return s;
  const int kx = lane % K, ky = (lane / K) % K, kz = lane / (K * K);
  int yy = s.j0[1] + ky;
  if (g.wall) {
    if (yy < 0 || yy >= g.ny) return s;  // beyond a wall: no weight
  } else {
    yy = wrap_idx(yy, g.ny);
  }
  s.W = phi_eval(K, (double)(s.j0[0] + kx) - X[0]) * phi_eval(K, (double)(s.j0[1] + ky) - X[1]) *
        phi_eval(K, (double)(s.j0[2] + kz) - X[2]);
  s.site = true;
  s.valid = s.W != 0.0;
  s.x = wrap_idx(s.j0[0] + kx, g.nx);
  s.y = yy;
  s.z = wrap_idx(s.j0[2] + kz, g.nz);
  return s;
}

// Interpolated rho_p and u_p of particle p at X.  With a.cache_fill (second
// coupling half, post-stream moments without the pending force) every node in
// the box stores its gathered moments, also at zero weight, so that a later
// position with the same first node finds all of them; with a.cache_use and
// an unchanged first node the cached moments replace the gather, and the
// pending half force is added exactly as the gather would add it.
template <int S, int K>
__device__ __forceinline__ void group_interp(const PartArgs& a, const double X[3], bool phys,
                                             int lane, double& rp, double up[3], long long p,
                                             const void* const* gin = nullptr, int ngin = 0,
                                             const int4* pre_base = nullptr,
                                             const double4* pre_m = nullptr) {
  constexpr int L = Lanes<K>::L;
  const SiteSlot sl = slot_of<K>(a.s.g, X, lane);
  const bool fill = a.cache_fill != 0 && !phys;
  bool hit = false;
  if (a.cache_use) {  // (pre_base, pre_m: the entries, loaded by the caller)
    const int4 b = pre_base ? *pre_base : a.mbase[p];
    hit = b.x == sl.j0[0] && b.y == sl.j0[1] && b.z == sl.j0[2];
  }
  double r = 0, ux = 0, uy = 0, uz = 0;
  if (sl.site && (sl.valid || fill)) {
    double drho, j[3];
    if (hit) {
      const double4 m = pre_m ? *pre_m : a.mcache[p * L + lane];
      drho = m.x;
      j[0] = m.y;
      j[1] = m.z;
      j[2] = m.w;
      if (phys) add_pending<S>(a.s, site_index(a.s.g, sl.x, sl.y, sl.z), j);
    } else {
      double fl[Q];
      site_phys<S>(a.s, sl.x, sl.y, sl.z, fl, drho, j, phys);
      if (fill) a.mcache[p * L + lane] = make_double4(drho, j[0], j[1], j[2]);
    }
    if (phys && a.fa_rd) add_field<S>(a.FA, site_index(a.s.g, sl.x, sl.y, sl.z), j);
    for (int f = 0; f < ngin; ++f) add_field<S>(gin[f], site_index(a.s.g, sl.x, sl.y, sl.z), j);
    if (sl.valid) {
      const double rr = a.s.rho0 + drho;
      r = sl.W * rr;
      ux = sl.W * j[0] / rr;
      uy = sl.W * j[1] / rr;
      uz = sl.W * j[2] / rr;
    }
  }
  if (fill && lane == 0) a.mbase[p] = make_int4(sl.j0[0], sl.j0[1], sl.j0[2], 0);
  rp = group_sum<L>(r);
  up[0] = group_sum<L>(ux);
  up[1] = group_sum<L>(uy);
  up[2] = group_sum<L>(uz);
}

// The mask word of the lane's stencil node at X, loaded ahead of the
// spreading so that its latency overlaps the gathers: bits are only set while
// a coupling kernel runs (the lattice pass clears them between kernels), so a
// bit seen set stays set, and one seen clear is set with an atomic.  A plain,
// cached load (see flag_site).
template <int K>
__device__ __forceinline__ uint64_t mask_preload(const PartArgs& a, const double X[3], int lane) {
  const SiteSlot sl = slot_of<K>(a.s.g, X, lane);
  if (!sl.valid) return ~0ull;
  uint64_t bit;
  return *mask_word(a.mask, a.s.g, sl.x, sl.y, sl.z, bit);
}

// Spread W F to the lane's stencil node; pre: the node's mask word from
// mask_preload at the same X (nullptr: load it here).
template <typename E, int K>
__device__ __forceinline__ void group_spread(const PartArgs& a, const double X[3],
                                             const double F[3], void* field, int lane,
                                             const uint64_t* pre = nullptr) {
  const SiteSlot sl = slot_of<K>(a.s.g, X, lane);
  if (!sl.valid) return;
  E* Fd = (E*)field;
  const long long s = site_index(a.s.g, sl.x, sl.y, sl.z);
  unsafeAtomicAdd(Fd + 4 * s + 0, (E)(sl.W * F[0]));
  unsafeAtomicAdd(Fd + 4 * s + 1, (E)(sl.W * F[1]));
  unsafeAtomicAdd(Fd + 4 * s + 2, (E)(sl.W * F[2]));
  uint64_t bit;
  uint64_t* mw = mask_word(a.mask, a.s.g, sl.x, sl.y, sl.z, bit);
  if (pre) {
    if (!(*pre & bit)) atomicOr((unsigned long long*)mw, bit);
  } else {
    flag_site(mw, bit);
  }
}

// Spreading of the 2-point kernel with the contributions of consecutive
// particles combined inside the wavefront before the atomics.  A wavefront
// holds 8 particles (8 lanes each, one per stencil node); consecutive
// particles of a chain sit about one spacing apart, so particle q + 1 shares
// on average three to four of its nodes with particle q.  From the last
// particle of the wavefront down to the second, each particle hands the
// (already combined) contribution of every node it shares with its
// predecessor to the predecessor's lane for that node, which adds it in FP64;
// only nodes that are not handed on issue the three float atomics.  The sum at
// a site is the same set of terms as with one atomic per contribution (the
// order of atomic additions is unspecified either way).
//
// Which lanes pair up follows from the particles' first nodes alone (read
// from lanes 8q into scalars): the predecessor's node k' is the successor's
// node k' - d, d the difference of their first nodes, and a pair counts when
// both lanes carry weight (a ballot).  Only the contributions themselves move
// between lanes, one shuffle round per particle.  pre: the node's mask word
// from mask_preload.
template <typename E>
__device__ __forceinline__ void group_spread_k2(const PartArgs& a, const double X[3],
                                                const double F[3], void* field, int lane,
                                                long long p, uint64_t pre) {
  const SiteSlot sl = slot_of<2>(a.s.g, X, lane);
  const long long sidx = sl.valid ? site_index(a.s.g, sl.x, sl.y, sl.z) : -1;
  double c0 = sl.valid ? sl.W * F[0] : 0.0, c1 = sl.valid ? sl.W * F[1] : 0.0,
         c2 = sl.valid ? sl.W * F[2] : 0.0;
  const int wl = (int)(threadIdx.x & 63), qi = wl >> 3;
  const int kx = lane & 1, ky = (lane >> 1) & 1, kz = lane >> 2;
  const uint64_t live = __ballot(sidx >= 0);  // lanes that carry weight
  const bool next = p + 1 < a.n;              // particle qi + 1 exists
  bool issue = sidx >= 0;
  int jx[8], jy[8], jz[8];  // first node of each particle of the wavefront
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    jx[q] = __builtin_amdgcn_readlane(sl.j0[0], 8 * q);
    jy[q] = __builtin_amdgcn_readlane(sl.j0[1], 8 * q);
    jz[q] = __builtin_amdgcn_readlane(sl.j0[2], 8 * q);
  }
#pragma unroll
  for (int i = 7; i >= 1; --i) {
    const int dx = jx[i] - jx[i - 1], dy = jy[i] - jy[i - 1], dz = jz[i] - jz[i - 1];
    // receiver (particle i - 1, node k'): its node k' - d of particle i
    const int sx = kx - dx, sy = ky - dy, sz = kz - dz;
    const bool rin = qi == i - 1 && next && sx >= 0 && sx <= 1 && sy >= 0 && sy <= 1 &&
                     sz >= 0 && sz <= 1;
    const int src = rin ? 8 * i + sx + 2 * sy + 4 * sz : wl;
    // donor (particle i, node k): the receiver's node k + d of particle i - 1
    const int tx = kx + dx, ty = ky + dy, tz = kz + dz;
    const bool din = qi == i && tx >= 0 && tx <= 1 && ty >= 0 && ty <= 1 && tz >= 0 && tz <= 1;
    const int dst = 8 * (i - 1) + tx + 2 * ty + 4 * tz;
    const double g0 = __shfl(c0, src, 64), g1 = __shfl(c1, src, 64), g2 = __shfl(c2, src, 64);
    if (rin && sidx >= 0 && ((live >> src) & 1)) {
      c0 += g0;
      c1 += g1;
      c2 += g2;
    }
    if (din && sidx >= 0 && ((live >> dst) & 1)) issue = false;  // handed on to particle i - 1
  }
  if (!issue) return;
  E* Fd = (E*)field;
  unsafeAtomicAdd(Fd + 4 * sidx + 0, (E)c0);
  unsafeAtomicAdd(Fd + 4 * sidx + 1, (E)c1);
  unsafeAtomicAdd(Fd + 4 * sidx + 2, (E)c2);
  uint64_t bit;
  uint64_t* mw = mask_word(a.mask, a.s.g, sl.x, sl.y, sl.z, bit);
  if (!(pre & bit)) atomicOr((unsigned long long*)mw, bit);
}

__device__ __forceinline__ void wrap3(const Geo& g, double r[3]) {
  r[0] = wrap_pos(r[0], (double)g.nx);
  if (!g.wall) r[1] = wrap_pos(r[1], (double)g.ny);
  r[2] = wrap_pos(r[2], (double)g.nz);
}

// P^1/2: r <- r + (h/2) v, wrapped (first drift of Alg. 3).
__global__ void k_drift(Geo g, long long n, double* pos, const double* vel, double dt) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double r[3];
  for (int k = 0; k < 3; ++k) r[k] = pos[3 * p + k] + dt * vel[3 * p + k];
  wrap3(g, r);
  for (int k = 0; k < 3; ++k) pos[3 * p + k] = r[k];
}

__global__ void k_wrap(Geo g, long long n, double* pos) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double r[3] = {pos[3 * p], pos[3 * p + 1], pos[3 * p + 2]};
  wrap3(g, r);
  for (int k = 0; k < 3; ++k) pos[3 * p + k] = r[k];
}

// F^h over the coupling step a.hh from the interpolated rho_p, u_p, and the
// kick of v: the Crank-Nicolson solution of Eq. fc-vel (Eq. modified-force)
// for force coupling, Eq. modified-ebf for the modified EBF.
__device__ __forceinline__ void couple_update(const PartArgs& a, long long p, double m, double rp,
                                              const double up[3], const double Fi[3], double v[3],
                                              double Fh[3]) {
  const double hh = a.hh, al = a.gamma * hh / m, be = a.gamma * hh / rp;
  if (a.coupling == LB_COUPLE_FC) {
    const double den = 1.0 + 0.5 * al + 0.5 * be;
    double zeta[4] = {0, 0, 0, 0};
    if (a.kT > 0.0) {
      // random force of Eq. viscous-coupling: variance 2 k_B T gamma / hh per
      // component, entering the implicit solution like the drag; deviates from
      // the Philox block (particle, step low, 2^16 + coupling step, step high)
      normals4<double>(philox(make_uint4((uint32_t)p, a.t0, 65536u + (uint32_t)a.jc, a.t1),
                              a.key0, a.key1), zeta);
      const double sig = sqrt(2.0 * a.kT * a.gamma / hh);
      for (int k = 0; k < 3; ++k) zeta[k] = sig * zeta[k] / den;
    }
    // Crank-Nicolson solution of Eq. fc-vel over hh (Eq. modified-force), the
    // fluid at the particle also accelerated by the body force: +(beta/2) F_ext
    for (int k = 0; k < 3; ++k) {
      Fh[k] = -(a.gamma * (v[k] - up[k]) + 0.5 * al * Fi[k] - 0.5 * be * a.fext[k]) / den;
      if (a.kT > 0.0) Fh[k] += zeta[k];
      v[k] += hh / m * (Fh[k] + Fi[k]);
    }
  } else {
    const double sm = al + be;
    for (int k = 0; k < 3; ++k) {
      const double d = v[k] - up[k];
      Fh[k] = -a.gamma / sm * d - al / sm * Fi[k];
      v[k] = v[k] - al / sm * d + (hh / m) * (be / sm) * Fi[k];
    }
  }
}

// One coupling step for FC / modified EBF: interpolate rho_p, u_p at r,
// compute F^h over h' = a.hh (h/2 for the half steps of Alg. 3, h/2n for the
// sub-steps of Eq. multistep), kick v, optionally drift, and spread -F^h
// (scaled by a.sw) or store it for the deterministic spread.
template <int S, int K>
__global__ __launch_bounds__(256) void k_couple_half(PartArgs a) {
  using E = typename Store<S>::R;
  constexpr int L = Lanes<K>::L;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long p = gid / L;
  const int lane = (int)(gid % L);
  if (p >= a.n) return;  // whole groups leave together
  double r[3], v[3], Fi[3] = {0, 0, 0};
  for (int k = 0; k < 3; ++k) {
    r[k] = a.pos[3 * p + k];
    v[k] = a.vel[3 * p + k];
    if (a.use_fint) Fi[k] = a.fint[3 * p + k];
  }
  if (a.drift_before) {  // P^1/2: r <- wrap(r + (h/2) v), as k_drift does
    for (int k = 0; k < 3; ++k) r[k] += a.hd * v[k];
    wrap3(a.s.g, r);
  }
  const uint64_t mpre = a.defer ? ~0ull : mask_preload<K>(a, r, lane);
  const double m = a.mass[p];
  double rp, up[3];
  group_interp<S, K>(a, r, a.phys != 0, lane, rp, up, p);
  double Fh[3];
  couple_update(a, p, m, rp, up, Fi, v, Fh);
  const double Ff[3] = {-a.sw * Fh[0], -a.sw * Fh[1], -a.sw * Fh[2]};
  if (a.defer) {
    if (lane == 0)
      for (int k = 0; k < 3; ++k) a.defer[3 * p + k] = Ff[k];
  } else {
    if constexpr (K == 2)
      group_spread_k2<E>(a, r, Ff, a.target ? a.FB : a.FA, lane, p, mpre);
    else
      group_spread<E, K>(a, r, Ff, a.target ? a.FB : a.FA, lane, &mpre);
  }
  if (lane == 0) {
    if (a.drift_after) {
      for (int k = 0; k < 3; ++k) r[k] += a.hd * v[k];
      wrap3(a.s.g, r);
    }
    if (a.drift_after || a.drift_before)
      for (int k = 0; k < 3; ++k) a.pos[3 * p + k] = r[k];
    for (int k = 0; k < 3; ++k) a.vel[3 * p + k] = v[k];
  }
}

// ----------------------------------------------- deterministic spreading
// Spreading (Eq. IBM-spreading) as an exact sum: every contribution W F is
// converted to a 128-bit fixed-point number q 2^-96 (two's complement, words
// lo and hi) and added to the site's accumulator with 64-bit integer
// atomics.  Integer addition is associative, so the sum does not depend on
// the order in which the contributions arrive; a finalize pass then adds the
// converted sum to the force field.  Range: contributions below 2^20 in
// magnitude (larger or non-finite ones become a marker that reads back as
// NaN), resolution 2^-96.
constexpr int kFixShift = 96;

__device__ __forceinline__ void to_fixed(double c, uint64_t& lo, uint64_t& hi) {
  const double a = fabs(c);
  if (!(a < 1048576.0)) {  // non-finite or beyond any force of a stable run
    lo = 0ull;
    hi = 1ull << 56;
    return;
  }
  lo = hi = 0ull;
  if (a == 0.0) return;
  int e;
  const double m = frexp(a, &e);                     // a = m 2^e, m in [1/2, 1)
  const uint64_t mant = (uint64_t)ldexp(m, 53);      // exact 53-bit integer
  const int sh = e - 53 + kFixShift;                 // a 2^96 = mant 2^sh, sh < 64
  if (sh > 0) {
    lo = mant << sh;
    hi = mant >> (64 - sh);
  } else if (sh > -64) {
    lo = mant >> (-sh);  // truncation below the resolution
  }
  if (c < 0.0) {
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
  }
}

__device__ __forceinline__ double from_fixed(uint64_t lo, uint64_t hi) {
  const bool neg = (int64_t)hi < 0;
  if (neg) {
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
  }
  if (hi >= (1ull << 54)) return __builtin_nan("");  // the marker of a non-finite contribution
  const double v = ldexp((double)hi, 64 - kFixShift) + ldexp((double)lo, -kFixShift);
  return neg ? -v : v;
}

// q += (lo, hi) modulo 2^128: the carry out of the low word is known from the
// value the low atomic returns, so the result is exact whatever the order.
__device__ __forceinline__ void fixed_add(uint64_t* q, uint64_t lo, uint64_t hi) {
  const uint64_t old = (uint64_t)atomicAdd((unsigned long long*)q, (unsigned long long)lo);
  const uint64_t h = hi + (old + lo < old ? 1ull : 0ull);
  if (h) atomicAdd((unsigned long long*)(q + 1), (unsigned long long)h);
}

// Adds W F of every particle (positions X, lattice forces F [n][3]) to the
// fixed-point accumulator acc [N][3][2] at its stencil nodes and flags them;
// then the closing drift of the coupling step when a.drift_after (X = a.pos).
template <int K>
__global__ __launch_bounds__(256) void k_spread_det(PartArgs a, const double* X, const double* F,
                                                    uint64_t* acc) {
  constexpr int L = Lanes<K>::L;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long p = gid / L;
  const int lane = (int)(gid % L);
  if (p >= a.n) return;  // whole groups leave together
  double r[3], f[3];
  for (int k = 0; k < 3; ++k) {
    r[k] = X[3 * p + k];
    f[k] = F[3 * p + k];
  }
  const SiteSlot sl = slot_of<K>(a.s.g, r, lane);
  if (sl.valid) {
    const long long s = site_index(a.s.g, sl.x, sl.y, sl.z);
    for (int k = 0; k < 3; ++k) {
      uint64_t lo, hi;
      to_fixed(sl.W * f[k], lo, hi);
      if (lo | hi) fixed_add(acc + 6 * s + 2 * k, lo, hi);
    }
    uint64_t bit;
    flag_site(mask_word(a.mask, a.s.g, sl.x, sl.y, sl.z, bit), bit);
  }
  if (lane == 0 && a.drift_after) {
    for (int k = 0; k < 3; ++k) r[k] += a.hd * a.vel[3 * p + k];
    wrap3(a.s.g, r);
    for (int k = 0; k < 3; ++k) a.pos[3 * p + k] = r[k];
  }
}

// field += the accumulated sum at site s if it is flagged, and the
// accumulator back to zero there (one lane per site: no two lanes touch a site).
template <typename E>
__device__ __forceinline__ void det_finalize_site(const Geo& g, const uint64_t* mask,
                                                  uint64_t* acc, E* field, long long s) {
  const int x = (int)(s % g.nx);
  const long long r = s / g.nx;
  const int y = (int)(r % g.ny), z = (int)(r / g.ny);
  uint64_t bit;
  const uint64_t w = *mask_word(const_cast<uint64_t*>(mask), g, x, y, z, bit);
  if (!(w & bit)) return;
  uint64_t* q = acc + 6 * s;
  for (int k = 0; k < 3; ++k) {
    const uint64_t lo = q[2 * k], hi = q[2 * k + 1];
    if (!(lo | hi)) continue;
    field[4 * s + k] += (E)from_fixed(lo, hi);
    q[2 * k] = 0ull;
    q[2 * k + 1] = 0ull;
  }
}

template <typename E>
__global__ __launch_bounds__(256) void k_det_finalize(Geo g, const uint64_t* mask, uint64_t* acc,
                                                      E* field) {
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < g.N) det_finalize_site<E>(g, mask, acc, field, s);
}

// IB (Alg. 2): predictor X~ = X + (h/2) I[X] u(t)
template <int S, int K>
__global__ __launch_bounds__(256) void k_ib_predict(PartArgs a) {
  constexpr int L = Lanes<K>::L;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long p = gid / L;
  const int lane = (int)(gid % L);
  if (p >= a.n) return;
  double X[3] = {a.pos[3 * p], a.pos[3 * p + 1], a.pos[3 * p + 2]}, rp, up[3];
  group_interp<S, K>(a, X, true, lane, rp, up, p);
  if (lane == 0) {
    for (int k = 0; k < 3; ++k) X[k] += 0.5 * up[k];
    wrap3(a.s.g, X);
    for (int k = 0; k < 3; ++k) a.aux[3 * p + k] = X[k];
  }
}

// IB: X <- X + (h/2) I[X~] u with the current physical u; with spread_fint
// also spreads +F_int at X~ into the A field (first half force).
template <int S, int K>
__global__ __launch_bounds__(256) void k_ib_advect(PartArgs a, int spread_fint) {
  using E = typename Store<S>::R;
  constexpr int L = Lanes<K>::L;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long p = gid / L;
  const int lane = (int)(gid % L);
  if (p >= a.n) return;
  const double Xt[3] = {a.aux[3 * p], a.aux[3 * p + 1], a.aux[3 * p + 2]};
  double rp, up[3];
  group_interp<S, K>(a, Xt, true, lane, rp, up, p);
  if (lane == 0) {
    double X[3];
    for (int k = 0; k < 3; ++k) X[k] = a.pos[3 * p + k] + 0.5 * up[k];
    wrap3(a.s.g, X);
    for (int k = 0; k < 3; ++k) a.pos[3 * p + k] = X[k];
  }
  if (spread_fint) {
    const double F[3] = {a.fint[3 * p], a.fint[3 * p + 1], a.fint[3 * p + 2]};
    group_spread<E, K>(a, Xt, F, a.FA, lane);
  }
}

// ======================================================================
// Intrinsic forces.
// ======================================================================

// Bonded groups: block b owns the particles perm[goff[b] .. goff[b+1]), a
// union of whole bonded clusters, so every bond partner is in the block's
// LDS.  mode 0: F_int at the current positions (stored, or added with acc).
// mode 1: nsub velocity-Verlet sub-steps of length dt with F_int only
// (the [P F_int P]^n factor of the multiple time-step split, Sec. 6).
// mode 2: the positions drift by dt (r <- wrap(r + dt v)), then mode 0.
// Bond partners of one particle, held in registers across the sub-steps
// (up to kMaxBondsReg; a particle with more partners reads the CSR list).
constexpr int kMaxBondsReg = 6;

struct Partners {
  int n;
  long long p;
  int loc[kMaxBondsReg];
};

__device__ __forceinline__ void load_partners(const BondArgs& b, long long p, Partners& P) {
  const int e0 = b.start[p], e1 = b.start[p + 1];
  P.p = p;
  P.n = e1 - e0;
#pragma unroll
  for (int k = 0; k < kMaxBondsReg; ++k) P.loc[k] = (k < P.n) ? b.loc[b.nbr[e0 + k]] : 0;
}

__device__ __forceinline__ void bond_pair(const BondArgs& b, const double r[3], const double* q,
                                          double F[3]) {
  double d[3];
  for (int k = 0; k < 3; ++k) d[k] = q[k] - r[k];
  d[0] -= b.g.nx * floor(d[0] / b.g.nx + 0.5);
  if (!b.g.wall) d[1] -= b.g.ny * floor(d[1] / b.g.ny + 0.5);
  d[2] -= b.g.nz * floor(d[2] / b.g.nz + 0.5);
  const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double s;
  if (b.type == LB_FENE)  // infinite energy from L = r0 on: NaN, not the formula's sign flip
    s = L < b.r0 ? b.k / (1.0 - L * L / (b.r0 * b.r0)) : __builtin_nan("");
  else
    s = L > 0.0 ? b.k * (L - b.r0) / L : 0.0;
  for (int k = 0; k < 3; ++k) F[k] += s * d[k];
}

__device__ __forceinline__ void bond_force(const BondArgs& b, const Partners& P, const double r[3],
                                           const double* lds, double F[3]) {
  F[0] = F[1] = F[2] = 0;
  if (P.n <= kMaxBondsReg) {
#pragma unroll
    for (int k = 0; k < kMaxBondsReg; ++k)
      if (k < P.n) bond_pair(b, r, lds + 3 * P.loc[k], F);
  } else {
    for (int e = b.start[P.p]; e < b.start[P.p + 1]; ++e) bond_pair(b, r, lds + 3 * b.loc[b.nbr[e]], F);
  }
}

__device__ __forceinline__ void bond_group(const BondArgs& b, int grp, int mode, int acc, int nsub,
                                           double dt, double* lds) {
  const int g0 = b.goff[grp], cnt = b.goff[grp + 1] - g0;
  const int t = threadIdx.x;
  const bool on = t < cnt;
  const long long p = on ? b.perm[g0 + t] : 0;
  double r[3] = {0, 0, 0}, v[3] = {0, 0, 0}, m = 1.0;
  Partners P;
  P.n = 0;
  P.p = p;
  if (on) {
    for (int k = 0; k < 3; ++k) {
      r[k] = b.pos[3 * p + k];
      v[k] = b.vel ? b.vel[3 * p + k] : 0.0;
    }
    if (b.mass) m = b.mass[p];
    load_partners(b, p, P);
  }
  if (mode == 0 || mode == 2) {
    if (mode == 2 && on) {  // drift by dt first (as k_drift does), store the positions
      for (int k = 0; k < 3; ++k) r[k] = r[k] + dt * v[k];
      wrap3(b.g, r);
      for (int k = 0; k < 3; ++k) b.pos[3 * p + k] = r[k];
    }
    if (on)
      for (int k = 0; k < 3; ++k) lds[3 * t + k] = r[k];
    __syncthreads();
    if (on) {
      double F[3];
      bond_force(b, P, r, lds, F);
      for (int k = 0; k < 3; ++k) b.fint[3 * p + k] = acc ? b.fint[3 * p + k] + F[k] : F[k];
    }
    return;
  }
  const double dtm = dt / m;
  for (int s = 0; s < nsub; ++s) {
    if (on) {
      for (int k = 0; k < 3; ++k) r[k] += 0.5 * dt * v[k];
      wrap3(b.g, r);
    }
    __syncthreads();
    if (on)
      for (int k = 0; k < 3; ++k) lds[3 * t + k] = r[k];
    __syncthreads();
    if (on) {
      double F[3];
      bond_force(b, P, r, lds, F);
      for (int k = 0; k < 3; ++k) {
        v[k] += dtm * F[k];
        r[k] += 0.5 * dt * v[k];
      }
      wrap3(b.g, r);
    }
  }
  if (on)
    for (int k = 0; k < 3; ++k) {
      b.pos[3 * p + k] = r[k];
      b.vel[3 * p + k] = v[k];
    }
}

__global__ void k_bond_groups(BondArgs b, int mode, int acc, int nsub, double dt) {
  extern __shared__ double lds[];
  bond_group(b, blockIdx.x, mode, acc, nsub, dt, lds);
}

// One coupled sub-step of Eq. multistep in one launch (SubArgs): drift dt/2 to
// the midpoint, F_int there (each particle advances its bond partners itself,
// with the same arithmetic as their own drift), interpolation of the fluid
// that every earlier sub-step has forced, F^h and kick over dt, spread of the
// lattice force at the midpoint, drift dt/2.  Everything that depends only on
// the particle index (its state, partner list and cached moments) is loaded
// first, and the partners' state is loaded before the interpolation's gathers
// but used after them, so that the launch waits on about three memory round
// trips: state, gathers, spreading atomics.
template <int S, int K>
__global__ __launch_bounds__(256) void k_mts_substep(PartArgs a, SubArgs u) {
  using E = typename Store<S>::R;
  constexpr int L = Lanes<K>::L;
  constexpr int NP = kSubPartners;
  static_assert(NP == 3, "the packed partner entry holds three partners");
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long p = gid / L;
  const int lane = (int)(gid % L);
  if (p >= a.n) return;  // whole groups leave together
  double pi[3], v[3];
  for (int k = 0; k < 3; ++k) {
    pi[k] = u.pin[3 * p + k];
    v[k] = u.vin[3 * p + k];
  }
  const int4 pn = u.bonds ? u.pn[p] : make_int4(0, 0, 0, 0);
  const double m = a.mass[p];
  int4 mb = make_int4(0, 0, 0, 0);
  double4 mc = make_double4(0, 0, 0, 0);
  if (a.cache_use) {
    mb = a.mbase[p];
    mc = a.mcache[p * L + lane];
  }
  double r[3];
  for (int k = 0; k < 3; ++k) r[k] = pi[k] + a.hd * v[k];
  wrap3(a.s.g, r);
  // the partners' start-of-sub-step state (pn.w <= NP: partners in pn.x..z)
  const int qs[3] = {pn.x, pn.y, pn.z};
  double pq[NP][3], vq[NP][3];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const long long q = j < pn.w ? qs[j] : p;
    for (int k = 0; k < 3; ++k) {
      pq[j][k] = u.pin[3 * q + k];
      vq[j][k] = u.vin[3 * q + k];
    }
  }
  const uint64_t mpre = mask_preload<K>(a, r, lane);
  double rp, up[3];
  group_interp<S, K>(a, r, a.phys != 0, lane, rp, up, p, u.gin, u.ngin, &mb, &mc);
  double Fi[3] = {0, 0, 0};
  if (pn.w <= NP) {
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      if (j < pn.w) {
        double rq[3];
        for (int k = 0; k < 3; ++k) rq[k] = pq[j][k] + a.hd * vq[j][k];
        wrap3(a.s.g, rq);
        bond_pair(u.b, r, rq, Fi);
      }
    }
  } else {  // more partners than held in registers: the CSR list
    for (int e = u.b.start[p]; e < u.b.start[p + 1]; ++e) {
      const long long q = u.b.nbr[e];
      double rq[3];
      for (int k = 0; k < 3; ++k) rq[k] = u.pin[3 * q + k] + a.hd * u.vin[3 * q + k];
      wrap3(a.s.g, rq);
      bond_pair(u.b, r, rq, Fi);
    }
  }
  double Fh[3];
  couple_update(a, p, m, rp, up, Fi, v, Fh);
  const double Ff[3] = {-a.sw * Fh[0], -a.sw * Fh[1], -a.sw * Fh[2]};
  void* field = u.gout ? u.gout : (a.target ? a.FB : a.FA);
  if constexpr (K == 2)
    group_spread_k2<E>(a, r, Ff, field, lane, p, mpre);
  else
    group_spread<E, K>(a, r, Ff, field, lane, &mpre);
  if (lane == 0) {
    for (int k = 0; k < 3; ++k) r[k] += a.hd * v[k];
    wrap3(a.s.g, r);
    for (int k = 0; k < 3; ++k) {
      u.pout[3 * p + k] = r[k];
      u.vout[3 * p + k] = v[k];
    }
  }
}

// The sub-step fields into the target field at every flagged site (every
// nonzero entry of a field lies on a site its spread flagged), one lane per
// site: no two lanes share a site, so plain loads and stores suffice.  The
// fields are left zero.
template <int S>
__global__ __launch_bounds__(256) void k_mts_fold(Geo g, const uint64_t* __restrict__ mask,
                                                  long long nwords, SubArgs u, int nf, void* T) {
  using V4 = typename Store<S>::V4;
  for_flagged_sites<64>(g, mask, nwords, [&](int x, int y, int z) {
    const long long s = site_index(g, x, y, z);
    V4 t = ((const V4*)T)[s];
    bool any = false;
    for (int f = 0; f < nf; ++f) {
      V4* G = (V4*)u.gin[f];
      const V4 w = G[s];
      if (w.x != 0 || w.y != 0 || w.z != 0) {
        t.x += w.x;
        t.y += w.y;
        t.z += w.z;
        G[s] = V4{0, 0, 0, 0};
        any = true;
      }
    }
    if (any) ((V4*)T)[s] = t;
  });
}

// ======================================================================
// Launchers (host side)
// ======================================================================
static dim3 lattice_block(const Geo& g) {
  int bx = ((g.nx + 63) / 64) * 64;
  if (bx > 256) bx = 256;
  return dim3(bx, 1, 1);
}
static dim3 lattice_grid(const Geo& g, dim3 b) {
  return dim3((g.nx + b.x - 1) / b.x, g.ny, g.nz);
}

#define LBC_STORAGE_SWITCH(S, CALL)                                 \
  switch (S) {                                                      \
    case LB_F64: { constexpr int SS = LB_F64; CALL; } break;        \
    case LB_F32: { constexpr int SS = LB_F32; CALL; } break;        \
    case LB_F16: { constexpr int SS = LB_F16; CALL; } break;        \
    default: { constexpr int SS = LB_BF16; CALL; } break;           \
  }

template <int S, bool CM, bool WALL, bool NS, bool MRT, bool SG>
__global__ __launch_bounds__(256) void k_stream_collide_lin(LatArgs a);

template <bool CM, bool WALL, bool NS = false, bool MRT = false, bool SG = false>
static void launch_sc(int storage, const LatArgs& a, dim3 gr, dim3 b, hipStream_t st) {
  if (a.g.wpr == 0) {  // linear mask: x extent not a multiple of 64
    const unsigned nb = (unsigned)((a.g.N + 255) / 256) + (unsigned)a.bond_groups;
    LBC_STORAGE_SWITCH(storage, (k_stream_collide_lin<SS, CM, WALL, NS, MRT, SG>
                                 <<<nb, 256, a.occ_lds, st>>>(a)));
  } else {
    LBC_STORAGE_SWITCH(storage,
                       (k_stream_collide<SS, CM, WALL, NS, MRT, SG><<<gr, b, a.occ_lds, st>>>(a)));
  }
}

// BGK and the two-rate collision share one kernel (BGK: equal rates); the
// comoving storage frame is a compile-time switch so that the rest frame
// carries none of its arithmetic.
hipError_t launch_stream_collide(int storage, bool comoving, const LatArgs& a_in, hipStream_t st) {
  const dim3 b = lattice_block(a_in.g);
  dim3 gr = lattice_grid(a_in.g, b);
  LatArgs a = a_in;
  if (a.bond_groups > 0) {  // extra workgroups run the bond groups
    if (a.occ_lds < a.bond_cap * 3 * (int)sizeof(double)) return hipErrorInvalidValue;
    if (a.g.wpr == 0) {  // linear-site pass: bond_groups workgroups in front
      if (a.bond_cap > 256) return hipErrorInvalidValue;
    } else {  // row-mapped pass: one more z slab of workgroups in front
      if ((unsigned)a.bond_groups > gr.x * gr.y || a.bond_cap > (int)b.x) return hipErrorInvalidValue;
      gr.z += 1;
    }
  }
  if (a.mrt) {  // general MRT (not with the comoving frame), with or without noise
    if (a.noise) {
      if (a.g.wall) launch_sc<false, true, true, true>(storage, a, gr, b, st);
      else launch_sc<false, false, true, true>(storage, a, gr, b, st);
    } else {
      if (a.g.wall) launch_sc<false, true, false, true>(storage, a, gr, b, st);
      else launch_sc<false, false, false, true>(storage, a, gr, b, st);
    }
  } else if (a.noise) {  // fluctuating collision (the comoving frame is not combined with it)
    if (a.g.wall) launch_sc<false, true, true>(storage, a, gr, b, st);
    else launch_sc<false, false, true>(storage, a, gr, b, st);
  } else if (a.sigma) {  // the viscous stress of the state the pass starts from, written out
    if (comoving) {
      if (a.g.wall) launch_sc<true, true, false, false, true>(storage, a, gr, b, st);
      else launch_sc<true, false, false, false, true>(storage, a, gr, b, st);
    } else {
      if (a.g.wall) launch_sc<false, true, false, false, true>(storage, a, gr, b, st);
      else launch_sc<false, false, false, false, true>(storage, a, gr, b, st);
    }
  } else if (comoving) {
    if (a.g.wall) launch_sc<true, true>(storage, a, gr, b, st);
    else launch_sc<true, false>(storage, a, gr, b, st);
  } else {
    if (a.g.wall) launch_sc<false, true>(storage, a, gr, b, st);
    else launch_sc<false, false>(storage, a, gr, b, st);
  }
  return hipGetLastError();
}

hipError_t launch_init(int storage, const InitArgs& a, hipStream_t st) {
  const dim3 b = lattice_block(a.g), gr = lattice_grid(a.g, b);
  LBC_STORAGE_SWITCH(storage, (k_init<SS><<<gr, b, 0, st>>>(a)));
  return hipGetLastError();
}

hipError_t launch_moments(int storage, const SiteArgs& a, double* rho, double* u, hipStream_t st) {
  const dim3 b = lattice_block(a.g), gr = lattice_grid(a.g, b);
  LBC_STORAGE_SWITCH(storage, (k_moments<SS><<<gr, b, 0, st>>>(a, rho, u)));
  return hipGetLastError();
}

hipError_t launch_populations(int storage, const SiteArgs& a, double* out, double gp, double gm,
                              hipStream_t st) {
  const dim3 b = lattice_block(a.g), gr = lattice_grid(a.g, b);
  const int csc = gp != 1.0 || gm != 1.0;
  LBC_STORAGE_SWITCH(storage, (k_populations<SS><<<gr, b, 0, st>>>(a, out, gp, gm, csc)));
  return hipGetLastError();
}

hipError_t launch_stress(int storage, const SiteArgs& a, double* out, double pref, double prefb,
                         hipStream_t st) {
  const dim3 b = lattice_block(a.g), gr = lattice_grid(a.g, b);
  LBC_STORAGE_SWITCH(storage, (k_stress<SS><<<gr, b, 0, st>>>(a, out, pref, prefb)));
  return hipGetLastError();
}

hipError_t launch_totals(int storage, const SiteArgs& a, double* partial, int nblk,
                         const double* vel, const double* mass, long long np, double* out,
                         hipStream_t st) {
  LBC_STORAGE_SWITCH(storage, (k_totals_sites<SS><<<nblk, 256, 0, st>>>(a, partial)));
  k_totals_final<<<1, 256, 0, st>>>(partial, nblk, vel, mass, np, out);
  return hipGetLastError();
}

static inline unsigned pblocks(long long n) { return (unsigned)((n + 127) / 128); }

hipError_t launch_drift(const Geo& g, long long n, double* pos, const double* vel, double dt,
                        hipStream_t st) {
  if (n > 0) k_drift<<<pblocks(n), 128, 0, st>>>(g, n, pos, vel, dt);
  return hipGetLastError();
}

hipError_t launch_wrap(const Geo& g, long long n, double* pos, hipStream_t st) {
  if (n > 0) k_wrap<<<pblocks(n), 128, 0, st>>>(g, n, pos);
  return hipGetLastError();
}

// Zero fill of n 8-byte words (a kernel, so that a caller capturing the
// library's calls in a HIP graph records kernel nodes only).
__global__ void k_zero(unsigned long long* p, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const long long n = (long long)(bytes / 8);
  if (n <= 0) return hipSuccess;
  const long long blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  k_zero<<<(unsigned)blocks, 256, 0, st>>>((unsigned long long*)p, n);
  return hipGetLastError();
}

#define LBC_KERNEL_SWITCH(K, CALL)                        \
  switch (K) {                                            \
    case 2: { constexpr int KK = 2; CALL; } break;        \
    case 3: { constexpr int KK = 3; CALL; } break;        \
    default: { constexpr int KK = 4; CALL; } break;       \
  }

static unsigned gblocks(long long n, int K) {
  const long long L = K == 2 ? 8 : (K == 3 ? 32 : 64);
  return (unsigned)((n * L + 255) / 256);
}

hipError_t launch_couple_half(int storage, const PartArgs& a, hipStream_t st) {
  if (a.n > 0)
    LBC_KERNEL_SWITCH(a.K, LBC_STORAGE_SWITCH(storage, (k_couple_half<SS, KK>
                                                        <<<gblocks(a.n, KK), 256, 0, st>>>(a))));
  return hipGetLastError();
}

hipError_t launch_mts_substep(int storage, const PartArgs& a, const SubArgs& u, hipStream_t st) {
  if (a.n > 0)
    LBC_KERNEL_SWITCH(a.K, LBC_STORAGE_SWITCH(storage, (k_mts_substep<SS, KK>
                                                        <<<gblocks(a.n, KK), 256, 0, st>>>(a, u))));
  return hipGetLastError();
}

hipError_t launch_mts_fold(int storage, const PartArgs& a, const SubArgs& u, int nf,
                           hipStream_t st) {
  if (nf <= 0) return hipSuccess;
  const Geo& g = a.s.g;
  const long long nwords = mask_nwords(g);
  const long long per_wg = 4ll * 64;  // 64 words per wavefront: the mask is sparse here
  const unsigned gr = (unsigned)std::min<long long>((nwords + per_wg - 1) / per_wg, 16384ll);
  void* T = a.target ? a.FB : a.FA;
  if (storage == LB_F64)
    k_mts_fold<LB_F64><<<gr, 256, 0, st>>>(g, a.mask, nwords, u, nf, T);
  else
    k_mts_fold<LB_F32><<<gr, 256, 0, st>>>(g, a.mask, nwords, u, nf, T);
  return hipGetLastError();
}

hipError_t launch_spread_det(const PartArgs& a, const double* X, const double* F, uint64_t* acc,
                             hipStream_t st) {
  if (a.n > 0)
    LBC_KERNEL_SWITCH(a.K, (k_spread_det<KK><<<gblocks(a.n, KK), 256, 0, st>>>(a, X, F, acc)));
  return hipGetLastError();
}

hipError_t launch_det_finalize(int storage, const Geo& g, const uint64_t* mask, uint64_t* acc,
                               void* field, hipStream_t st) {
  const unsigned nb = (unsigned)((g.N + 255) / 256);
  if (storage == LB_F64)
    k_det_finalize<double><<<nb, 256, 0, st>>>(g, mask, acc, (double*)field);
  else
    k_det_finalize<float><<<nb, 256, 0, st>>>(g, mask, acc, (float*)field);
  return hipGetLastError();
}

hipError_t launch_ib_predict(int storage, const PartArgs& a, hipStream_t st) {
  if (a.n > 0)
    LBC_KERNEL_SWITCH(a.K, LBC_STORAGE_SWITCH(storage, (k_ib_predict<SS, KK>
                                                        <<<gblocks(a.n, KK), 256, 0, st>>>(a))));
  return hipGetLastError();
}

hipError_t launch_ib_advect(int storage, const PartArgs& a, int spread_fint, hipStream_t st) {
  if (a.n > 0)
    LBC_KERNEL_SWITCH(a.K, LBC_STORAGE_SWITCH(storage, (k_ib_advect<SS, KK>
                                                        <<<gblocks(a.n, KK), 256, 0, st>>>(a, spread_fint))));
  return hipGetLastError();
}

hipError_t launch_bond_groups(const BondArgs& b, int ngroups, int gcap, int mode, int acc,
                              int nsub, double dt, hipStream_t st) {
  if (ngroups > 0)
    k_bond_groups<<<ngroups, gcap, (size_t)gcap * 3 * sizeof(double), st>>>(b, mode, acc, nsub, dt);
  return hipGetLastError();
}


// ======================================================================
// Batched ensemble step: many periodic boxes of different sizes advance
// together.  Every kernel is a persistent grid that strides over a flat work
// list: (slot, 256-site chunk) for the lattice, (slot, particle group) for
// the coupling halves.  A slot takes part while steps_done < steps_target;
// the per-slot state (ping-pong buffer, pending body-force half, step count)
// lives on the device, so a captured graph of steps stays valid while slots
// are admitted and retired.
// ======================================================================
__device__ __forceinline__ bool ens_active(const EnsSlot& s) {
  return s.live && s.steps_done < s.steps_target;
}

// Fused pass over linear site indices: a wavefront covers 64 consecutive
// sites whatever the row length, and owns one word of a linear force mask
// (wpr == 0).  Used by the batched ensemble pass and by single boxes whose x
// extent is not a multiple of 64 (where row-aligned wavefronts would idle
// lanes).  Site coordinates come from a 32-bit quotient by nx and ny.
// V is a view of the pass parameters (kernel arguments or a slot record);
// its accessors read them where they are used, so the compiler can reload
// them from memory instead of holding every one in scalar registers.
struct LatView {
  const LatArgs& a;
  __device__ const Geo& g() const { return a.g; }
  __device__ double rnx() const { return a.rnx; }
  __device__ double rny() const { return a.rny; }
  __device__ const void* fin() const { return a.fin; }
  __device__ void* fout() const { return a.fout; }
  __device__ void* FA() const { return a.FA; }
  __device__ void* FB() const { return a.FB; }
  __device__ uint64_t* mask() const { return a.mask; }
  __device__ double F(int c) const { return c == 0 ? a.Fx : (c == 1 ? a.Fy : a.Fz); }
  __device__ double rho0() const { return a.rho0; }
  __device__ float scale() const { return a.scale; }
  __device__ float inv() const { return a.inv; }
  __device__ double omp() const { return a.omp; }
  __device__ double omm() const { return a.omm; }
  __device__ double uin(int c) const { return a.uin[c]; }
  __device__ const double* cm() const { return a.cm; }
  __device__ const float* cmf() const { return a.cmf; }
  __device__ bool ib_copy() const { return a.ib_copy != 0; }
  __device__ bool clear_mask() const { return a.clear_mask != 0; }
  __device__ void* sigma() const { return a.sigma; }
  __device__ double sp() const { return a.sp; }
  template <typename R>
  __device__ void noise(PassK<R>& k) const {
    k.ap = R(a.ap);
    k.am = R(a.am);
    k.k0 = a.key0;
    k.k1 = a.key1;
    k.t0 = a.t0;
    k.t1 = a.t1;
  }
  template <typename R>
  __device__ void mrt(PassK<R>& k) const {
    for (int c = 0; c < 6; ++c) {
      k.lg[c] = R(a.lg[c]);
      k.ag[c] = R(a.ag[c]);
    }
  }
};

struct SlotView {
  const EnsSlot& s;
  __device__ const Geo& g() const { return s.g; }
  __device__ double rnx() const { return s.rnx; }
  __device__ double rny() const { return s.rny; }
  __device__ const void* fin() const { return s.f[s.cur]; }
  __device__ void* fout() const { return s.f[1 - s.cur]; }
  __device__ void* FA() const { return s.FA; }
  __device__ void* FB() const { return s.FB; }
  __device__ uint64_t* mask() const { return s.mask; }
  __device__ double F(int c) const {
    return (1 + s.pend) * (c == 0 ? s.fx : (c == 1 ? s.fy : s.fz));
  }
  __device__ double rho0() const { return s.rho0; }
  __device__ float scale() const { return s.scale; }
  __device__ float inv() const { return s.inv; }
  __device__ double omp() const { return s.omp; }
  __device__ double omm() const { return s.omm; }
  __device__ double uin(int c) const { return s.uref[c]; }
  __device__ const double* cm() const { return s.cm; }
  __device__ const float* cmf() const { return s.cmf; }
  __device__ bool ib_copy() const { return false; }
  __device__ bool clear_mask() const { return s.steps_done % kMaskKeep == 0; }
  __device__ void* sigma() const { return nullptr; }
  __device__ double sp() const { return 0.0; }
  template <typename R>
  __device__ void noise(PassK<R>&) const {}  // ensemble members are deterministic
  template <typename R>
  __device__ void mrt(PassK<R>&) const {}  // ... and use the two-rate collision
};

template <int S, bool CM, bool WALL, class V, bool NS = false, bool MRT = false, bool SG = false>
__device__ __forceinline__ void linear_site(const V& v, uint32_t s) {
  using St = Store<S>;
  using T = typename St::T;
  using R = typename St::R;
  const Geo& g = v.g();
  if (s >= (uint32_t)g.N) return;
  const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny, nz = (uint32_t)g.nz;
  const size_t P = (size_t)g.ps;  // population stride
  uint32_t x, y;
  const uint32_t r = div_rem(s, nx, v.rnx(), x);
  const uint32_t z = div_rem(r, ny, v.rny(), y);
  const uint32_t xs[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
  const uint32_t ys[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
  const uint32_t zr[3] = {(z == 0 ? nz - 1 : z - 1) * ny, z * ny, (z == nz - 1 ? 0 : z + 1) * ny};
  const T* __restrict__ fin = (const T*)v.fin();
  uint64_t* mp = v.mask() + (s >> 6);
  const uint64_t word = *mp;
  R f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const uint32_t off = (zr[1 - CZ[i]] + ys[1 - CY[i]]) * nx + xs[1 - CX[i]];
    const T* src = fin + (size_t)i * P + off;
    if (WALL && ((CY[i] == 1 && y == 0) || (CY[i] == -1 && y == ny - 1)))
      src = fin + (size_t)OPP[i] * P + s;  // halfway bounce-back: opposite population, same site
    f[i] = St::raw(src);
  }
  R Fx = R(v.F(0)), Fy = R(v.F(1)), Fz = R(v.F(2));
  if (word) {  // a 64-aligned group of 64 lanes owns this mask word
    if (v.ib_copy())
      take_forces_ib<S>(word, mp, s, s & 63, v.FA(), v.FB(), Fx, Fy, Fz);
    else
      take_forces<S>(word, mp, s, s & 63, v.FA(), v.FB(), v.clear_mask(), Fx, Fy, Fz);
  }
  PassK<R> k;
  k.rho0 = R(v.rho0());
  k.sc = R(v.scale());
  k.inv = R(v.inv());
  k.hp = R(0.5) * R(v.omp());
  k.hm = R(0.5) * R(v.omm());
  if (CM) {
    for (int c = 0; c < 3; ++c) k.ui[c] = R(v.uin(c));
  }
  k.cm = pick_terms<R>(v.cm(), v.cmf());
  if (NS) v.noise(k);
  if (MRT) {
    v.mrt(k);
    fused_site_mrt<S, NS>(f, Fx, Fy, Fz, k, (T*)v.fout(), P, s);
  } else {
    fused_site<S, CM, NS, SG>(f, Fx, Fy, Fz, k, (T*)v.fout(), P, s, (R*)v.sigma(), (size_t)g.N,
                              R(v.sp()));
  }
}

template <int S, bool CM, bool WALL, bool NS, bool MRT, bool SG>
__global__ __launch_bounds__(256) void k_stream_collide_lin(LatArgs a) {
  uint32_t b = blockIdx.x;
  if (a.bond_groups > 0) {  // the first bond_groups workgroups run the intrinsic-force sub-steps
    if (b < (uint32_t)a.bond_groups) {
      extern __shared__ double bond_lds[];
      bond_group(a.bond, (int)b, 1, 0, a.bond_nsub, a.bond_dt, bond_lds);
      return;
    }
    b -= (uint32_t)a.bond_groups;
  }
  linear_site<S, CM, WALL, LatView, NS, MRT, SG>(LatView{a}, b * 256u + threadIdx.x);
}

// The slot table is read-only during the lattice pass (only k_ens_advance
// writes it); with restrict-qualified arguments its fields are scalar loads.
template <int S, bool CM>
__device__ __forceinline__ void ens_lattice_item(const EnsSlot& sl, uint32_t chunk) {
  linear_site<S, CM, false>(SlotView{sl}, chunk * 256u + threadIdx.x);
}

template <int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S == LB_F64 ? 4 : 8))) void k_ens_lattice(const EnsSlot* __restrict__ slots,
                                                     const int2* __restrict__ items,
                                                     const int* __restrict__ nitems) {
  const int n = *nitems;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 w = items[it];
    const EnsSlot& sl = slots[w.x];
    if (!ens_active(sl)) continue;
    if (sl.comoving)
      ens_lattice_item<S, true>(sl, (uint32_t)w.y);
    else
      ens_lattice_item<S, false>(sl, (uint32_t)w.y);
  }
}

// half 0: P^1/2 then the first coupling half (physical u, spread into FA);
// half 1: the second coupling half (post-stream u, spread into FB), then P^1/2.
template <int S, int K>
__global__ __launch_bounds__(256) void k_ens_couple(EnsArgs e, int half) {
  using E = typename Store<S>::R;
  constexpr int L = Lanes<K>::L;
  const int n = *e.npitems;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 w = e.pitems[it];
    const EnsSlot& sl = e.slots[w.x];
    if (!ens_active(sl) || sl.coupling == LB_COUPLE_NONE) continue;
    const long long p = (long long)w.y + threadIdx.x / L;
    const int lane = threadIdx.x % L;
    if (p >= sl.np) continue;  // whole lane groups leave together
    PartArgs a;
    a.s.g = sl.g;
    a.s.f = half == 0 ? sl.f[sl.cur] : sl.f[1 - sl.cur];
    a.s.FB = sl.FB;
    a.s.rho0 = sl.rho0;
    a.s.pfx = sl.pend * sl.fx;
    a.s.pfy = sl.pend * sl.fy;
    a.s.pfz = sl.pend * sl.fz;
    a.s.inv = sl.inv;
    for (int k = 0; k < 3; ++k) {  // reference of the buffer read (the new one in half 1)
      const double fk = k == 0 ? sl.fx : (k == 1 ? sl.fy : sl.fz);
      a.s.uref[k] = sl.comoving ? sl.uref[k] + (half == 1 ? fk / sl.rho0 : 0.0) : 0.0;
    }
    a.FA = sl.FA;
    a.FB = sl.FB;
    a.mask = sl.mask;
    a.K = K;
    a.mcache = sl.mcache;
    a.mbase = sl.mbase;
    a.cache_use = half == 0 ? sl.mvalid : 0;
    a.cache_fill = half == 1 ? 1 : 0;
    a.fa_rd = 0;
    const double hh = 0.5;
    double r[3], v[3];
    for (int k = 0; k < 3; ++k) {
      r[k] = sl.pos[3 * p + k];
      v[k] = sl.vel[3 * p + k];
    }
    if (half == 0) {
      for (int k = 0; k < 3; ++k) r[k] += hh * v[k];
      wrap3(sl.g, r);
    }
    const uint64_t mpre = mask_preload<K>(a, r, lane);
    const double m = sl.mass[p];
    double rp, up[3];
    group_interp<S, K>(a, r, half == 0, lane, rp, up, p);
    const double al = sl.gamma * hh / m, be = sl.gamma * hh / rp;
    double Fh[3];
    if (sl.coupling == LB_COUPLE_FC) {
      const double den = 1.0 + 0.5 * al + 0.5 * be;
      const double fe[3] = {sl.fx, sl.fy, sl.fz};
      for (int k = 0; k < 3; ++k) {
        Fh[k] = -(sl.gamma * (v[k] - up[k]) - 0.5 * be * fe[k]) / den;
        v[k] += hh / m * Fh[k];
      }
    } else {
      const double sm = al + be;
      for (int k = 0; k < 3; ++k) {
        const double d = v[k] - up[k];
        Fh[k] = -sl.gamma / sm * d;
        v[k] = v[k] - al / sm * d;
      }
    }
    const double Ff[3] = {-Fh[0], -Fh[1], -Fh[2]};
    if (sl.det_on) {  // stored; k_ens_spread_det spreads it (and drifts after half 1)
      if (lane == 0)
        for (int k = 0; k < 3; ++k) sl.aux[3 * p + k] = Ff[k];
    } else {
      group_spread<E, K>(a, r, Ff, half == 0 ? sl.FA : sl.FB, lane, &mpre);
    }
    if (lane == 0) {
      if (half == 1 && !sl.det_on) {
        for (int k = 0; k < 3; ++k) r[k] += hh * v[k];
        wrap3(sl.g, r);
      }
      for (int k = 0; k < 3; ++k) {
        sl.pos[3 * p + k] = r[k];
        sl.vel[3 * p + k] = v[k];
      }
    }
  }
}

// Deterministic spreading of the stored lattice forces of one coupling half
// of every deterministic slot (fixed-point accumulation, see k_spread_det),
// then the final P^1/2 after half 1.
template <int K>
__global__ __launch_bounds__(256) void k_ens_spread_det(EnsArgs e, int half) {
  constexpr int L = Lanes<K>::L;
  const int n = *e.npitems;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 w = e.pitems[it];
    const EnsSlot& sl = e.slots[w.x];
    if (!ens_active(sl) || sl.coupling == LB_COUPLE_NONE || !sl.det_on) continue;
    const long long p = (long long)w.y + threadIdx.x / L;
    const int lane = threadIdx.x % L;
    if (p >= sl.np) continue;  // whole lane groups leave together
    double r[3], f[3];
    for (int k = 0; k < 3; ++k) {
      r[k] = sl.pos[3 * p + k];
      f[k] = sl.aux[3 * p + k];
    }
    const SiteSlot ss = slot_of<K>(sl.g, r, lane);
    if (ss.valid) {
      const long long s = site_index(sl.g, ss.x, ss.y, ss.z);
      for (int k = 0; k < 3; ++k) {
        uint64_t lo, hi;
        to_fixed(ss.W * f[k], lo, hi);
        if (lo | hi) fixed_add(sl.det + 6 * s + 2 * k, lo, hi);
      }
      uint64_t bit;
      flag_site(mask_word(sl.mask, sl.g, ss.x, ss.y, ss.z, bit), bit);
    }
    if (lane == 0 && half == 1) {
      for (int k = 0; k < 3; ++k) r[k] += 0.5 * sl.vel[3 * p + k];
      wrap3(sl.g, r);
      for (int k = 0; k < 3; ++k) sl.pos[3 * p + k] = r[k];
    }
  }
}

// The finalize of the deterministic spread for every deterministic slot, over
// the lattice work list (one lane per site).
template <int S>
__global__ __launch_bounds__(256) void k_ens_det_finalize(EnsArgs e, int half) {
  using E = typename Store<S>::R;
  const int n = *e.nlitems;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 w = e.litems[it];
    const EnsSlot& sl = e.slots[w.x];
    if (!ens_active(sl) || sl.coupling == LB_COUPLE_NONE || !sl.det_on || sl.np == 0) continue;
    const long long s = (long long)w.y * 256 + threadIdx.x;
    if (s < sl.g.N) det_finalize_site<E>(sl.g, sl.mask, sl.det, (E*)(half ? sl.FB : sl.FA), s);
  }
}

__global__ void k_ens_advance(EnsArgs e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= e.nslots) return;
  EnsSlot& sl = e.slots[i];
  if (!ens_active(sl)) return;
  sl.cur = 1 - sl.cur;
  sl.pend = 1;
  sl.steps_done += 1;
  if (sl.coupling != LB_COUPLE_NONE && sl.np > 0) sl.mvalid = 1;  // filled by the second half
  if (sl.comoving) {
    sl.uref[0] += sl.fx / sl.rho0;
    sl.uref[1] += sl.fy / sl.rho0;
    sl.uref[2] += sl.fz / sl.rho0;
    const double uo[3] = {sl.uref[0] + sl.fx / sl.rho0, sl.uref[1] + sl.fy / sl.rho0,
                          sl.uref[2] + sl.fz / sl.rho0};
    comoving_terms(sl.scale, sl.rho0, sl.uref, uo, sl.cm, sl.cmf);
  }
}

hipError_t launch_ens_step(int storage, int K, const EnsArgs& e, int lat_grid, int part_grid,
                           int det, hipStream_t st) {
  for (int half = 0; half < 2; ++half) {
    if (half == 1)
      LBC_STORAGE_SWITCH(storage, (k_ens_lattice<SS><<<lat_grid, 256, 0, st>>>(e.slots, e.litems,
                                                                              e.nlitems)));
    LBC_KERNEL_SWITCH(K, LBC_STORAGE_SWITCH(storage, (k_ens_couple<SS, KK><<<part_grid, 256, 0, st>>>(e, half))));
    if (det) {
      LBC_KERNEL_SWITCH(K, (k_ens_spread_det<KK><<<part_grid, 256, 0, st>>>(e, half)));
      LBC_STORAGE_SWITCH(storage, (k_ens_det_finalize<SS><<<lat_grid, 256, 0, st>>>(e, half)));
    }
  }
  k_ens_advance<<<(e.nslots + 63) / 64, 64, 0, st>>>(e);
  return hipGetLastError();
}

}  // namespace lbc
