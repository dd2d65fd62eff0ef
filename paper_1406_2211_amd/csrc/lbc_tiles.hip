// lbc_tiles.hip -- interpolation and spreading for dense Lagrangian markers
// (immersed-boundary shells).
//
//   interpolation (Eq. IBM-interpolation): from the velocity of the sites the
//   last spread flagged, computed once per step (see "interpolation, flagged
//   sites" below); no binning needed.
//   spreading (Eq. IBM-spreading): markers are binned into 8x8x8 lattice
//   tiles by the cell containing them (counting sort: count, single-block
//   scan that also lists the occupied tiles in increasing order, scatter).
//   Workgroups loop over the occupied tiles; each sums its markers' stencil
//   contributions over a region of 11^3 sites (the tile, one site below it
//   and two above) in LDS and adds the region to the field once.  The region
//   is the union of the 2-, 3- and 4-point stencils of the tile's cells (the
//   4-point stencil reaches one node below a marker's cell and two above
//   it); a node outside it (the marker has crossed a cell face out of the
//   tile since the binning, or a periodic seam) is added to the field
//   directly.  On the shell channel (128x128x256, 41 088 markers, binning
//   every 8 steps) that is about 20 of 2.6 million nodes per step.
#include <algorithm>

#include "lbc_device.h"
#include "lbc_internal.h"

namespace lbc {

constexpr int kTile = 8;
constexpr int kLo = 1;     // region starts one site below the tile
constexpr int kReg = 11;   // region edge: tile + 1 below + 2 above
constexpr int kRegSites = kReg * kReg * kReg;

__device__ __forceinline__ int tile_of(const TileArgs& t, const double X[3], int c[3]) {
  const int n[3] = {t.g.nx, t.g.ny, t.g.nz};
  for (int a = 0; a < 3; ++a) {
    int j = safe_floor(X[a]);
    if (j < 0) j = 0;
    if (j >= n[a]) j = n[a] - 1;
    c[a] = j / kTile;
  }
  return (c[2] * t.ty + c[1]) * t.tx + c[0];
}

// ------------------------------------------------------------------ binning
__global__ void k_bin_clear(TileArgs t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < t.ntiles) t.count[i] = 0;
  if (i == 0) t.nocc[0] = 0;
}

__global__ void k_bin_count(TileArgs t, const double* pos, long long n) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double X[3] = {pos[3 * p], pos[3 * p + 1], pos[3 * p + 2]};
  int c[3];
  const int tl = tile_of(t, X, c);
  t.ptile[p] = tl;
  atomicAdd(t.count + tl, 1);
}

// Single workgroup: exclusive scan of the tile counts (start, cursor) and the
// list of occupied tiles in increasing tile order.  Each lane owns a run of
// consecutive tiles; the run totals are scanned across the wavefront with
// shuffles and across wavefronts through LDS.
__global__ __launch_bounds__(1024) void k_bin_scan(TileArgs t) {
  __shared__ int wsum[16][2];
  const int per = (t.ntiles + 1023) / 1024;
  const int b = threadIdx.x * per;
  const int e = min(b + per, t.ntiles);
  int cs = 0, os = 0;
  for (int i = b; i < e; ++i) {
    const int c = t.count[i];
    cs += c;
    os += c > 0 ? 1 : 0;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int ic = cs, io = os;  // inclusive scans over the wavefront
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int pc = __shfl_up(ic, o, 64), po = __shfl_up(io, o, 64);
    if (lane >= o) {
      ic += pc;
      io += po;
    }
  }
  if (lane == 63) {
    wsum[wv][0] = ic;
    wsum[wv][1] = io;
  }
  __syncthreads();
  int pc = 0, po = 0;
  for (int w = 0; w < wv; ++w) {
    pc += wsum[w][0];
    po += wsum[w][1];
  }
  int start = pc + ic - cs, occ = po + io - os;
  for (int i = b; i < e; ++i) {
    const int c = t.count[i];
    t.start[i] = start;
    t.cursor[i] = start;
    start += c;
    if (c > 0) t.occ[occ++] = i;
  }
  if (threadIdx.x == 1023) {
    t.start[t.ntiles] = pc + ic;
    t.nocc[0] = po + io;
  }
}

__global__ void k_bin_scatter(TileArgs t, long long n) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int slot = atomicAdd(t.cursor + t.ptile[p], 1);
  t.sorted[slot] = (int)p;
}

// ------------------------------------------------------------- region maps
struct Region {
  int o[3];  // unwrapped integer coordinate of region slot 0
};

__device__ __forceinline__ Region region_of(const TileArgs& t, int tl) {
  Region r;
  const int cx = tl % t.tx, cy = (tl / t.tx) % t.ty, cz = tl / (t.tx * t.ty);
  r.o[0] = cx * kTile - kLo;
  r.o[1] = cy * kTile - kLo;
  r.o[2] = cz * kTile - kLo;
  return r;
}

// Site (wrapped) of region slot (ix, iy, iz); false beyond a wall.
__device__ __forceinline__ bool slot_site(const Geo& g, const Region& r, int ix, int iy, int iz,
                                          int& x, int& y, int& z) {
  x = wrap_idx(r.o[0] + ix, g.nx);
  z = wrap_idx(r.o[2] + iz, g.nz);
  y = r.o[1] + iy;
  if (g.wall) return y >= 0 && y < g.ny;
  y = wrap_idx(y, g.ny);
  return true;
}

// Wrapped site of a node; false beyond a wall.
__device__ __forceinline__ bool node_site(const Geo& g, const int j[3], int& x, int& y, int& z) {
  x = wrap_idx(j[0], g.nx);
  z = wrap_idx(j[2], g.nz);
  y = j[1];
  if (g.wall) return y >= 0 && y < g.ny;
  y = wrap_idx(y, g.ny);
  return true;
}

// Arithmetic type of interpolation and spreading weights and of the staged
// moments: FP64 with FP64 storage, FP32 otherwise (node offsets j - X are
// formed in FP64 from the FP64 positions and then rounded).
template <int S>
struct TileT {
  using W = double;
};
template <>
struct TileT<LB_F32> {
  using W = float;
};
template <>
struct TileT<LB_F16> {
  using W = float;
};
template <>
struct TileT<LB_BF16> {
  using W = float;
};

// ------------------------------------------------ interpolation, flagged sites
// The sites whose force-mask bit is set after the lattice pass are those where
// the pending immersed-boundary field is nonzero: the stencil sites of the
// last spread, at the predictor positions X~.  The markers interpolate at X~
// (the final advection of the previous step) and at points that have drifted
// by a fraction of a site from there, so nearly all of their stencil nodes
// are flagged.  k_flag_vel computes the physical velocity (pull gather plus
// pending half force, the redefined velocity of Sec. 4) of every flagged site
// once into a dense field U, each entry stamped with the number of the call;
// k_marker_interp interpolates each marker from U alone, and a marker that
// meets a node without the current stamp is listed and redone by
// k_marker_slow, which gathers such nodes from the populations (same
// arithmetic).  So the flags decide speed, not results.

// Stamp of a velocity entry, kept in its fourth component as raw bits.
__device__ __forceinline__ float stamp_value(float, uint32_t st) { return __uint_as_float(st); }
__device__ __forceinline__ double stamp_value(double, uint32_t st) {
  return __longlong_as_double((long long)st);
}
__device__ __forceinline__ bool stamped(float w, uint32_t st) { return __float_as_uint(w) == st; }
__device__ __forceinline__ bool stamped(double w, uint32_t st) {
  return __double_as_longlong(w) == (long long)st;
}

// j mod n for a stencil node: one compare-and-add for a node within a box
// length of the box, the division otherwise.
__device__ __forceinline__ int wrap_near(int j, int n) {
  const int r = j < 0 ? j + n : (j >= n ? j - n : j);
  return (unsigned)r < (unsigned)n ? r : wrap_idx(j, n);
}

// Mask words per wavefront of the velocity pass: on the c3 shells 8 words
// (about 20 flagged sites per wavefront) took 19.8 us against 21.1 for 16,
// and the step 0.198 ms against 0.200 (32 words: 0.212, 4 words: 0.199).
constexpr int kVelWords = 8;

template <int S>
__global__ __launch_bounds__(256) void k_flag_vel(SiteArgs s, const uint64_t* __restrict__ mask,
                                                  long long nwords, void* Uv, uint32_t stamp) {
  using W = typename TileT<S>::W;
  using V4 = typename Store<S>::V4;
  for_flagged_sites<kVelWords>(s.g, mask, nwords, [&](int x, int y, int z) {
    W drho, j[3];
    site_phys_r<S, W>(s, x, y, z, drho, j);
    const W rr = W(s.rho0) + drho;
    V4 u;
    u.x = j[0] / rr;
    u.y = j[1] / rr;
    u.z = j[2] / rr;
    u.w = stamp_value(W(0), stamp);
    ((V4*)Uv)[site_index(s.g, x, y, z)] = u;
  });
}

// One axis of a K-point stencil (Appendix A kernels) in closed form: the
// first node j0 and two parameters t, q from which each of the K weights
// follows in two operations (the K = 4 and K = 3 weights share one square
// root).  K = 4: t = X - floor(X), j0 = floor(X) - 1, q = sqrt(1 + 4t - 4t^2),
//   weights (3 - 2t - q, 3 - 2t + q, 1 + 2t + q, 1 + 2t - q) / 8;
// K = 3: t = X - round(X), j0 = round(X) - 1, q = sqrt(1 - 3t^2),
//   weights ((2 - 3t - q) / 6, (1 + q) / 3, (2 + 3t - q) / 6);
// K = 2: t = X - floor(X), j0 = floor(X), weights (1 - t, t).
// These are the piecewise definitions evaluated at the node distances
// -1 - t, -t, 1 - t, 2 - t (K = 4) and -1 - t, -t, 1 - t (K = 3, 2).  The
// position is clamped as in safe_floor, so any X gives an in-range node.
template <int K, typename W>
__device__ __forceinline__ void stencil_t(double X, int& j0, W& t, W& q) {
  const double f = floor(fmin(fmax(K == 3 ? X + 0.5 : X, -1073741824.0), 1073741824.0));
  j0 = (int)f - (K == 2 ? 0 : 1);
  t = (W)(X - f);
  q = K == 4 ? sqrt(W(1) + W(4) * t - W(4) * t * t) : (K == 3 ? sqrt(W(1) - W(3) * t * t) : W(0));
}
template <int K, typename W>
__device__ __forceinline__ W node_weight(int k, W t, W q) {
  if (K == 4) {
    const W a = k < 2 ? W(3) : W(1), b = k < 2 ? W(-2) : W(2), c = (k == 1 || k == 2) ? W(1) : W(-1);
    return (a + b * t + c * q) * W(0.125);
  }
  if (K == 3) {
    if (k == 1) return (W(1) + q) * (W(1) / W(3));
    return (W(2) + (k == 0 ? W(-3) : W(3)) * t - q) * (W(1) / W(6));
  }
  return k == 0 ? W(1) - t : t;
}

// Lanes per marker: one per (x, y) column of stencil nodes, K rounded up to a
// power of two in x and y, so that in each z plane the lanes of a marker read
// whole x rows of the velocity field.
template <int K>
struct ColGroup {
  static constexpr int KP = K == 2 ? 2 : 4;
  static constexpr int G = KP * KP;
};

// Interpolated velocity of one stencil (Eq. IBM-interpolation),
// u_p = sum W u(node), W = phi(x) phi(y) phi(z): lane r takes the node column
// (r % KP, r / KP) over the K z planes, and the marker's lanes sum.  FAST:
// nodes are read from U only, and the return value (the same on every lane of
// the group) tells whether each node carried the stamp; otherwise a node
// without it is gathered from the populations and the return value is true.
template <int S, int K, bool FAST>
__device__ __forceinline__ bool marker_interp_at(const SiteArgs& s, const void* Uv,
                                                 uint32_t stamp, const double X[3], int r,
                                                 double up[3]) {
  using W = typename TileT<S>::W;
  using V4 = typename Store<S>::V4;
  constexpr int KP = ColGroup<K>::KP, G = ColGroup<K>::G;
  int j0[3];
  W t[3], q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) stencil_t<K, W>(X[a], j0[a], t[a], q[a]);
  const int kx = r % KP, ky = r / KP;
  const int jx = j0[0] + kx, jy = j0[1] + ky;
  W ux = 0, uy = 0, uz = 0;
  bool all = true;
  if (kx < K && ky < K && !(s.g.wall && (jy < 0 || jy >= s.g.ny))) {
    const W wxy = node_weight<K, W>(kx, t[0], q[0]) * node_weight<K, W>(ky, t[1], q[1]);
    const uint32_t nx = (uint32_t)s.g.nx, ny = (uint32_t)s.g.ny;
    const uint32_t x = (uint32_t)wrap_near(jx, s.g.nx);
    const uint32_t y = (uint32_t)(s.g.wall ? jy : wrap_near(jy, s.g.ny));
#pragma unroll
    for (int kz = 0; kz < K; ++kz) {
      const uint32_t z = (uint32_t)wrap_near(j0[2] + kz, s.g.nz);
      const W Wt = wxy * node_weight<K, W>(kz, t[2], q[2]);
      V4 u = ((const V4*)Uv)[(z * ny + y) * nx + x];  // fewer than 2^32 sites
      const bool ok = stamped(u.w, stamp);
      if (!FAST && !ok) {  // a node that was not flagged: gather it
        W drho, j[3];
        site_phys_r<S, W>(s, (int)x, (int)y, (int)z, drho, j);
        const W rr = W(s.rho0) + drho;
        u.x = j[0] / rr;
        u.y = j[1] / rr;
        u.z = j[2] / rr;
      }
      all = all && ok;
      ux += Wt * u.x;
      uy += Wt * u.y;
      uz += Wt * u.z;
    }
  }
  up[0] = (double)group_sum_dpp<G, W>(ux);
  up[1] = (double)group_sum_dpp<G, W>(uy);
  up[2] = (double)group_sum_dpp<G, W>(uz);
  if (!FAST) return true;
  const int lane = (int)threadIdx.x & 63;
  const uint64_t miss = __ballot(!all);
  const uint64_t gm = ((1ull << G) - 1ull) << (lane / G * G);
  return (miss & gm) == 0ull;
}

// One marker's interpolations and half drifts.
// mode 0: IB predictor       aux = wrap(pos + h/2 u(pos))
// mode 1: IB advection       pos = wrap(pos + h/2 u(aux))
// mode 2: both, in that order (at = pos); the first advection only needs the
//         state before the lattice pass, like the predictor.
// mode 3: mode 1 of one step followed by mode 2 of the next (at = aux): the
//         final advection of a step and the predictor and first advection of
//         the next read the same fluid state.
// FAST stops, with nothing written, at the first stencil with a node outside
// the velocity field's current stamp and returns false.
template <int S, int K, bool FAST>
__device__ __forceinline__ bool marker_run(const SiteArgs& s, const void* Uv, uint32_t stamp,
                                           const double* at, double* pos, double* aux, int mode,
                                           long long p, int r) {
  const double X[3] = {at[3 * p], at[3 * p + 1], at[3 * p + 2]};
  double P[3] = {0.0, 0.0, 0.0};
  if (mode == 1 || mode == 3)
    for (int a = 0; a < 3; ++a) P[a] = pos[3 * p + a];
  auto half_drift = [&](const double from[3], const double u[3], double to[3]) {
    for (int a = 0; a < 3; ++a) to[a] = from[a] + 0.5 * u[a];
    to[0] = wrap_pos(to[0], (double)s.g.nx);
    if (!s.g.wall) to[1] = wrap_pos(to[1], (double)s.g.ny);
    to[2] = wrap_pos(to[2], (double)s.g.nz);
  };
  // Interpolation points in order: mode 0, 1: X; mode 2: X, then
  // X~ = X + h/2 u(X); mode 3: X (= X~ of the previous step), then
  // Xs = P + h/2 u(X), then X~ = Xs + h/2 u(Xs).
  const int nint = mode == 3 ? 3 : (mode == 2 ? 2 : 1);
  double q[3] = {X[0], X[1], X[2]}, Xs[3] = {X[0], X[1], X[2]}, u[3], Y[3];
#pragma unroll 1
  for (int it = 0; it < nint; ++it) {
    if (!marker_interp_at<S, K, FAST>(s, Uv, stamp, q, r, u)) return false;
    if (it + 1 == nint) break;
    if (mode == 3 && it == 0) {
      half_drift(P, u, Xs);
      for (int a = 0; a < 3; ++a) q[a] = Xs[a];
    } else {
      half_drift(Xs, u, q);
    }
  }
  if (mode == 0) {
    half_drift(X, u, Y);
    if (r == 0)
      for (int a = 0; a < 3; ++a) aux[3 * p + a] = Y[a];
  } else if (mode == 1) {
    half_drift(P, u, Y);
    if (r == 0)
      for (int a = 0; a < 3; ++a) pos[3 * p + a] = Y[a];
  } else {
    half_drift(Xs, u, Y);
    if (r == 0)
      for (int a = 0; a < 3; ++a) {
        aux[3 * p + a] = q[a];
        pos[3 * p + a] = Y[a];
      }
  }
  return true;
}

// One marker per group of G lanes, from the velocity field only.  A marker
// that meets a node without the current stamp is listed: miss[stamp & 1]
// counts, the list follows the two counters.  Six wavefronts per SIMD for
// the 32-bit weights (80 registers, no spills); FP64 keeps its register
// count.
template <int S, int K>
__global__ __launch_bounds__(256, S == LB_F64 ? 1 : 6) void k_marker_interp(
    SiteArgs s, const void* Uv, uint32_t stamp, const double* at, double* pos, double* aux,
    int mode, long long n, int* miss) {
  constexpr int G = ColGroup<K>::G;
  const long long p = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int r = (int)threadIdx.x % G;
  if (p >= n) return;  // whole groups leave together
  if (marker_run<S, K, true>(s, Uv, stamp, at, pos, aux, mode, p, r)) return;
  if (r == 0) miss[2 + atomicAdd(miss + (stamp & 1u), 1)] = (int)p;
}

// The listed markers, with the nodes that lack the stamp gathered from the
// populations (a grid-stride loop over the list); also clears the counter
// that the next call uses.
template <int S, int K>
__global__ __launch_bounds__(256) void k_marker_slow(SiteArgs s, const void* Uv, uint32_t stamp,
                                                     const double* at, double* pos, double* aux,
                                                     int mode, int* miss) {
  constexpr int G = ColGroup<K>::G;
  const int cnt = miss[stamp & 1u];
  const long long lanes = (long long)gridDim.x * blockDim.x;
  for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g / G < cnt; g += lanes)
    marker_run<S, K, false>(s, Uv, stamp, at, pos, aux, mode, miss[2 + g / G], (int)(g % G));
  if (blockIdx.x == 0 && threadIdx.x == 0) miss[(stamp + 1u) & 1u] = 0;
}

// ------------------------------------------------------------------ spreading
// One workgroup per occupied tile (Eq. IBM-spreading, F(x) = sum_p W(x - X_p)
// F_p, the adjoint of the interpolation, with the same closed-form weights):
// the tile's markers are staged in LDS, their stencil contributions are
// summed in a dense FP64 LDS accumulator over the tile's region, and every
// nonzero region site is then added to the global field once, with an
// atomic (the regions of neighbouring tiles overlap).  The accumulator is
// FP64 whatever the field precision: LDS atomic adds measured about three
// times faster in FP64 than in FP32 on this device (c3 spreading 31 against
// 100 us).  The flags for the lattice pass are collected per region row in
// LDS and set with one cached load and at most one atomic per mask word of
// the row, instead of a dependent load per site.
constexpr int kSpreadChunk = 128;  // markers staged per round
constexpr int kRegRows = kReg * kReg;

template <typename E, int K>
__global__ __launch_bounds__(256) void k_tile_spread(TileArgs t, const double* at, const double* F,
                                                     void* field) {
  constexpr int KP = ColGroup<K>::KP, G = ColGroup<K>::G;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* acc = (double*)lds_raw;                 // [3][kRegSites]
  double* mx = acc + 3 * kRegSites;               // [chunk][6]: position, force
  uint32_t* rowbits = (uint32_t*)(mx + 6 * kSpreadChunk);  // [kRegRows]: nonzero x slots
  static_assert(kReg <= 32, "a region row's slots fit one 32-bit mask");
  E* Fd = (E*)field;
  const int nocc = t.nocc[0];
  auto global_add = [&](int jx, int jy, int jz, E f0, E f1, E f2) {
    const int j[3] = {jx, jy, jz};
    int x, y, z;
    if (!node_site(t.g, j, x, y, z)) return;  // beyond a wall
    const long long sidx = site_index(t.g, x, y, z);
    unsafeAtomicAdd(Fd + 4 * sidx + 0, f0);
    unsafeAtomicAdd(Fd + 4 * sidx + 1, f1);
    unsafeAtomicAdd(Fd + 4 * sidx + 2, f2);
    uint64_t bit;
    flag_site(mask_word(t.mask, t.g, x, y, z, bit), bit);
  };
  for (int ot = blockIdx.x; ot < nocc; ot += gridDim.x) {
    const int tl = t.occ[ot];
    const Region r = region_of(t, tl);
    const int b0 = t.start[tl], b1 = t.start[tl + 1];
    for (int k = threadIdx.x; k < 3 * kRegSites; k += blockDim.x) acc[k] = 0.0;
    for (int k = threadIdx.x; k < kRegRows; k += blockDim.x) rowbits[k] = 0u;
    for (int c0 = b0; c0 < b1; c0 += kSpreadChunk) {
      const int nc = min(kSpreadChunk, b1 - c0);
      __syncthreads();  // accumulator cleared, or the previous chunk done with mx
      for (int i = threadIdx.x; i < nc; i += blockDim.x) {
        const long long p = t.sorted[c0 + i];
        for (int a = 0; a < 3; ++a) {
          mx[6 * i + a] = at[3 * p + a];
          mx[6 * i + 3 + a] = F[3 * p + a];
        }
      }
      __syncthreads();
      // one lane per (x, y) column of a marker's stencil, over its z nodes
      for (int i = (int)threadIdx.x / G; i < nc; i += (int)blockDim.x / G) {
        const int rr = (int)threadIdx.x % G, kx = rr % KP, ky = rr / KP;
        if (kx >= K || ky >= K) continue;
        const double* m = mx + 6 * i;
        int j0[3];
        E tt[3], qq[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) stencil_t<K, E>(m[a], j0[a], tt[a], qq[a]);
        const int jx = j0[0] + kx, jy = j0[1] + ky;
        if (t.g.wall && (jy < 0 || jy >= t.g.ny)) continue;  // beyond a wall: no node
        const E wxy = node_weight<K, E>(kx, tt[0], qq[0]) * node_weight<K, E>(ky, tt[1], qq[1]);
        const int ix = jx - r.o[0], iy = jy - r.o[1];
        const bool in_xy = ix >= 0 && ix < kReg && iy >= 0 && iy < kReg;
#pragma unroll
        for (int kz = 0; kz < K; ++kz) {
          const double W = (double)(wxy * node_weight<K, E>(kz, tt[2], qq[2]));
          const double f0 = W * m[3], f1 = W * m[4], f2 = W * m[5];
          const int jz = j0[2] + kz, iz = jz - r.o[2];
          if (in_xy && iz >= 0 && iz < kReg) {
            double* a = acc + (iz * kReg + iy) * kReg + ix;
            atomicAdd(a, f0);
            atomicAdd(a + kRegSites, f1);
            atomicAdd(a + 2 * kRegSites, f2);
          } else {
            global_add(jx, jy, jz, (E)f0, (E)f1, (E)f2);
          }
        }
      }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kRegSites; k += blockDim.x) {
      const E a0 = (E)acc[k], a1 = (E)acc[kRegSites + k], a2 = (E)acc[2 * kRegSites + k];
      if (a0 == E(0) && a1 == E(0) && a2 == E(0)) continue;
      int x, y, z;
      if (!slot_site(t.g, r, k % kReg, (k / kReg) % kReg, k / (kReg * kReg), x, y, z)) continue;
      const long long sidx = site_index(t.g, x, y, z);
      unsafeAtomicAdd(Fd + 4 * sidx + 0, a0);
      unsafeAtomicAdd(Fd + 4 * sidx + 1, a1);
      unsafeAtomicAdd(Fd + 4 * sidx + 2, a2);
      atomicOr(rowbits + k / kReg, 1u << (k % kReg));
    }
    __syncthreads();
    // flags: per region row, runs of slots in the same mask word
    for (int row = threadIdx.x; row < kRegRows; row += blockDim.x) {
      uint32_t bits = rowbits[row];
      uint64_t* cur = nullptr;
      uint64_t acc_bits = 0;
      while (bits) {
        const int ix = __ffs(bits) - 1;
        bits &= bits - 1u;
        int x, y, z;
        slot_site(t.g, r, ix, row % kReg, row / kReg, x, y, z);  // (a wall row has no bits)
        uint64_t bit;
        uint64_t* mw = mask_word(t.mask, t.g, x, y, z, bit);
        if (mw != cur) {
          if (cur && (*cur & acc_bits) != acc_bits) atomicOr((unsigned long long*)cur, acc_bits);
          cur = mw;
          acc_bits = 0;
        }
        acc_bits |= bit;
      }
      if (cur && (*cur & acc_bits) != acc_bits) atomicOr((unsigned long long*)cur, acc_bits);
    }
    __syncthreads();  // the accumulator and the row masks are cleared for the next tile
  }
}

// ------------------------------------------------------------------ shells
// Rigid-shell tethers: block per shell.  Markers are unwrapped around the
// first marker, centred, the least-squares rotation of the template onto
// them is found from the dominant eigenvector of Horn's symmetric 4x4
// quaternion matrix (cyclic Jacobi), and F_j = -k (y_j - c - R t_j).
// Every index below is a compile-time constant after unrolling, so A and V
// stay in registers (indexed at run time they went to scratch memory).
__device__ __forceinline__ void sym4_eig_max(double A[4][4], double q[4]) {
  double V[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int it = 0; it < 50; ++it) {
    double off = 0, dia = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) (i == j ? dia : off) += A[i][j] * A[i][j];
    if (off == 0.0 || off < 1e-32 * dia) break;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int r = p + 1; r < 4; ++r) {
        const double apr = A[p][r];
        if (apr == 0.0) continue;
        const double theta = 0.5 * (A[r][r] - A[p][p]) / apr;
        const double t = copysign(1.0, theta) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = rsqrt(t * t + 1.0), s = t * c;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double x = A[k][p], y = A[k][r];
          A[k][p] = c * x - s * y;
          A[k][r] = s * x + c * y;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double x = A[p][k], y = A[r][k];
          A[p][k] = c * x - s * y;
          A[r][k] = s * x + c * y;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double x = V[k][p], y = V[k][r];
          V[k][p] = c * x - s * y;
          V[k][r] = s * x + c * y;
        }
      }
  }
  double bv = A[0][0];
#pragma unroll
  for (int k = 0; k < 4; ++k) q[k] = V[k][0];
#pragma unroll
  for (int j = 1; j < 4; ++j)
    if (A[j][j] > bv) {
      bv = A[j][j];
#pragma unroll
      for (int k = 0; k < 4; ++k) q[k] = V[k][j];
    }
}

// Dominant eigenvector of Horn's traceless symmetric 4x4 matrix A without an
// iterative eigen-solve: the largest root of the characteristic polynomial
// p(l) = l^4 - (tr A^2 / 2) l^2 - (tr A^3 / 3) l + det A by Newton's method
// from the upper bound ||A||_F (p is convex above its largest root, so the
// iterates decrease monotonically onto it; the same idea as Theobald's
// quaternion characteristic polynomial method), then the column of
// adj(A - l I) with the largest diagonal entry, which is proportional to the
// eigenvector of a simple root.  Returns false when the eigen-residual is not
// at rounding level (a near-degenerate top eigenvalue); the caller then uses
// the Jacobi solve.  Every index is a compile-time constant after unrolling.
__device__ __forceinline__ int skip_idx(int i, int k) { return k < i ? k : k + 1; }

__device__ __forceinline__ bool quat_top(const double A[4][4], double q[4]) {
  double fro2 = 0, tr3 = 0;
  double B[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      fro2 += A[i][j] * A[i][j];
      double b = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) b += A[i][k] * A[k][j];
      B[i][j] = b;
    }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) tr3 += B[i][j] * A[j][i];
  if (!(fro2 > 0.0)) {  // A = 0: any rotation fits; the identity, as the Jacobi solve gives
    q[0] = 1.0;
    q[1] = q[2] = q[3] = 0.0;
    return true;
  }
  // det A by cofactors along row 0
  double det = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c0 = skip_idx(j, 0), c1 = skip_idx(j, 1), c2 = skip_idx(j, 2);
    const double m = A[1][c0] * (A[2][c1] * A[3][c2] - A[2][c2] * A[3][c1]) -
                     A[1][c1] * (A[2][c0] * A[3][c2] - A[2][c2] * A[3][c0]) +
                     A[1][c2] * (A[2][c0] * A[3][c1] - A[2][c1] * A[3][c0]);
    det += ((j & 1) ? -1.0 : 1.0) * A[0][j] * m;
  }
  const double a2 = 0.5 * fro2, a1 = tr3 / 3.0;
  double l = sqrt(fro2);
  for (int it = 0; it < 60; ++it) {
    const double l2 = l * l;
    const double p = (l2 - a2) * l2 - a1 * l + det;
    const double dp = (4.0 * l2 - 2.0 * a2) * l - a1;
    if (!(dp > 0.0)) break;
    const double dl = p / dp;
    l -= dl;
    if (fabs(dl) <= 1e-15 * fabs(l)) break;
  }
  // adjugate of M = A - l I: adj[i][j] = (-1)^(i+j) det(M without row j, column i)
  double M[4][4], best = -1.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) M[i][j] = A[i][j] - (i == j ? l : 0.0);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double col[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r0 = skip_idx(c, 0), r1 = skip_idx(c, 1), r2 = skip_idx(c, 2);
      const int k0 = skip_idx(i, 0), k1 = skip_idx(i, 1), k2 = skip_idx(i, 2);
      const double m = M[r0][k0] * (M[r1][k1] * M[r2][k2] - M[r1][k2] * M[r2][k1]) -
                       M[r0][k1] * (M[r1][k0] * M[r2][k2] - M[r1][k2] * M[r2][k0]) +
                       M[r0][k2] * (M[r1][k0] * M[r2][k1] - M[r1][k1] * M[r2][k0]);
      col[i] = (((i + c) & 1) ? -1.0 : 1.0) * m;
    }
    if (fabs(col[c]) > best) {
      best = fabs(col[c]);
#pragma unroll
      for (int i = 0; i < 4; ++i) q[i] = col[i];
    }
  }
  const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!(nq > 0.0)) return false;
#pragma unroll
  for (int i = 0; i < 4; ++i) q[i] /= nq;
  double res = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double r = -l * q[i];
#pragma unroll
    for (int j = 0; j < 4; ++j) r += A[i][j] * q[j];
    res = fmax(res, fabs(r));
  }
  return res <= 1e-12 * sqrt(fro2);
}

// Sum of N values over the workgroup, every lane getting the sums: DPP wave
// sums, one LDS slot per wavefront, then each lane adds the slots.
template <int N>
__device__ __forceinline__ void block_sum_n(double v[N], double* lds /*[N * 16]*/) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_sum_dpp(v[k]);
  if (lane == 0)
    for (int k = 0; k < N; ++k) lds[N * wv + k] = v[k];
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    double t = 0;
    for (int w = 0; w < nw; ++w) t += lds[N * w + k];
    v[k] = t;
  }
  __syncthreads();  // lds is reused by the next sum
}

// A shell of up to kShellPerLane * 256 markers keeps each lane's unwrapped
// positions and template vectors in registers across the three passes
// (centre, cross-covariance, forces), so every marker is loaded once.
constexpr int kShellPerLane = 4;

// The tether forces of one shell, computed by the whole workgroup; red
// [16 * 9] and sh_R [9] are LDS.
__device__ __forceinline__ void shell_block(const ShellArgs& sa, int shell, double* red,
                                            double* sh_R) {
  const int M = sa.M;
  const long long base = (long long)shell * M;
  const double* X = sa.pos + 3 * base;
  const double X0[3] = {X[0], X[1], X[2]};
  const double L[3] = {(double)sa.g.nx, (double)sa.g.ny, (double)sa.g.nz};
  const double rL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
  // minimum image around the first marker (a shell spans less than half a box)
  auto unwrap = [&](int j, double y[3]) {
    for (int k = 0; k < 3; ++k) {
      y[k] = X[3 * j + k] - X0[k];
      if (k != 1 || !sa.g.wall) y[k] -= L[k] * floor(y[k] * rL[k] + 0.5);
      y[k] += X0[k];
    }
  };
  const bool held = M <= kShellPerLane * (int)blockDim.x;
  double yh[kShellPerLane][3], th[kShellPerLane][3];
  if (held) {
#pragma unroll
    for (int q = 0; q < kShellPerLane; ++q) {
      const int j = (int)threadIdx.x + q * (int)blockDim.x;
      if (j < M) {
        unwrap(j, yh[q]);
        for (int a = 0; a < 3; ++a) th[q][a] = sa.tmpl[3 * j + a];
      }
    }
  }
  // each lane's markers: from registers, or loaded again for a larger shell
  auto for_markers = [&](auto&& fn) {
    if (held) {
#pragma unroll
      for (int q = 0; q < kShellPerLane; ++q) {
        const int j = (int)threadIdx.x + q * (int)blockDim.x;
        if (j < M) fn(j, yh[q], th[q]);
      }
    } else {
      for (int j = threadIdx.x; j < M; j += blockDim.x) {
        double y[3], t[3];
        unwrap(j, y);
        for (int a = 0; a < 3; ++a) t[a] = sa.tmpl[3 * j + a];
        fn(j, y, t);
      }
    }
  };
  double c[3] = {0, 0, 0};
  for_markers([&](int, const double* y, const double*) {
    for (int k = 0; k < 3; ++k) c[k] += y[k];
  });
  block_sum_n<3>(c, red);
  for (int k = 0; k < 3; ++k) c[k] /= M;
  double S[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for_markers([&](int, const double* y, const double* t) {
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) S[3 * a + b] += t[a] * (y[b] - c[b]);
  });
  block_sum_n<9>(S, red);
  if (threadIdx.x == 0) {
    const double Sxx = S[0], Sxy = S[1], Sxz = S[2], Syx = S[3], Syy = S[4], Syz = S[5],
                 Szx = S[6], Szy = S[7], Szz = S[8];
    double A[4][4] = {{Sxx + Syy + Szz, Syz - Szy, Szx - Sxz, Sxy - Syx},
                      {Syz - Szy, Sxx - Syy - Szz, Sxy + Syx, Szx + Sxz},
                      {Szx - Sxz, Sxy + Syx, -Sxx + Syy - Szz, Syz + Szy},
                      {Sxy - Syx, Szx + Sxz, Syz + Szy, -Sxx - Syy + Szz}};
    double q[4];
    if (!quat_top(A, q)) sym4_eig_max(A, q);
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    sh_R[0] = w * w + x * x - y * y - z * z;
    sh_R[1] = 2 * (x * y - w * z);
    sh_R[2] = 2 * (x * z + w * y);
    sh_R[3] = 2 * (x * y + w * z);
    sh_R[4] = w * w - x * x + y * y - z * z;
    sh_R[5] = 2 * (y * z - w * x);
    sh_R[6] = 2 * (x * z - w * y);
    sh_R[7] = 2 * (y * z + w * x);
    sh_R[8] = w * w - x * x - y * y + z * z;
    if (sa.rot)
      for (int k = 0; k < 9; ++k) sa.rot[9 * shell + k] = sh_R[k];
  }
  __syncthreads();
  for_markers([&](int j, const double* y, const double* t) {
    for (int a = 0; a < 3; ++a) {
      const double tgt = sh_R[3 * a] * t[0] + sh_R[3 * a + 1] * t[1] + sh_R[3 * a + 2] * t[2];
      sa.fint[3 * (base + j) + a] = -sa.k * (y[a] - c[a] - tgt);
    }
  });
}

__global__ __launch_bounds__(256) void k_shell_forces(ShellArgs sa) {
  __shared__ double red[16 * 9];
  __shared__ double sh_R[9];
  shell_block(sa, blockIdx.x, red, sh_R);
}

// The listed markers redone, then the tether forces, in one launch for a
// marker set made of whole shells: each shell's workgroup takes the markers
// of its shell from the list that the interpolation left (a stencil node
// without the current stamp), redoes them with gathers exactly as
// k_marker_slow does, and computes the shell's forces from the positions of
// all its markers (the fast interpolation wrote the others before this
// launch).  Takes the place of k_marker_slow followed by k_shell_forces.
template <int S, int K>
__global__ __launch_bounds__(256) void k_shell_redo_forces(ShellArgs sa, SiteArgs s,
                                                           const void* Uv, uint32_t stamp,
                                                           const double* at, double* pos,
                                                           double* aux, int mode, int* miss) {
  constexpr int G = ColGroup<K>::G;
  constexpr int kScan = 1024;  // list entries scanned per round (so at most as many are the shell's)
  __shared__ int mine[kScan];
  __shared__ int nmine;
  __shared__ double red[16 * 9];
  __shared__ double sh_R[9];
  const int shell = (int)blockIdx.x;
  const int cnt = miss[stamp & 1u];
  const long long lo = (long long)shell * sa.M, hi = lo + sa.M;
  for (int b0 = 0; b0 < cnt; b0 += kScan) {
    if (threadIdx.x == 0) nmine = 0;
    __syncthreads();
    const int b1 = min(cnt, b0 + kScan);
    for (int j = b0 + (int)threadIdx.x; j < b1; j += (int)blockDim.x) {
      const int p = miss[2 + j];
      if (p >= lo && p < hi) mine[atomicAdd(&nmine, 1)] = p;
    }
    __syncthreads();
    const int nm = nmine;
    for (int g = (int)threadIdx.x; g / G < nm; g += (int)blockDim.x)  // whole groups leave together
      marker_run<S, K, false>(s, Uv, stamp, at, pos, aux, mode, mine[g / G], g % G);
    __syncthreads();  // the redone positions are visible to the workgroup; nmine is free
  }
  if (shell == 0 && threadIdx.x == 0) miss[(stamp + 1u) & 1u] = 0;  // the next call's counter
  shell_block(sa, shell, red, sh_R);
}

// ------------------------------------------------------------------ launchers
hipError_t launch_bin(const TileArgs& t, const double* pos, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_bin_clear<<<(t.ntiles + 255) / 256, 256, 0, st>>>(t);
  k_bin_count<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(t, pos, n);
  k_bin_scan<<<1, 1024, 0, st>>>(t);
  k_bin_scatter<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(t, n);
  return hipGetLastError();
}

// Persistent grid over the occupied tiles (their number is only known on the
// device): per_cu workgroups per CU, at most one per tile.
static int cu_count() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    cus = (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
              ? prop.multiProcessorCount
              : 256;
  }
  return cus;
}

static unsigned tile_grid(const TileArgs& t, int per_cu) {
  return (unsigned)std::min(t.ntiles, per_cu * cu_count());
}

#define LBC_TILE_K_SWITCH(K, CALL)                        \
  switch (K) {                                            \
    case 2: { constexpr int KK = 2; CALL; } break;        \
    case 3: { constexpr int KK = 3; CALL; } break;        \
    default: { constexpr int KK = 4; CALL; } break;       \
  }
#define LBC_TILE_S_SWITCH(S, CALL)                                  \
  switch (S) {                                                      \
    case LB_F64: { constexpr int SS = LB_F64; CALL; } break;        \
    case LB_F32: { constexpr int SS = LB_F32; CALL; } break;        \
    case LB_F16: { constexpr int SS = LB_F16; CALL; } break;        \
    default: { constexpr int SS = LB_BF16; CALL; } break;           \
  }

hipError_t launch_flag_interp(int storage, int K, const SiteArgs& s, const uint64_t* mask,
                              void* U, uint32_t stamp, const double* at, double* pos, double* aux,
                              int mode, long long n, int* miss, bool all_miss, bool redo,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long nwords = mask_nwords(s.g);
  const long long per_wg = 4ll * kVelWords;
  const unsigned gv = (unsigned)std::min<long long>((nwords + per_wg - 1) / per_wg, 64ll * cu_count());
  const long long lanes = n * (K == 2 ? 4 : 16);
  const unsigned gi = (unsigned)((lanes + 255) / 256);
  // The listed markers are few once the flags follow the markers; right after
  // the fluid or the markers were set every marker is listed.
  const unsigned gs = all_miss ? gi : 64u;
  LBC_TILE_S_SWITCH(storage, (k_flag_vel<SS><<<gv, 256, 0, st>>>(s, mask, nwords, U, stamp)));
  LBC_TILE_K_SWITCH(K, LBC_TILE_S_SWITCH(storage, (k_marker_interp<SS, KK><<<gi, 256, 0, st>>>(
                                                      s, U, stamp, at, pos, aux, mode, n, miss))));
  if (redo)
    LBC_TILE_K_SWITCH(K, LBC_TILE_S_SWITCH(storage, (k_marker_slow<SS, KK><<<gs, 256, 0, st>>>(
                                                        s, U, stamp, at, pos, aux, mode, miss))));
  return hipGetLastError();
}

hipError_t launch_shell_redo_forces(int storage, int K, const ShellArgs& sa, int nshell,
                                    const SiteArgs& s, const void* U, uint32_t stamp,
                                    const double* at, double* pos, double* aux, int mode,
                                    int* miss, hipStream_t st) {
  if (nshell <= 0) return hipSuccess;
  LBC_TILE_K_SWITCH(K, LBC_TILE_S_SWITCH(storage, (k_shell_redo_forces<SS, KK><<<nshell, 256, 0, st>>>(
                                                      sa, s, U, stamp, at, pos, aux, mode, miss))));
  return hipGetLastError();
}

hipError_t launch_shell_forces(const ShellArgs& s, int nshell, hipStream_t st) {
  if (nshell > 0) k_shell_forces<<<nshell, 256, 0, st>>>(s);
  return hipGetLastError();
}

hipError_t launch_tile_spread(int storage, int K, const TileArgs& t, const double* at,
                              const double* F, void* field, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  // 38 KB of LDS: four workgroups per CU, so that the occupied tiles of a
  // dense marker set are worked on at once.
  const size_t lds = sizeof(double) * (3 * kRegSites + 6 * kSpreadChunk) + 4 * kRegRows;
  const unsigned gr = tile_grid(t, 4);
  if (storage == LB_F64) {
    LBC_TILE_K_SWITCH(K, (k_tile_spread<double, KK><<<gr, 256, lds, st>>>(t, at, F, field)));
  } else {
    LBC_TILE_K_SWITCH(K, (k_tile_spread<float, KK><<<gr, 256, lds, st>>>(t, at, F, field)));
  }
  return hipGetLastError();
}

}  // namespace lbc
