// lbc_tiles.hip -- binned, LDS-staged interpolation and spreading for dense
// Lagrangian markers (immersed-boundary shells).
//
// Markers are binned into 8x8x8 lattice tiles by the cell containing them
// (counting sort: count, single-block scan that also lists the occupied tiles
// in increasing order, scatter).  Workgroups loop over the occupied tiles;
// for each they work on a region of 13^3 sites: the tile, two sites below it
// and three above.  That covers the 2-, 3- and 4-point stencils of every
// marker binned into the tile, also after it has moved by up to one lattice
// spacing in any direction since the binning (the 4-point stencil reaches one
// node below the marker's cell and two above it).  A marker whose stencil
// leaves the region (it moved further, or across a periodic seam) takes the
// direct path that gathers from global memory.  The markers of a tile are
// staged in LDS too, in chunks.
//
//   interpolation (Eq. IBM-interpolation): the region sites that some marker
//   stencil covers are marked in an LDS bitmap and listed; their physical
//   velocities u are computed once (pull gather + pending half force) into
//   LDS (FP64 with FP64 storage, FP32 otherwise); each marker then sums K^3
//   weighted LDS entries, one lane per z-plane of stencil nodes and a butterfly
//   reduction over the lane group.
//   spreading (Eq. IBM-spreading): the stencil sites are listed the same way;
//   markers add W F into an FP64 LDS accumulator of the listed sites (LDS
//   atomics, one lane per z-plane of stencil nodes); the workgroup then adds
//   every nonzero listed site to the global force field once and flags it for
//   the lattice pass.
// Workgroups have 256 lanes, four per CU in the grid, so that nearly every
// tile of a dense marker set is worked on at once.
#include <algorithm>

#include "lbc_device.h"
#include "lbc_internal.h"

namespace lbc {

constexpr int kTile = 8;
constexpr int kLo = 2;     // region starts two sites below the tile
constexpr int kReg = 13;   // region edge: tile + 2 below + 3 above
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

// Interpolation lane groups: one lane per z-plane of stencil nodes, K planes
// rounded up to a power of two (2 lanes for K = 2, 4 for K = 3, 4), so that a
// 256-lane workgroup interpolates 64 markers at once and the group reduction
// takes one or two butterfly levels.
template <int K>
struct RowLanes {
  static constexpr int L = K == 2 ? 2 : 4;
};

// Weighted sum over the lane's plane of K x K nodes of the region moments (or
// of gathered moments for a row with a node that was not staged), reduced
// over the marker's lane group: u_p = sum_nodes W u(node),
// W = phi(x) phi(y) phi(z).
template <int S, int K>
__device__ __forceinline__ void row_interp(const SiteArgs& s, const Region& r,
                                           const typename TileT<S>::W* mu,
                                           const uint32_t* rowm, const double X[3], int lane,
                                           double up[3]) {
  using W = typename TileT<S>::W;
  constexpr int L = RowLanes<K>::L;
  const int kz = lane;
  int j0[3];
  bool inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    j0[a] = first_node<K>(X[a]);
    inside = inside && j0[a] - r.o[a] >= 0 && j0[a] - r.o[a] + K <= kReg;
  }
  W ux = 0, uy = 0, uz = 0;
  if (kz < K) {
    W wx[K], wy[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      wx[k] = phi_eval_t<W>(K, (W)((double)(j0[0] + k) - X[0]));
      wy[k] = phi_eval_t<W>(K, (W)((double)(j0[1] + k) - X[1]));
    }
    const W wz = phi_eval_t<W>(K, (W)((double)(j0[2] + kz) - X[2]));
    constexpr uint32_t km = (1u << K) - 1u;
    uint32_t miss = 0;  // rows with a node that was not staged
#pragma unroll
    for (int ky = 0; ky < K; ++ky) {
      const int jy = j0[1] + ky;
      if (s.g.wall && (jy < 0 || jy >= s.g.ny)) continue;  // beyond a wall: no node
      bool staged = inside;  // the row's K nodes must all have been staged
      if (staged) {
        const uint32_t bits = rowm[(j0[2] + kz - r.o[2]) * kReg + (jy - r.o[1])];
        staged = ((bits >> (j0[0] - r.o[0])) & km) == km;
      }
      if (!staged) {
        miss |= 1u << ky;
        continue;
      }
      const W* row = mu + ((j0[2] + kz - r.o[2]) * kReg + (jy - r.o[1])) * kReg + (j0[0] - r.o[0]);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const W Wt = wx[k] * (wy[ky] * wz);
        if (Wt == W(0)) continue;
        ux += Wt * row[k];
        uy += Wt * row[kRegSites + k];
        uz += Wt * row[2 * kRegSites + k];
      }
    }
    // direct path (rare): gather the missing rows' nodes from global memory,
    // weights recomputed so that no array is indexed at run time
#pragma unroll 1
    for (int ky = 0; miss != 0u && ky < K; ++ky) {
      const int jy = j0[1] + ky;
      if (!((miss >> ky) & 1u)) continue;
      const W wyz = phi_eval_t<W>(K, (W)((double)jy - X[1])) * wz;
      const int y = s.g.wall ? jy : wrap_idx(jy, s.g.ny), z = wrap_idx(j0[2] + kz, s.g.nz);
#pragma unroll 1
      for (int k = 0; k < K; ++k) {
        const W Wt = phi_eval_t<W>(K, (W)((double)(j0[0] + k) - X[0])) * wyz;
        if (Wt == W(0)) continue;
        W drho, j[3];
        site_phys_r_seq<S, W>(s, wrap_idx(j0[0] + k, s.g.nx), y, z, drho, j);
        const W rr = W(s.rho0) + drho;
        ux += Wt * (j[0] / rr);
        uy += Wt * (j[1] / rr);
        uz += Wt * (j[2] / rr);
      }
    }
  }
  up[0] = (double)group_sum_t<L, W>(ux);
  up[1] = (double)group_sum_t<L, W>(uy);
  up[2] = (double)group_sum_t<L, W>(uz);
}

// Interpolation and spreading workgroups are small (256 lanes) so that the
// occupied tiles of a dense marker set are worked on nearly all at once: the
// grid holds four per CU.  In FP32 four interpolation workgroups are resident
// per CU (128 registers, which the rolled direct-path gather keeps within
// reach; the staged velocities, one marker chunk and the staging lists take
// 38 KB of LDS) and three spreading ones (40 KB of LDS each).
constexpr int kInterpLanes = 256;
constexpr int kInterpWgPerCu = 4;
constexpr int kInterpChunk = 128;
constexpr int kSpreadLanes = 256;
constexpr int kSpreadWgPerCu = 4;
constexpr int kSpreadChunk = 128;
constexpr int kSpreadCap = 1024;  // accumulated sites per tile

// Markers of the tile being processed, staged in LDS in chunks of C
// (index and the positions and forces the kernel reads), so that the marker
// loops never wait on dependent global loads.
template <int C>
struct MarkerLds {
  static constexpr int kChunk = C;
  int p[C];
  double X[C][3];  // position the stencil is built at
  double Y[C][3];  // second vector: pos (interpolation) or force (spreading)
};

// Which region slots the interpolation stages.  Only the slots inside some
// marker's stencil are read, about a quarter of the region for markers on a
// surface, so the workgroup first marks the stencils of its markers (at the
// positions it knows, widened by kMarkDelta for the drifts of the pass) in a
// bitmap with one kReg-bit x mask per (y, z) row, then lists the marked slots
// and stages only those.  A stencil row with an unstaged node takes the
// direct path, so the bitmap decides speed, not results.
constexpr double kMarkDelta = 0.05;
constexpr int kRows = kReg * kReg;
constexpr int kListWaves = (kRegSites + 63) / 64;
static_assert(kListWaves <= 64, "segment offsets are scanned by one wavefront");

struct StageLds {
  uint32_t rowm[kRows];         // x mask of marked slots per (y, z) row
  int cnt[kListWaves];          // marked slots per 64-slot segment, then their offsets
  unsigned short list[kRegSites];  // marked slots, increasing
  int nlist;
};

// Mark the slots of the K-point stencils of X - d .. X + d (per axis),
// clipped to the region; lanes g of a group of G cover the rows.
template <int K>
__device__ __forceinline__ void mark_stencil(const Region& r, const double X[3], double d,
                                             uint32_t* rowm, int g, int G) {
  int lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = max(first_node<K>(X[a] - d) - r.o[a], 0);
    hi[a] = min(first_node<K>(X[a] + d) + K - 1 - r.o[a], kReg - 1);
  }
  if (lo[0] > hi[0] || lo[1] > hi[1] || lo[2] > hi[2]) return;
  const uint32_t xb = ((1u << (hi[0] - lo[0] + 1)) - 1u) << lo[0];
  const int ny = hi[1] - lo[1] + 1, nrow = ny * (hi[2] - lo[2] + 1);
  for (int q = g; q < nrow; q += G)
    atomicOr(rowm + (lo[2] + q / ny) * kReg + lo[1] + q % ny, xb);
}

// List the slots marked in sg->rowm in increasing order: per 64-slot segment
// a wave ballot counts them, one wavefront scans the counts into offsets, and
// every marked slot writes itself at its offset plus its rank in the ballot.
// idx (optional) receives each listed slot's list position.  Called after a
// barrier that follows the marking; ends with a barrier.
__device__ __forceinline__ void list_marked(StageLds* sg, unsigned short* idx) {
  const int wv = (int)threadIdx.x / 64;
  for (int k0 = 0; k0 < kRegSites; k0 += (int)blockDim.x) {
    const int seg = k0 / 64 + wv, k = k0 + (int)threadIdx.x;  // wave wv: slots 64 seg ..
    if (seg >= kListWaves) continue;  // (uniform over the wave)
    const bool on = k < kRegSites && ((sg->rowm[k / kReg] >> (k % kReg)) & 1u);
    const uint64_t b = __ballot(on);
    if (threadIdx.x % 64 == 0) sg->cnt[seg] = (int)__popcll(b);
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // segment counts -> exclusive offsets (one wave)
    const int l = (int)threadIdx.x, v = l < kListWaves ? sg->cnt[l] : 0;
    int incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int u = __shfl_up(incl, d, 64);
      if (l >= d) incl += u;
    }
    if (l < kListWaves) sg->cnt[l] = incl - v;
    if (l == 63) sg->nlist = incl;
  }
  __syncthreads();
  for (int k0 = 0; k0 < kRegSites; k0 += (int)blockDim.x) {
    const int seg = k0 / 64 + wv, k = k0 + (int)threadIdx.x;
    if (seg >= kListWaves) continue;
    const bool on = k < kRegSites && ((sg->rowm[k / kReg] >> (k % kReg)) & 1u);
    const uint64_t b = __ballot(on);
    const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
    if (on) {
      const int at = sg->cnt[seg] + below;
      sg->list[at] = (unsigned short)k;
      if (idx) idx[k] = (unsigned short)at;
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------- interpolation
// mode 0: IB predictor       aux = wrap(pos + h/2 u(pos))
// mode 1: IB advection       pos = wrap(pos + h/2 u(aux))
// mode 2: both, in that order, from one staged region (at = pos); the first
//         advection only needs the state before the lattice pass, like the
//         predictor, so both read the same LDS moments.
// mode 3: mode 1 of one step followed by mode 2 of the next (at = aux): the
//         final advection of a step and the predictor and first advection of
//         the next read the same fluid state, so one staging serves all three.
// A marker whose stencil leaves the region gathers its nodes from global
// memory instead (same arithmetic per node).  Workgroups loop over the
// occupied tiles (persistent grid).
template <int S, int K>
__global__ __launch_bounds__(kInterpLanes) void k_tile_interp(TileArgs t, SiteArgs s,
                                                              const double* at, double* pos,
                                                              double* aux, int mode) {
  constexpr int L = RowLanes<K>::L;
  constexpr int G = 16;  // lanes per marker while marking
  using W = typename TileT<S>::W;
  using MK = MarkerLds<kInterpChunk>;
  constexpr int kChunk = MK::kChunk;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  W* mu = (W*)lds_raw;                                                // 3 * kRegSites
  MK* mk = (MK*)(lds_raw + sizeof(W) * 3 * kRegSites);                // one chunk
  StageLds* sg = (StageLds*)(lds_raw + sizeof(W) * 3 * kRegSites + sizeof(MK));
  const int lane = threadIdx.x % L;
  const int nocc = t.nocc[0];
  const bool two = mode == 1 || mode == 3;  // pos is read as well as at
  auto load_chunk = [&](int c0, int nc) {
    for (int i = threadIdx.x; i < nc; i += blockDim.x) {
      const int p = t.sorted[c0 + i];
      mk->p[i] = p;
      for (int a = 0; a < 3; ++a) {
        mk->X[i][a] = at[3 * (long long)p + a];
        mk->Y[i][a] = two ? pos[3 * (long long)p + a] : 0.0;
      }
    }
  };
  for (int ot = blockIdx.x; ot < nocc; ot += gridDim.x) {
    const int tl = t.occ[ot];
    const Region r = region_of(t, tl);
    const int b0 = t.start[tl], b1 = t.start[tl + 1];
    // first marker chunk, and a cleared bitmap
    load_chunk(b0, min(kChunk, b1 - b0));
    for (int k = threadIdx.x; k < kRows; k += blockDim.x) sg->rowm[k] = 0u;
    __syncthreads();
    // mark the stencils the pass will read: at at and, where it is also
    // interpolated from, at pos (mode 3: the final advection starts there)
    for (int i = (int)threadIdx.x / G; i < b1 - b0; i += (int)blockDim.x / G) {
      double X[3], Y[3];
      if (i < kChunk) {
        for (int a = 0; a < 3; ++a) {
          X[a] = mk->X[i][a];
          Y[a] = mk->Y[i][a];
        }
      } else {
        const long long p = t.sorted[b0 + i];
        for (int a = 0; a < 3; ++a) {
          X[a] = at[3 * p + a];
          Y[a] = two ? pos[3 * p + a] : 0.0;
        }
      }
      mark_stencil<K>(r, X, kMarkDelta, sg->rowm, (int)threadIdx.x % G, G);
      if (mode == 3) mark_stencil<K>(r, Y, kMarkDelta, sg->rowm, (int)threadIdx.x % G, G);
    }
    __syncthreads();
    list_marked(sg, nullptr);
    const int nlist = sg->nlist;
    for (int i = threadIdx.x; i < nlist; i += blockDim.x) {
      const int k = sg->list[i];
      const int ix = k % kReg, iy = (k / kReg) % kReg, iz = k / (kReg * kReg);
      int x, y, z;
      W u0 = W(0), u1 = W(0), u2 = W(0);  // beyond a wall: never read
      if (slot_site(s.g, r, ix, iy, iz, x, y, z)) {
        W drho, j[3];
        site_phys_r<S, W>(s, x, y, z, drho, j);
        const W rr = W(s.rho0) + drho;
        u0 = j[0] / rr;
        u1 = j[1] / rr;
        u2 = j[2] / rr;
      }
      mu[k] = u0;
      mu[kRegSites + k] = u1;
      mu[2 * kRegSites + k] = u2;
    }
    auto interp_at = [&](const double X[3], double up[3]) {
      row_interp<S, K>(s, r, mu, sg->rowm, X, lane, up);
    };
    auto half_drift = [&](const double from[3], const double u[3], double to[3]) {
      for (int a = 0; a < 3; ++a) to[a] = from[a] + 0.5 * u[a];
      to[0] = wrap_pos(to[0], (double)s.g.nx);
      if (!s.g.wall) to[1] = wrap_pos(to[1], (double)s.g.ny);
      to[2] = wrap_pos(to[2], (double)s.g.nz);
    };
    for (int c0 = b0; c0 < b1; c0 += kChunk) {
      const int nc = min(kChunk, b1 - c0);
      if (c0 != b0) {
        __syncthreads();  // previous chunk done with mk
        load_chunk(c0, nc);
      }
      __syncthreads();  // staged moments (first chunk) or the new chunk ready
      for (int i = (int)threadIdx.x / L; i < nc; i += (int)blockDim.x / L) {  // groups leave together
        const long long p = mk->p[i];
        const double X[3] = {mk->X[i][0], mk->X[i][1], mk->X[i][2]};
        const double P[3] = {mk->Y[i][0], mk->Y[i][1], mk->Y[i][2]};
        // Interpolation points in order (one call site, so the interpolation
        // is compiled once): mode 0, 1: X; mode 2: X, then X~ = X + h/2 u(X);
        // mode 3: X (= X~ of the previous step), then Xs = P + h/2 u(X), then
        // X~ = Xs + h/2 u(Xs).  Xs is the point the last half drift starts from.
        const int nint = mode == 3 ? 3 : (mode == 2 ? 2 : 1);
        double q[3] = {X[0], X[1], X[2]}, Xs[3] = {X[0], X[1], X[2]}, u[3], Y[3];
#pragma unroll 1
        for (int it = 0; it < nint; ++it) {
          interp_at(q, u);
          if (it + 1 == nint) break;
          if (mode == 3 && it == 0) {
            half_drift(P, u, Xs);
            for (int a = 0; a < 3; ++a) q[a] = Xs[a];
          } else {
            half_drift(Xs, u, q);
          }
        }
        if (mode == 0) {  // predictor only
          half_drift(X, u, Y);
          if (lane == 0)
            for (int a = 0; a < 3; ++a) aux[3 * p + a] = Y[a];
        } else if (mode == 1) {  // advection with the velocity at X~ = at
          half_drift(P, u, Y);
          if (lane == 0)
            for (int a = 0; a < 3; ++a) pos[3 * p + a] = Y[a];
        } else {  // X~ = q, and X <- Xs + h/2 u(X~)
          half_drift(Xs, u, Y);
          if (lane == 0)
            for (int a = 0; a < 3; ++a) {
              aux[3 * p + a] = q[a];
              pos[3 * p + a] = Y[a];
            }
        }
      }
    }
    __syncthreads();  // region moments and bitmap are overwritten by the next tile
  }
}

// ------------------------------------------------------------------ spreading
// The accumulator is FP64 whatever the field precision: LDS atomic adds run
// several times faster in FP64 than in FP32 on this device.  It holds only
// the region sites the tile's stencils cover (listed as in the
// interpolation, at most kSpreadCap of them; a node listed beyond that adds
// to the global field directly), so that the workgroup's LDS stays small.
// Global adds go through atomics: the regions of neighbouring tiles overlap.
template <typename E, int K>
__global__ __launch_bounds__(kSpreadLanes) void k_tile_spread(TileArgs t, const double* at,
                                                              const double* F, void* field) {
  constexpr int L = RowLanes<K>::L;
  constexpr int G = 16;  // lanes per marker while marking
  using MK = MarkerLds<kSpreadChunk>;
  constexpr int kChunk = MK::kChunk;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* acc = (double*)lds_raw;                                    // 3 * kSpreadCap
  MK* mk = (MK*)(lds_raw + sizeof(double) * 3 * kSpreadCap);        // one chunk
  StageLds* sg = (StageLds*)((unsigned char*)mk + sizeof(MK));
  unsigned short* idx = (unsigned short*)((unsigned char*)sg + sizeof(StageLds));  // kRegSites
  E* Fd = (E*)field;
  const int lane = threadIdx.x % L;
  const int nocc = t.nocc[0];
  auto load_chunk = [&](int c0, int nc) {
    for (int i = threadIdx.x; i < nc; i += blockDim.x) {
      const int p = t.sorted[c0 + i];
      mk->p[i] = p;
      for (int a = 0; a < 3; ++a) {
        mk->X[i][a] = at[3 * (long long)p + a];
        mk->Y[i][a] = F[3 * (long long)p + a];
      }
    }
  };
  auto global_add = [&](int jx, int jy, int jz, double f0, double f1, double f2) {
    const int j[3] = {jx, jy, jz};
    int x, y, z;
    if (!node_site(t.g, j, x, y, z)) return;  // beyond a wall
    const long long sidx = site_index(t.g, x, y, z);
    unsafeAtomicAdd(Fd + 4 * sidx + 0, (E)f0);
    unsafeAtomicAdd(Fd + 4 * sidx + 1, (E)f1);
    unsafeAtomicAdd(Fd + 4 * sidx + 2, (E)f2);
    uint64_t bit;
    flag_site(mask_word(t.mask, t.g, x, y, z, bit), bit);
  };
  for (int ot = blockIdx.x; ot < nocc; ot += gridDim.x) {
    const int tl = t.occ[ot];
    const Region r = region_of(t, tl);
    const int b0 = t.start[tl], b1 = t.start[tl + 1];
    load_chunk(b0, min(kChunk, b1 - b0));
    for (int k = threadIdx.x; k < kRows; k += blockDim.x) sg->rowm[k] = 0u;
    __syncthreads();
    for (int i = (int)threadIdx.x / G; i < b1 - b0; i += (int)blockDim.x / G) {
      double X[3];
      if (i < kChunk) {
        for (int a = 0; a < 3; ++a) X[a] = mk->X[i][a];
      } else {
        const long long p = t.sorted[b0 + i];
        for (int a = 0; a < 3; ++a) X[a] = at[3 * p + a];
      }
      mark_stencil<K>(r, X, 0.0, sg->rowm, (int)threadIdx.x % G, G);
    }
    __syncthreads();
    list_marked(sg, idx);
    const int nacc = min(sg->nlist, kSpreadCap);
    for (int k = threadIdx.x; k < 3 * nacc; k += blockDim.x) acc[k] = 0.0;
    for (int c0 = b0; c0 < b1; c0 += kChunk) {
      const int nc = min(kChunk, b1 - c0);
      if (c0 != b0) {
        __syncthreads();  // previous chunk done with mk
        load_chunk(c0, nc);
      }
      __syncthreads();  // accumulator cleared (first chunk) or the new chunk ready
      for (int i = (int)threadIdx.x / L; i < nc; i += (int)blockDim.x / L) {
        const int kz = lane;
        if (kz >= K) continue;
        const double X[3] = {mk->X[i][0], mk->X[i][1], mk->X[i][2]};
        const double Fp[3] = {mk->Y[i][0], mk->Y[i][1], mk->Y[i][2]};
        int j0[3];
        bool inside = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          j0[a] = first_node<K>(X[a]);
          inside = inside && j0[a] - r.o[a] >= 0 && j0[a] - r.o[a] + K <= kReg;
        }
        E wx[K], wy[K];  // weights in the field precision
#pragma unroll
        for (int k = 0; k < K; ++k) {
          wx[k] = phi_eval_t<E>(K, (E)((double)(j0[0] + k) - X[0]));
          wy[k] = phi_eval_t<E>(K, (E)((double)(j0[1] + k) - X[1]));
        }
        const E wz = phi_eval_t<E>(K, (E)((double)(j0[2] + kz) - X[2]));
#pragma unroll
        for (int ky = 0; ky < K; ++ky) {
          const int jy = j0[1] + ky;
          if (t.g.wall && (jy < 0 || jy >= t.g.ny)) continue;  // beyond a wall
          const int rowslot = inside ? ((j0[2] + kz - r.o[2]) * kReg + (jy - r.o[1])) * kReg +
                                           (j0[0] - r.o[0])
                                     : 0;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const double W = (double)(wx[k] * wy[ky] * wz);
            if (W == 0.0) continue;
            const double f0 = W * Fp[0], f1 = W * Fp[1], f2 = W * Fp[2];
            const int q = inside ? (int)idx[rowslot + k] : kSpreadCap;
            if (q < kSpreadCap) {
              double* a = acc + 3 * q;
              atomicAdd(a + 0, f0);
              atomicAdd(a + 1, f1);
              atomicAdd(a + 2, f2);
            } else {
              global_add(j0[0] + k, jy, j0[2] + kz, f0, f1, f2);
            }
          }
        }
      }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nacc; q += blockDim.x) {
      const E a0 = (E)acc[3 * q], a1 = (E)acc[3 * q + 1], a2 = (E)acc[3 * q + 2];
      if (a0 == E(0) && a1 == E(0) && a2 == E(0)) continue;
      const int k = sg->list[q];
      const int ix = k % kReg, iy = (k / kReg) % kReg, iz = k / (kReg * kReg);
      int x, y, z;
      if (!slot_site(t.g, r, ix, iy, iz, x, y, z)) continue;
      const long long sidx = site_index(t.g, x, y, z);
      unsafeAtomicAdd(Fd + 4 * sidx + 0, a0);
      unsafeAtomicAdd(Fd + 4 * sidx + 1, a1);
      unsafeAtomicAdd(Fd + 4 * sidx + 2, a2);
      uint64_t bit;
      flag_site(mask_word(t.mask, t.g, x, y, z, bit), bit);
    }
    __syncthreads();  // accumulator, lists and chunk are reused by the next tile
  }
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
static unsigned tile_grid(const TileArgs& t, int per_cu) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    cus = (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
              ? prop.multiProcessorCount
              : 256;
  }
  return (unsigned)std::min(t.ntiles, per_cu * cus);
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

hipError_t launch_tile_interp(int storage, int K, const TileArgs& t, const SiteArgs& s,
                              const double* at, double* pos, double* aux, int mode, long long n,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  LBC_TILE_K_SWITCH(K, LBC_TILE_S_SWITCH(storage, (k_tile_interp<SS, KK>
      <<<tile_grid(t, kInterpWgPerCu), kInterpLanes,
         sizeof(typename TileT<SS>::W) * 3 * kRegSites + sizeof(MarkerLds<kInterpChunk>) +
             sizeof(StageLds), st>>>(t, s, at, pos, aux, mode))));
  return hipGetLastError();
}

hipError_t launch_tile_spread(int storage, int K, const TileArgs& t, const double* at,
                              const double* F, void* field, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const size_t lds = sizeof(double) * 3 * kSpreadCap + sizeof(MarkerLds<kSpreadChunk>) +
                     sizeof(StageLds) + sizeof(unsigned short) * kRegSites;
  const unsigned gr = tile_grid(t, kSpreadWgPerCu);
  if (storage == LB_F64) {
    LBC_TILE_K_SWITCH(K, (k_tile_spread<double, KK><<<gr, kSpreadLanes, lds, st>>>(t, at, F, field)));
  } else {
    LBC_TILE_K_SWITCH(K, (k_tile_spread<float, KK><<<gr, kSpreadLanes, lds, st>>>(t, at, F, field)));
  }
  return hipGetLastError();
}

}  // namespace lbc
