// lbc_tiles.hip -- binned, LDS-staged interpolation and spreading for dense
// Lagrangian markers (immersed-boundary shells).
//
// Markers are binned into 8x8x8 lattice tiles by the cell containing them
// (counting sort: count, single-block scan that also lists the occupied tiles
// in increasing order, scatter).  Workgroups loop over the occupied tiles;
// for each they work on a staged region of 12^3 sites: the tile and two sites
// on each side.  That covers the 2-, 3- and 4-point stencils of every marker
// binned into the tile, also after it has moved down by up to one lattice
// spacing or up within its cell.  A marker whose stencil leaves the region
// (it crossed the upper cell face or a periodic seam, or the binning is a few
// steps old) takes the direct path that gathers from global memory.  The
// markers of a tile are staged in LDS too, in chunks.
//
//   interpolation (Eq. IBM-interpolation): physical moments rho, u of every
//   region site are computed once (pull gather + pending half force) into LDS
//   in FP64; each marker then sums K^3 weighted LDS entries, one lane per
//   x-row of stencil nodes and a butterfly reduction over the lane group.
//   spreading (Eq. IBM-spreading): markers add W F into an FP64 LDS
//   accumulator of the region (LDS atomics, one lane per stencil site); the
//   workgroup then adds every nonzero region site to the global force field
//   once and flags it for the lattice pass.
// Workgroups have 1024 lanes so that staging and flushing a region take two
// rounds of loads with sixteen wavefronts in flight.
#include <algorithm>

#include "lbc_device.h"
#include "lbc_internal.h"

namespace lbc {

constexpr int kTile = 8;
constexpr int kLo = 2;     // region starts two sites below the tile
constexpr int kReg = 12;   // region edge: tile + 2 below + 2 above
constexpr int kRegSites = kReg * kReg * kReg;

__device__ __forceinline__ int tile_of(const TileArgs& t, const double X[3], int c[3]) {
  const int n[3] = {t.g.nx, t.g.ny, t.g.nz};
  for (int a = 0; a < 3; ++a) {
    int j = (int)floor(X[a]);
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

// One lane of a marker's lane group: stencil node (kx, ky, kz) = lane
// (x fastest) of the K-point stencil whose first node is j0 (Appendix A
// kernels), its weight (evaluated in T), and the node's region slot.
template <int K>
struct Node {
  bool on;       // lane carries a node of nonzero weight
  bool inside;   // the whole stencil lies in the staged region (same for the group)
  double W;
  int j[3];      // unwrapped node coordinates
  int slot;      // region slot (when inside)
};

template <int K, typename T>
__device__ __forceinline__ Node<K> node_of(const Region& r, const double X[3], int lane) {
  Node<K> n;
  const int k[3] = {lane % K, (lane / K) % K, lane / (K * K)};
  n.inside = true;
  T w = T(1);
  int rel[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int j0 = first_node<K>(X[a]);
    n.inside = n.inside && j0 - r.o[a] >= 0 && j0 - r.o[a] + K <= kReg;
    n.j[a] = j0 + k[a];
    rel[a] = n.j[a] - r.o[a];
    w *= phi_eval_t<T>(K, (T)((double)n.j[a] - X[a]));
  }
  n.W = (double)w;
  n.on = lane < K * K * K && n.W != 0.0;
  n.slot = (rel[2] * kReg + rel[1]) * kReg + rel[0];
  return n;
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
  using M4 = double4;
};
template <>
struct TileT<LB_F32> {
  using W = float;
  using M4 = float4;
};
template <>
struct TileT<LB_F16> {
  using W = float;
  using M4 = float4;
};
template <>
struct TileT<LB_BF16> {
  using W = float;
  using M4 = float4;
};

// Interpolation lane groups: one lane per x-row of stencil nodes (ky, kz),
// K^2 rows rounded up to a power of two (4 lanes for K = 2, 16 for K = 3, 4).
template <int K>
struct RowLanes {
  static constexpr int L = K == 2 ? 4 : 16;
};

// Weighted sum over the lane's row of K nodes of the region moments (or of
// gathered moments when the stencil leaves the region), reduced over the
// marker's lane group: u_p = sum_nodes W u(node), W = phi(x) phi(y) phi(z).
template <int S, int K>
__device__ __forceinline__ void row_interp(const SiteArgs& s, const Region& r,
                                           const typename TileT<S>::M4* mom, const double X[3],
                                           int lane, double up[3]) {
  using W = typename TileT<S>::W;
  constexpr int L = RowLanes<K>::L;
  const int ky = lane % K, kz = lane / K;
  int j0[3];
  bool inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    j0[a] = first_node<K>(X[a]);
    inside = inside && j0[a] - r.o[a] >= 0 && j0[a] - r.o[a] + K <= kReg;
  }
  W ux = 0, uy = 0, uz = 0;
  if (lane < K * K) {
    W wx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) wx[k] = phi_eval_t<W>(K, (W)((double)(j0[0] + k) - X[0]));
    const W wy = phi_eval_t<W>(K, (W)((double)(j0[1] + ky) - X[1]));
    const W wz = phi_eval_t<W>(K, (W)((double)(j0[2] + kz) - X[2]));
    if (inside) {
      const typename TileT<S>::M4* row =
          mom + ((j0[2] + kz - r.o[2]) * kReg + (j0[1] + ky - r.o[1])) * kReg + (j0[0] - r.o[0]);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const W Wt = wx[k] * wy * wz;
        if (Wt == W(0)) continue;
        const typename TileT<S>::M4 m = row[k];
        if (m.x == W(0)) continue;  // beyond a wall
        ux += Wt * m.y;
        uy += Wt * m.z;
        uz += Wt * m.w;
      }
    } else {
      const int jy = j0[1] + ky;
      const bool in_y = !s.g.wall || (jy >= 0 && jy < s.g.ny);
      for (int k = 0; k < K && in_y; ++k) {
        const W Wt = wx[k] * wy * wz;
        if (Wt == W(0)) continue;
        const int x = wrap_idx(j0[0] + k, s.g.nx), z = wrap_idx(j0[2] + kz, s.g.nz);
        const int y = s.g.wall ? jy : wrap_idx(jy, s.g.ny);
        W drho, j[3];
        site_phys_r<S, W>(s, x, y, z, drho, j);
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

// Markers of the tile being processed, staged in LDS in chunks of kChunk
// (index and the positions and forces the kernel reads), so that the marker
// loops never wait on dependent global loads.
constexpr int kChunk = 256;

struct MarkerLds {
  int p[kChunk];
  double X[kChunk][3];  // position the stencil is built at
  double Y[kChunk][3];  // second vector: pos (interpolation) or force (spreading)
};

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
__global__ __launch_bounds__(1024) void k_tile_interp(TileArgs t, SiteArgs s, const double* at,
                                                      double* pos, double* aux, int mode) {
  constexpr int L = RowLanes<K>::L;
  using W = typename TileT<S>::W;
  using M4 = typename TileT<S>::M4;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  M4* mom = (M4*)lds_raw;                                          // kRegSites
  MarkerLds* mk = (MarkerLds*)(lds_raw + sizeof(M4) * kRegSites);  // one chunk
  const int lane = threadIdx.x % L;
  const int nocc = t.nocc[0];
  for (int ot = blockIdx.x; ot < nocc; ot += gridDim.x) {
    const int tl = t.occ[ot];
    const Region r = region_of(t, tl);
    for (int k = threadIdx.x; k < kRegSites; k += blockDim.x) {
      const int ix = k % kReg, iy = (k / kReg) % kReg, iz = k / (kReg * kReg);
      int x, y, z;
      M4 m;
      m.x = m.y = m.z = m.w = W(0);
      if (slot_site(s.g, r, ix, iy, iz, x, y, z)) {
        W drho, j[3];
        site_phys_r<S, W>(s, x, y, z, drho, j);
        const W rr = W(s.rho0) + drho;
        m.x = rr;
        m.y = j[0] / rr;
        m.z = j[1] / rr;
        m.w = j[2] / rr;
      }
      mom[k] = m;
    }
    auto interp_at = [&](const double X[3], double up[3]) {
      row_interp<S, K>(s, r, mom, X, lane, up);
    };
    auto half_drift = [&](const double from[3], const double u[3], double to[3]) {
      for (int a = 0; a < 3; ++a) to[a] = from[a] + 0.5 * u[a];
      to[0] = wrap_pos(to[0], (double)s.g.nx);
      if (!s.g.wall) to[1] = wrap_pos(to[1], (double)s.g.ny);
      to[2] = wrap_pos(to[2], (double)s.g.nz);
    };
    const int b0 = t.start[tl], b1 = t.start[tl + 1];
    for (int c0 = b0; c0 < b1; c0 += kChunk) {
      const int nc = min(kChunk, b1 - c0);
      __syncthreads();  // previous chunk (or region staging) done with mk
      for (int i = threadIdx.x; i < nc; i += blockDim.x) {
        const int p = t.sorted[c0 + i];
        mk->p[i] = p;
        for (int a = 0; a < 3; ++a) {
          mk->X[i][a] = at[3 * (long long)p + a];
          mk->Y[i][a] = (mode == 1 || mode == 3) ? pos[3 * (long long)p + a] : 0.0;
        }
      }
      __syncthreads();
      for (int i = (int)threadIdx.x / L; i < nc; i += (int)blockDim.x / L) {  // groups leave together
        const long long p = mk->p[i];
        const double X[3] = {mk->X[i][0], mk->X[i][1], mk->X[i][2]};
        double up[3], Y[3];
        interp_at(X, up);
        if (mode == 0) {  // predictor only
          half_drift(X, up, Y);
          if (lane == 0)
            for (int a = 0; a < 3; ++a) aux[3 * p + a] = Y[a];
        } else if (mode == 1) {  // advection with the velocity at X~ = at
          const double P[3] = {mk->Y[i][0], mk->Y[i][1], mk->Y[i][2]};
          half_drift(P, up, Y);
          if (lane == 0)
            for (int a = 0; a < 3; ++a) pos[3 * p + a] = Y[a];
        } else {
          // mode 2: predictor, then the first advection from the same staged
          // state; mode 3: first the final advection of the previous step
          double Xs[3], Xt[3], u0[3], u2[3];
          if (mode == 3) {
            const double P[3] = {mk->Y[i][0], mk->Y[i][1], mk->Y[i][2]};
            half_drift(P, up, Xs);
            interp_at(Xs, u0);
          } else {
            for (int a = 0; a < 3; ++a) {
              Xs[a] = X[a];
              u0[a] = up[a];
            }
          }
          half_drift(Xs, u0, Xt);
          interp_at(Xt, u2);
          half_drift(Xs, u2, Y);
          if (lane == 0)
            for (int a = 0; a < 3; ++a) {
              aux[3 * p + a] = Xt[a];
              pos[3 * p + a] = Y[a];
            }
        }
      }
    }
    __syncthreads();  // region moments are overwritten by the next tile
  }
}

// ------------------------------------------------------------------ spreading
// The region accumulator is FP64 whatever the field precision: LDS atomic
// adds run several times faster in FP64 than in FP32 on this device.
template <typename E, int K>
__global__ __launch_bounds__(1024) void k_tile_spread(TileArgs t, const double* at,
                                                      const double* F, void* field) {
  constexpr int L = Lanes<K>::L;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  MarkerLds* mk = (MarkerLds*)lds_raw;                     // one chunk
  double* acc = (double*)(lds_raw + sizeof(MarkerLds));    // 3 * kRegSites
  E* Fd = (E*)field;
  const int lane = threadIdx.x % L;
  const int nocc = t.nocc[0];
  for (int ot = blockIdx.x; ot < nocc; ot += gridDim.x) {
    const int tl = t.occ[ot];
    const Region r = region_of(t, tl);
    for (int k = threadIdx.x; k < 3 * kRegSites; k += blockDim.x) acc[k] = 0.0;
    const int b0 = t.start[tl], b1 = t.start[tl + 1];
    for (int c0 = b0; c0 < b1; c0 += kChunk) {
      const int nc = min(kChunk, b1 - c0);
      __syncthreads();  // previous chunk done with mk (and acc cleared)
      for (int i = threadIdx.x; i < nc; i += blockDim.x) {
        const int p = t.sorted[c0 + i];
        mk->p[i] = p;
        for (int a = 0; a < 3; ++a) {
          mk->X[i][a] = at[3 * (long long)p + a];
          mk->Y[i][a] = F[3 * (long long)p + a];
        }
      }
      __syncthreads();
      for (int i = (int)threadIdx.x / L; i < nc; i += (int)blockDim.x / L) {
        const double X[3] = {mk->X[i][0], mk->X[i][1], mk->X[i][2]};
        const Node<K> n = node_of<K, E>(r, X, lane);  // weights in the field precision
        if (!n.on) continue;
        if (t.g.wall && (n.j[1] < 0 || n.j[1] >= t.g.ny)) continue;  // beyond a wall
        const double f0 = n.W * mk->Y[i][0], f1 = n.W * mk->Y[i][1], f2 = n.W * mk->Y[i][2];
        if (n.inside) {
          double* a = acc + 3 * n.slot;
          atomicAdd(a + 0, f0);
          atomicAdd(a + 1, f1);
          atomicAdd(a + 2, f2);
        } else {
          int x, y, z;
          node_site(t.g, n.j, x, y, z);
          const long long sidx = site_index(t.g, x, y, z);
          unsafeAtomicAdd(Fd + 4 * sidx + 0, (E)f0);
          unsafeAtomicAdd(Fd + 4 * sidx + 1, (E)f1);
          unsafeAtomicAdd(Fd + 4 * sidx + 2, (E)f2);
          uint64_t bit;
          flag_site(mask_word(t.mask, t.g, x, y, z, bit), bit);
        }
      }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kRegSites; k += blockDim.x) {
      const E a0 = (E)acc[3 * k], a1 = (E)acc[3 * k + 1], a2 = (E)acc[3 * k + 2];
      if (a0 == E(0) && a1 == E(0) && a2 == E(0)) continue;
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
    __syncthreads();  // acc is cleared for the next tile
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
// device): two 1024-lane workgroups per CU, at most one per tile.
static unsigned tile_grid(const TileArgs& t) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    cus = (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
              ? prop.multiProcessorCount
              : 256;
  }
  return (unsigned)std::min(t.ntiles, 2 * cus);
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
      <<<tile_grid(t), 1024, sizeof(typename TileT<SS>::M4) * kRegSites + sizeof(MarkerLds), st>>>(
          t, s, at, pos, aux, mode))));
  return hipGetLastError();
}

hipError_t launch_tile_spread(int storage, int K, const TileArgs& t, const double* at,
                              const double* F, void* field, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const size_t lds = sizeof(MarkerLds) + sizeof(double) * 3 * kRegSites;
  if (storage == LB_F64) {
    LBC_TILE_K_SWITCH(K, (k_tile_spread<double, KK><<<tile_grid(t), 1024, lds, st>>>(t, at, F, field)));
  } else {
    LBC_TILE_K_SWITCH(K, (k_tile_spread<float, KK><<<tile_grid(t), 1024, lds, st>>>(t, at, F, field)));
  }
  return hipGetLastError();
}

}  // namespace lbc
