// lbc_tiles.hip -- binned, LDS-staged interpolation and spreading for dense
// Lagrangian markers (immersed-boundary shells).
//
// Markers are binned into 8x8x8 lattice tiles by the cell containing them
// (counting sort: count, single-block scan that also lists the occupied tiles
// in increasing order, scatter).  A workgroup then owns one occupied tile and
// works on a staged region of 12^3 sites: the tile and two sites on each side.
// That covers the 2-, 3- and 4-point stencils of every marker binned into the
// tile, also after it has moved down by up to one lattice spacing or up within
// its cell, so one binning serves the whole time step.  A marker whose stencil
// leaves the region (it crossed the upper cell face or a periodic seam) takes
// the direct path that gathers from global memory.
//
//   interpolation (Eq. IBM-interpolation): physical moments rho, u of every
//   region site are computed once (pull gather + pending half force) into LDS
//   in FP64; each marker then sums K^3 weighted LDS entries.
//   spreading (Eq. IBM-spreading): markers add W F into an LDS accumulator of
//   the region (LDS atomics); the workgroup then adds every nonzero region site
//   to the global force field once and sets its mask bit if not yet set.
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
// list of occupied tiles in increasing tile order.
__global__ __launch_bounds__(1024) void k_bin_scan(TileArgs t) {
  __shared__ int sc[1024];
  __shared__ int so[1024];
  __shared__ int carry[2];
  if (threadIdx.x == 0) carry[0] = carry[1] = 0;
  __syncthreads();
  for (int base = 0; base < t.ntiles; base += 1024) {
    const int i = base + threadIdx.x;
    const int c = i < t.ntiles ? t.count[i] : 0;
    sc[threadIdx.x] = c;
    so[threadIdx.x] = c > 0 ? 1 : 0;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // Hillis-Steele inclusive scans
      const int a = threadIdx.x >= off ? sc[threadIdx.x - off] : 0;
      const int b = threadIdx.x >= off ? so[threadIdx.x - off] : 0;
      __syncthreads();
      sc[threadIdx.x] += a;
      so[threadIdx.x] += b;
      __syncthreads();
    }
    if (i < t.ntiles) {
      const int start = carry[0] + sc[threadIdx.x] - c;
      t.start[i] = start;
      t.cursor[i] = start;
      if (c > 0) t.occ[carry[1] + so[threadIdx.x] - 1] = i;
    }
    __syncthreads();
    if (threadIdx.x == 1023) {
      carry[0] += sc[1023];
      carry[1] += so[1023];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    t.start[t.ntiles] = carry[0];
    t.nocc[0] = carry[1];
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

// Stencil of a marker in region slots; false if any node falls outside.
template <int K>
__device__ __forceinline__ bool stencil_in_region(const Region& r, const double X[3], int j0[3],
                                                  double w[3][4]) {
  bool ok = true;
  for (int a = 0; a < 3; ++a) {
    const int j = stencil(K, X[a], w[a]);
    j0[a] = j - r.o[a];
    ok = ok && j0[a] >= 0 && j0[a] + K <= kReg;
  }
  return ok;
}

// ------------------------------------------------------- direct fallbacks
template <int S, int K>
__device__ void direct_interp(const SiteArgs& s, const double X[3], bool phys, double& rp,
                              double up[3]) {
  double w[3][4];
  int j0[3];
  for (int a = 0; a < 3; ++a) j0[a] = stencil(K, X[a], w[a]);
  rp = 0;
  up[0] = up[1] = up[2] = 0;
  for (int kz = 0; kz < K; ++kz)
    for (int ky = 0; ky < K; ++ky) {
      int yy = j0[1] + ky;
      if (s.g.wall) {
        if (yy < 0 || yy >= s.g.ny) continue;
      } else {
        yy = wrap_idx(yy, s.g.ny);
      }
      for (int kx = 0; kx < K; ++kx) {
        const double W = w[0][kx] * w[1][ky] * w[2][kz];
        if (W == 0.0) continue;
        double fl[Q], drho, j[3];
        site_phys<S>(s, wrap_idx(j0[0] + kx, s.g.nx), yy, wrap_idx(j0[2] + kz, s.g.nz), fl, drho,
                     j, phys);
        const double rr = s.rho0 + drho;
        rp += W * rr;
        for (int a = 0; a < 3; ++a) up[a] += W * j[a] / rr;
      }
    }
}

template <typename E, int K>
__device__ void direct_spread(const TileArgs& t, const double X[3], const double F[3], E* Fd) {
  double w[3][4];
  int j0[3];
  for (int a = 0; a < 3; ++a) j0[a] = stencil(K, X[a], w[a]);
  for (int kz = 0; kz < K; ++kz)
    for (int ky = 0; ky < K; ++ky) {
      int yy = j0[1] + ky;
      if (t.g.wall) {
        if (yy < 0 || yy >= t.g.ny) continue;
      } else {
        yy = wrap_idx(yy, t.g.ny);
      }
      for (int kx = 0; kx < K; ++kx) {
        const double W = w[0][kx] * w[1][ky] * w[2][kz];
        if (W == 0.0) continue;
        const int xx = wrap_idx(j0[0] + kx, t.g.nx), zz = wrap_idx(j0[2] + kz, t.g.nz);
        const long long sidx = site_index(t.g, xx, yy, zz);
        for (int a = 0; a < 3; ++a) unsafeAtomicAdd(Fd + 4 * sidx + a, (E)(W * F[a]));
        uint64_t bit;
        uint64_t* mw = mask_word(t.mask, t.g, xx, yy, zz, bit);
        atomicOr((unsigned long long*)mw, bit);
      }
    }
}

// ------------------------------------------------------------- interpolation
// mode 0: IB predictor       aux = wrap(pos + h/2 u(pos))
// mode 1: IB advection       pos = wrap(pos + h/2 u(aux))
// mode 2: both, in that order, from one staged region (at = pos); the first
//         advection only needs the state before the lattice pass, like the
//         predictor, so both read the same LDS moments.
template <int S, int K>
__global__ __launch_bounds__(256) void k_tile_interp(TileArgs t, SiteArgs s, const double* at,
                                                     double* pos, double* aux, int mode) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double4* mom = (double4*)lds_raw;  // kRegSites
  if ((int)blockIdx.x >= t.nocc[0]) return;
  const int tl = t.occ[blockIdx.x];
  const Region r = region_of(t, tl);
  for (int k = threadIdx.x; k < kRegSites; k += blockDim.x) {
    const int ix = k % kReg, iy = (k / kReg) % kReg, iz = k / (kReg * kReg);
    int x, y, z;
    double4 m = make_double4(0, 0, 0, 0);
    if (slot_site(s.g, r, ix, iy, iz, x, y, z)) {
      double fl[Q], drho, j[3];
      site_phys<S>(s, x, y, z, fl, drho, j, true);
      const double rr = s.rho0 + drho;
      m = make_double4(rr, j[0] / rr, j[1] / rr, j[2] / rr);
    }
    mom[k] = m;
  }
  __syncthreads();
  const int b0 = t.start[tl], b1 = t.start[tl + 1];
  auto interp_at = [&](const double X[3], double up[3]) {
    double w[3][4];
    int j0[3];
    double rp = 0;
    up[0] = up[1] = up[2] = 0;
    if (stencil_in_region<K>(r, X, j0, w)) {
      for (int kz = 0; kz < K; ++kz)
        for (int ky = 0; ky < K; ++ky)
          for (int kx = 0; kx < K; ++kx) {
            const double W = w[0][kx] * w[1][ky] * w[2][kz];
            if (W == 0.0) continue;
            const double4 m = mom[((j0[2] + kz) * kReg + (j0[1] + ky)) * kReg + (j0[0] + kx)];
            if (m.x == 0.0) continue;  // beyond a wall
            rp += W * m.x;
            up[0] += W * m.y;
            up[1] += W * m.z;
            up[2] += W * m.w;
          }
    } else {
      direct_interp<S, K>(s, X, true, rp, up);
    }
  };
  auto half_drift = [&](const double from[3], const double u[3], double to[3]) {
    for (int a = 0; a < 3; ++a) to[a] = from[a] + 0.5 * u[a];
    to[0] = wrap_pos(to[0], (double)s.g.nx);
    if (!s.g.wall) to[1] = wrap_pos(to[1], (double)s.g.ny);
    to[2] = wrap_pos(to[2], (double)s.g.nz);
  };
  for (int q = b0 + threadIdx.x; q < b1; q += blockDim.x) {
    const long long p = t.sorted[q];
    const double X[3] = {at[3 * p], at[3 * p + 1], at[3 * p + 2]};
    double up[3], Y[3];
    interp_at(X, up);
    if (mode == 0) {  // predictor only
      half_drift(X, up, Y);
      for (int a = 0; a < 3; ++a) aux[3 * p + a] = Y[a];
    } else if (mode == 1) {  // advection with the velocity at X~ = at
      const double P[3] = {pos[3 * p], pos[3 * p + 1], pos[3 * p + 2]};
      half_drift(P, up, Y);
      for (int a = 0; a < 3; ++a) pos[3 * p + a] = Y[a];
    } else {  // mode 2: predictor, then the first advection from the same staged state
      double Xt[3], u2[3];
      half_drift(X, up, Xt);
      for (int a = 0; a < 3; ++a) aux[3 * p + a] = Xt[a];
      interp_at(Xt, u2);
      half_drift(X, u2, Y);
      for (int a = 0; a < 3; ++a) pos[3 * p + a] = Y[a];
    }
  }
}

// ------------------------------------------------------------------ spreading
template <typename E, int K>
__global__ __launch_bounds__(256) void k_tile_spread(TileArgs t, const double* at, const double* F,
                                                     void* field) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  E* acc = (E*)lds_raw;  // 3 * kRegSites
  if ((int)blockIdx.x >= t.nocc[0]) return;
  const int tl = t.occ[blockIdx.x];
  const Region r = region_of(t, tl);
  for (int k = threadIdx.x; k < 3 * kRegSites; k += blockDim.x) acc[k] = E(0);
  __syncthreads();
  E* Fd = (E*)field;
  const int b0 = t.start[tl], b1 = t.start[tl + 1];
  for (int q = b0 + threadIdx.x; q < b1; q += blockDim.x) {
    const long long p = t.sorted[q];
    const double X[3] = {at[3 * p], at[3 * p + 1], at[3 * p + 2]};
    const double f[3] = {F[3 * p], F[3 * p + 1], F[3 * p + 2]};
    double w[3][4];
    int j0[3];
    if (stencil_in_region<K>(r, X, j0, w)) {
      for (int kz = 0; kz < K; ++kz)
        for (int ky = 0; ky < K; ++ky) {
          const int yabs = r.o[1] + j0[1] + ky;
          if (t.g.wall && (yabs < 0 || yabs >= t.g.ny)) continue;
          for (int kx = 0; kx < K; ++kx) {
            const double W = w[0][kx] * w[1][ky] * w[2][kz];
            if (W == 0.0) continue;
            E* a = acc + 3 * (((j0[2] + kz) * kReg + (j0[1] + ky)) * kReg + (j0[0] + kx));
            atomicAdd(a + 0, (E)(W * f[0]));
            atomicAdd(a + 1, (E)(W * f[1]));
            atomicAdd(a + 2, (E)(W * f[2]));
          }
        }
    } else {
      direct_spread<E, K>(t, X, f, Fd);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kRegSites; k += blockDim.x) {
    const E a0 = acc[3 * k], a1 = acc[3 * k + 1], a2 = acc[3 * k + 2];
    if (a0 == E(0) && a1 == E(0) && a2 == E(0)) continue;
    const int ix = k % kReg, iy = (k / kReg) % kReg, iz = k / (kReg * kReg);
    int x, y, z;
    if (!slot_site(t.g, r, ix, iy, iz, x, y, z)) continue;
    const long long sidx = site_index(t.g, x, y, z);
    unsafeAtomicAdd(Fd + 4 * sidx + 0, a0);
    unsafeAtomicAdd(Fd + 4 * sidx + 1, a1);
    unsafeAtomicAdd(Fd + 4 * sidx + 2, a2);
    uint64_t bit;
    uint64_t* mw = mask_word(t.mask, t.g, x, y, z, bit);
    if (!(__atomic_load_n(mw, __ATOMIC_RELAXED) & bit)) atomicOr((unsigned long long*)mw, bit);
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

static unsigned tile_grid(const TileArgs& t, long long n) {
  return (unsigned)(n < t.ntiles ? n : t.ntiles);
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
  const size_t lds = sizeof(double4) * kRegSites;
  LBC_TILE_K_SWITCH(K, LBC_TILE_S_SWITCH(storage, (k_tile_interp<SS, KK>
      <<<tile_grid(t, n), 256, lds, st>>>(t, s, at, pos, aux, mode))));
  return hipGetLastError();
}

hipError_t launch_tile_spread(int storage, int K, const TileArgs& t, const double* at,
                              const double* F, void* field, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (storage == LB_F64) {
    const size_t lds = sizeof(double) * 3 * kRegSites;
    LBC_TILE_K_SWITCH(K, (k_tile_spread<double, KK><<<tile_grid(t, n), 256, lds, st>>>(t, at, F, field)));
  } else {
    const size_t lds = sizeof(float) * 3 * kRegSites;
    LBC_TILE_K_SWITCH(K, (k_tile_spread<float, KK><<<tile_grid(t, n), 256, lds, st>>>(t, at, F, field)));
  }
  return hipGetLastError();
}

}  // namespace lbc
