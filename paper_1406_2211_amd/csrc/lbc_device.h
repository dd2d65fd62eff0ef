// lbc_device.h -- device-side building blocks of the gfx950 lattice Boltzmann
// library: the D3Q19 velocity set in library order, storage traits for the
// population precisions, the pull gather used by every kernel that needs the
// post-stream populations, and small FP64 helpers for the particle side.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbc.h"
#include "lbc_internal.h"

namespace lbc {

// D3Q19 with opposite directions adjacent: i and i+1 are opposites for odd i,
// so the two-rate collision works on the pairs (1,2), (3,4), ..., (17,18).
constexpr int Q = 19;
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
// weights: rest 1/3, faces 1/18, edges 1/36
constexpr int WCLASS[Q] = {0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2};

template <typename R>
__device__ __forceinline__ R wgt(int i) {
  return WCLASS[i] == 0 ? R(1) / R(3) : (WCLASS[i] == 1 ? R(1) / R(18) : R(1) / R(36));
}

// ------------------------------------------------------------ random numbers
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds, each
// multiplying words 0 and 2 by the published constants (full 64-bit products)
// and mixing the halves with words 1 and 3 and the key, which advances by the
// published Weyl increments between rounds.
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
    // three-input exclusive or in one instruction (truth table 0x96)
    c = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96), (uint32_t)p1,
                   __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96),
                   (uint32_t)p0);
  }
  return c;
}

// Uniform in (0, 1) from the top 23 bits, u = (x / 2^9 + 1/2) / 2^23: 24
// significant bits, exact in FP32 and FP64 (a 24-bit version would need 25
// and round in FP32 for half of the values, which moves u near 1 and with it
// the small radii sqrt(-2 ln u) of the transform), and four
// normal deviates by the Box-Muller transform of the pairs (x, y), (z, w):
// r = sqrt(-2 ln u1), (r cos 2 pi u2, r sin 2 pi u2).  FP64 uses the library
// functions (the angle through sincospi, an exact argument reduction).  FP32
// uses the hardware transcendentals: log2, square root, and sine and cosine
// of a whole number of revolutions (u2 in (0, 1)), each within a few ulp.
template <typename R>
__device__ __forceinline__ R unit23(uint32_t x) {
  return (R(x >> 9) + R(0.5)) * R(1.1920928955078125e-07);  // 2^-23
}

__device__ __forceinline__ void box_muller(float u1, float u2, float& a, float& b) {
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
  a = r * __builtin_amdgcn_cosf(u2);
  b = r * __builtin_amdgcn_sinf(u2);
}
__device__ __forceinline__ void box_muller(double u1, double u2, double& a, double& b) {
  const double r = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  a = r * cs;
  b = r * sn;
}

template <typename R>
__device__ __forceinline__ void normals4(uint4 b, R g[4]) {
  box_muller(unit23<R>(b.x), unit23<R>(b.y), g[0], g[1]);
  box_muller(unit23<R>(b.z), unit23<R>(b.w), g[2], g[3]);
}

// Deviate index of velocity c_i: its rank in increasing 9(cx+1) + 3(cy+1) + (cz+1).
struct VelRank {
  int r[Q];
  constexpr VelRank() : r() {
    for (int i = 0; i < Q; ++i) {
      int n = 0;
      for (int j = 0; j < Q; ++j)
        n += (9 * (CX[j] + 1) + 3 * (CY[j] + 1) + CZ[j] + 1) <
             (9 * (CX[i] + 1) + 3 * (CY[i] + 1) + CZ[i] + 1);
      r[i] = n;
    }
  }
};
constexpr VelRank kVelRank{};

// Storage reference in the comoving frame: e_i(U) = f^eq_i(rho0, U) - w_i rho0
// (zero density deviation); stored value = f - w rho0 - e_i(U_ref).
template <typename R>
__device__ __forceinline__ R eref(int i, R rho0, R ux, R uy, R uz) {
  const R cu = R(CX[i]) * ux + R(CY[i]) * uy + R(CZ[i]) * uz;
  return wgt<R>(i) * rho0 * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * (ux * ux + uy * uy + uz * uz));
}

// ------------------------------------------------------------------ storage
template <int S>
struct Store;
template <>
struct Store<LB_F64> {
  using T = double;
  using R = double;
  using V4 = double4;
  static __device__ __forceinline__ R ld(const T* p, R) { return *p; }
  static __device__ __forceinline__ R raw(const T* p) { return *p; }
  // non-temporal load (the row-mapped pass reads each population once)
  static __device__ __forceinline__ R raw_nt(const T* p) { return __builtin_nontemporal_load(p); }
  // populations are written once per pass and not re-read by it: non-temporal
  static __device__ __forceinline__ void st(T* p, R v, R) { __builtin_nontemporal_store(v, p); }
  static __device__ __forceinline__ void st_raw(T* p, R v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Store<LB_F32> {
  using T = float;
  using R = float;
  using V4 = float4;
  static __device__ __forceinline__ R ld(const T* p, R) { return *p; }
  static __device__ __forceinline__ R raw(const T* p) { return *p; }
  static __device__ __forceinline__ R raw_nt(const T* p) { return __builtin_nontemporal_load(p); }
  static __device__ __forceinline__ void st(T* p, R v, R) { __builtin_nontemporal_store(v, p); }
  static __device__ __forceinline__ void st_raw(T* p, R v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Store<LB_F16> {
  using T = __half;
  using R = float;
  using V4 = float4;
  // stored value is scale * (f - w rho0); inv is 1/scale (a power of two)
  static __device__ __forceinline__ R ld(const T* p, R inv) { return __half2float(*p) * inv; }
  static __device__ __forceinline__ R raw(const T* p) { return __half2float(*p); }
  static __device__ __forceinline__ R raw_nt(const T* p) {
    return __half2float(__ushort_as_half(__builtin_nontemporal_load((const unsigned short*)p)));
  }
  static __device__ __forceinline__ void st(T* p, R v, R scale) { st_raw(p, v * scale); }
  static __device__ __forceinline__ void st_raw(T* p, R v) {
    __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(v)), (unsigned short*)p);
  }
};
template <>
struct Store<LB_BF16> {
  using T = __hip_bfloat16;
  using R = float;
  using V4 = float4;
  static __device__ __forceinline__ R ld(const T* p, R inv) { return __bfloat162float(*p) * inv; }
  static __device__ __forceinline__ R raw(const T* p) { return __bfloat162float(*p); }
  static __device__ __forceinline__ R raw_nt(const T* p) {
    // bf16 is the top half of an FP32 word
    return __uint_as_float((uint32_t)__builtin_nontemporal_load((const unsigned short*)p) << 16);
  }
  static __device__ __forceinline__ void st(T* p, R v, R scale) { st_raw(p, v * scale); }
  static __device__ __forceinline__ void st_raw(T* p, R v) {
    const __hip_bfloat16 b = __float2bfloat16(v);
    __builtin_nontemporal_store(*(const unsigned short*)&b, (unsigned short*)p);
  }
};

__device__ __forceinline__ long long site_index(const Geo& g, int x, int y, int z) {
  return ((long long)z * g.ny + y) * g.nx + x;
}

// Force-mask word and bit of a site.  Boxes whose x extent is a multiple of
// 64 keep one word per 64 x-sites of a row (wpr words per row, so a
// row-aligned wavefront owns its word); other boxes and ensemble slots
// (wpr == 0) use one word per 64 consecutive linear site indices.
//
// A set bit means: the lattice pass reads (and zeroes) FA and FB at this
// site.  Bits persist across steps and are cleared by the lattice pass only
// every kMaskKeep steps, so a particle that keeps touching the same sites
// finds its bits set and spreads without an atomic on the mask; a bit that
// is no longer needed costs the pass one read of zeros until the next clear.
// (The immersed-boundary pass instead rewrites each word to the sites of its
// pending field, see take_forces.)
constexpr int kMaskKeep = 32;

__device__ __forceinline__ uint64_t* mask_word(uint64_t* m, const Geo& g, int x, int y, int z,
                                               uint64_t& bit) {
  if (g.wpr == 0) {
    const long long s = site_index(g, x, y, z);
    bit = 1ull << (s & 63);
    return m + (s >> 6);
  }
  bit = 1ull << (x & 63);
  return m + ((long long)z * g.ny + y) * g.wpr + (x >> 6);
}

// Flag a site for the next lattice pass (after its force was added): a plain
// load first, since in steady state the bit is usually set already.  The load
// goes through the caches (an atomic load of device or system scope would
// bypass them and take a memory round trip per site): bits are only set while
// a kernel flags sites and cleared by the lattice pass, a kernel boundary
// away, so a cached copy can at worst lack a bit set meanwhile by another
// workgroup, which costs one redundant atomic.
__device__ __forceinline__ void flag_site(uint64_t* mw, uint64_t bit) {
  if (!(*mw & bit)) atomicOr((unsigned long long*)mw, bit);
}

// Quotient and remainder of n / d for 32-bit n and d >= 1, with rd = 1/d
// (double, rounded) from the host: n * rd is within 1e-6 of n / d, so its
// truncation is the quotient or one off, and one correction step fixes it.
__device__ __forceinline__ uint32_t div_rem(uint32_t n, uint32_t d, double rd, uint32_t& rem) {
  uint32_t q = (uint32_t)((double)n * rd);
  long long r = (long long)n - (long long)q * d;
  if (r < 0) {
    q -= 1;
    r += d;
  } else if (r >= (long long)d) {
    q += 1;
    r -= d;
  }
  rem = (uint32_t)r;
  return q;
}

// Pull gather: fbar_i(x) = f*_i(x - c_i), periodic, or the reflected opposite
// population of the same site when x - c_i lies beyond a y wall (halfway
// bounce-back).  Values are converted to the compute type R.
template <int S, typename R>
__device__ __forceinline__ void pull(const typename Store<S>::T* __restrict__ f, const Geo& g,
                                     int x, int y, int z, R inv, R out[Q]) {
  const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
  const long long own = site_index(g, x, y, z);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    long long src;
    const bool bb = g.wall && ((CY[i] == 1 && y == 0) || (CY[i] == -1 && y == g.ny - 1));
    if (bb) {
      src = (long long)OPP[i] * g.ps + own;
    } else {
      const int xs = CX[i] == 1 ? xm : (CX[i] == -1 ? xp : x);
      const int ys = CY[i] == 1 ? ym : (CY[i] == -1 ? yp : y);
      const int zs = CZ[i] == 1 ? zm : (CZ[i] == -1 ? zp : z);
      src = (long long)i * g.ps + site_index(g, xs, ys, zs);
    }
    out[i] = Store<S>::ld(f + src, inv);
  }
}

// The pending half force of site s added to its momentum: rho u = sum f c +
// (h/2)(FB + pend F_ext) (the redefined velocity of Sec. 4).
template <int S>
__device__ __forceinline__ void add_pending(const SiteArgs& a, long long s, double j[3]) {
  using V4 = typename Store<S>::V4;
  const V4 fb = ((const V4*)a.FB)[s];
  j[0] += 0.5 * ((double)fb.x + a.pfx);
  j[1] += 0.5 * ((double)fb.y + a.pfy);
  j[2] += 0.5 * ((double)fb.z + a.pfz);
}

// (h/2) of a pending force field added to the momentum at site s.
template <int S>
__device__ __forceinline__ void add_field(const void* field, long long s, double j[3]) {
  using V4 = typename Store<S>::V4;
  const V4 f = ((const V4*)field)[s];
  j[0] += 0.5 * (double)f.x;
  j[1] += 0.5 * (double)f.y;
  j[2] += 0.5 * (double)f.z;
}

// Physical moments at one site: rho and rho u = sum f c + (h/2)(FB + pend F_ext)
// (the redefined velocity of Sec. 4).
template <int S>
__device__ __forceinline__ void site_phys(const SiteArgs& a, int x, int y, int z, double fl[Q],
                                          double& drho, double j[3], bool phys) {
  using St = Store<S>;
  pull<S, double>((const typename St::T*)a.f, a.g, x, y, z, (double)a.inv, fl);
  if (a.uref[0] != 0.0 || a.uref[1] != 0.0 || a.uref[2] != 0.0) {
#pragma unroll
    for (int i = 0; i < Q; ++i) fl[i] += eref<double>(i, a.rho0, a.uref[0], a.uref[1], a.uref[2]);
  }
  drho = 0;
  j[0] = j[1] = j[2] = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += fl[i];
    j[0] += CX[i] * fl[i];
    j[1] += CY[i] * fl[i];
    j[2] += CZ[i] * fl[i];
  }
  if (phys) add_pending<S>(a, site_index(a.g, x, y, z), j);
}

// Physical moments at one site in the compute type R, for kernels that stage
// many sites and round the moments to R anyway (R = float for FP32 and 16-bit
// storage keeps the 19 gathered values in half the registers).
template <int S, typename R>
__device__ __forceinline__ void site_phys_r(const SiteArgs& a, int x, int y, int z, R& drho,
                                            R j[3]) {
  using St = Store<S>;
  using V4 = typename St::V4;
  R fl[Q];
  pull<S, R>((const typename St::T*)a.f, a.g, x, y, z, (R)a.inv, fl);
  if (a.uref[0] != 0.0 || a.uref[1] != 0.0 || a.uref[2] != 0.0) {
#pragma unroll
    for (int i = 0; i < Q; ++i)
      fl[i] += eref<R>(i, (R)a.rho0, (R)a.uref[0], (R)a.uref[1], (R)a.uref[2]);
  }
  drho = 0;
  j[0] = j[1] = j[2] = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += fl[i];
    if (CX[i]) j[0] += R(CX[i]) * fl[i];
    if (CY[i]) j[1] += R(CY[i]) * fl[i];
    if (CZ[i]) j[2] += R(CZ[i]) * fl[i];
  }
  const V4 fb = ((const V4*)a.FB)[site_index(a.g, x, y, z)];
  j[0] += R(0.5) * ((R)fb.x + (R)a.pfx);
  j[1] += R(0.5) * ((R)fb.y + (R)a.pfy);
  j[2] += R(0.5) * ((R)fb.z + (R)a.pfz);
}

// site_phys_r with the populations loaded one after another (a rolled loop):
// the same operations in the same order, for a rarely taken path whose 19
// loads in flight would otherwise set the register budget of a whole kernel.
template <int S, typename R>
__device__ __forceinline__ void site_phys_r_seq(const SiteArgs& a, int x, int y, int z, R& drho,
                                                R j[3]) {
  using St = Store<S>;
  using V4 = typename St::V4;
  const typename St::T* __restrict__ f = (const typename St::T*)a.f;
  const Geo& g = a.g;
  const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
  const long long own = site_index(g, x, y, z);
  const bool ref = a.uref[0] != 0.0 || a.uref[1] != 0.0 || a.uref[2] != 0.0;
  drho = 0;
  j[0] = j[1] = j[2] = 0;
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    long long src;
    const bool bb = g.wall && ((CY[i] == 1 && y == 0) || (CY[i] == -1 && y == g.ny - 1));
    if (bb) {
      src = (long long)OPP[i] * g.ps + own;
    } else {
      const int xs = CX[i] == 1 ? xm : (CX[i] == -1 ? xp : x);
      const int ys = CY[i] == 1 ? ym : (CY[i] == -1 ? yp : y);
      const int zs = CZ[i] == 1 ? zm : (CZ[i] == -1 ? zp : z);
      src = (long long)i * g.ps + site_index(g, xs, ys, zs);
    }
    R fl = St::ld(f + src, (R)a.inv);
    if (ref) fl += eref<R>(i, (R)a.rho0, (R)a.uref[0], (R)a.uref[1], (R)a.uref[2]);
    drho += fl;
    if (CX[i]) j[0] += R(CX[i]) * fl;
    if (CY[i]) j[1] += R(CY[i]) * fl;
    if (CZ[i]) j[2] += R(CZ[i]) * fl;
  }
  const V4 fb = ((const V4*)a.FB)[own];
  j[0] += R(0.5) * ((R)fb.x + (R)a.pfx);
  j[1] += R(0.5) * ((R)fb.y + (R)a.pfy);
  j[2] += R(0.5) * ((R)fb.z + (R)a.pfz);
}

// deviation equilibrium f^eq_i(rho,u) - w_i rho0 = w_i [drho + rho P_i(u)],
// P_i(u) = 3 c.u + 9/2 (c.u)^2 - 3/2 u.u
template <typename R>
__device__ __forceinline__ R feq_dev(int i, R drho, R rho, R ux, R uy, R uz, R usq) {
  const R cu = R(CX[i]) * ux + R(CY[i]) * uy + R(CZ[i]) * uz;
  return wgt<R>(i) * (drho + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq));
}

// Constants of one fused lattice pass in the compute type.  Storage units:
// the stored value of population i is S (f_i - w_i rho0 - e_i(U)), with S the
// 16-bit scale (1 otherwise) and e_i(U) the comoving reference of the buffer
// (zero unless the comoving frame is on).
template <typename R>
struct PassK {
  R rho0, sc, inv;  // rho0, S, 1/S
  R hp, hm;         // (1 - lambda+)/2 and (1 - lambda-)/2
  R ui[3];          // reference velocity of the input buffer (comoving frame)
  const R* cm;      // comoving reference terms per pair, see comoving_terms
  // fluctuating collision: S sqrt(mu lambda (2 - lambda)) for the even / odd
  // moments, the generator key and the step index
  R ap, am;
  uint32_t k0, k1, t0, t1;
  // general MRT: rate of each moment group (bulk, shear, vector ghosts,
  // pseudo-vector ghosts, scalar ghost, tensor ghosts) and, with noise, the
  // amplitude S sqrt(mu lambda (2 - lambda)) of each group
  R lg[6], ag[6];
};

// Thermal noise of the fluctuating collision (Eq. mrt-fluct) at one site, in
// population form and storage units.  With g_i the site's normal deviates
// (five Philox blocks with counter (site, step low, block, step high)),
// z_i = sqrt(w_i) g_i has every moment m_k(z) / sqrt(b_k) standard normal and
// independent; removing its density and momentum,
//   zc_i = z_i - w_i (m0(z) + 3 c_i . j(z)),
// and scaling the parts even and odd over opposite pairs by
// sqrt(rho mu lambda+- (2 - lambda+-)) adds to each non-conserved moment
// sqrt(rho) phi_k r_k with phi_k = sqrt(mu b_k lambda_k (2 - lambda_k)), the
// amplitude that keeps its variance at the equilibrium mu rho b_k.
template <typename R>
__device__ __forceinline__ void site_noise(const PassK<R>& k, uint32_t site, R rho, R n[Q]) {
  R g[20];
#pragma unroll
  for (int b = 0; b < 5; ++b) normals4<R>(philox(make_uint4(site, k.t0, b, k.t1), k.k0, k.k1), g + 4 * b);
  const R s0 = sqrt(R(1) / R(3)), s1 = sqrt(R(1) / R(18)), s2 = sqrt(R(1) / R(36));
  R z[Q], m0 = 0, mx = 0, my = 0, mz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    z[i] = (WCLASS[i] == 0 ? s0 : (WCLASS[i] == 1 ? s1 : s2)) * g[kVelRank.r[i]];
    m0 += z[i];
    if (CX[i]) mx += R(CX[i]) * z[i];
    if (CY[i]) my += R(CY[i]) * z[i];
    if (CZ[i]) mz += R(CZ[i]) * z[i];
  }
  const R sr = sqrt(rho);
  const R ep = sr * k.ap, om = sr * k.am;
  n[0] = ep * (z[0] - wgt<R>(0) * m0);
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    const R w = wgt<R>(i);
    const R cm = R(3) * (R(CX[i]) * mx + R(CY[i]) * my + R(CZ[i]) * mz);
    const R a = z[i] - w * (m0 + cm), b = z[i + 1] - w * (m0 - cm);
    const R e = R(0.5) * (a + b), o = R(0.5) * (a - b);
    n[i] = ep * e + om * o;
    n[i + 1] = ep * e - om * o;
  }
}

// Comoving frame: the reference parts of the storage-unit equilibria, the same
// for every site of a box in one pass.  Pair p = 1..9 is (2p-1, 2p), p = 0 the
// rest population; with B0 = w S rho0, U_in/U_out the references of the input
// and output buffers:
//   cm[0*10+p] = B0 (9/2 (c.U_in)^2 - 3/2 U_in.U_in)    (even, input)
//   cm[1*10+p] = 3 B0 (c.U_in)                         (odd, input)
//   cm[2*10+p], cm[3*10+p]: the same with U_out          (output)
// They are subtracted from the equilibria formed in fused_site.
__host__ __device__ inline void comoving_terms(double S, double rho0, const double ui[3],
                                               const double uo[3], double cm[40], float cmf[40]) {
  const double isq = ui[0] * ui[0] + ui[1] * ui[1] + ui[2] * ui[2];
  const double osq = uo[0] * uo[0] + uo[1] * uo[1] + uo[2] * uo[2];
  const double w0 = 1.0 / 3.0;
  cm[0] = w0 * S * rho0 * (-1.5 * isq);
  cm[10] = 0.0;
  cm[20] = w0 * S * rho0 * (-1.5 * osq);
  cm[30] = 0.0;
  for (int p = 1; p <= 9; ++p) {
    const int i = 2 * p - 1;
    const double w = WCLASS[i] == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
    const double B0 = w * S * rho0;
    const double ci = CX[i] * ui[0] + CY[i] * ui[1] + CZ[i] * ui[2];
    const double co = CX[i] * uo[0] + CY[i] * uo[1] + CZ[i] * uo[2];
    cm[p] = B0 * (4.5 * ci * ci - 1.5 * isq);
    cm[10 + p] = 3.0 * B0 * ci;
    cm[20 + p] = B0 * (4.5 * co * co - 1.5 * osq);
    cm[30 + p] = 3.0 * B0 * co;
  }
  for (int q = 0; q < 40; ++q) cmf[q] = (float)cm[q];
}

template <typename R>
__host__ __device__ inline const R* pick_terms(const double* cm, const float* cmf);
template <>
__host__ __device__ inline const double* pick_terms<double>(const double* cm, const float*) {
  return cm;
}
template <>
__host__ __device__ inline const float* pick_terms<float>(const double*, const float* cmf) {
  return cmf;
}

// One site of the fused pass: both pending half forces as one equilibrium
// shift, then the collision, then the store.  f: the pulled (post-stream)
// populations in storage units; F: the total pending force (both halves).
//   f*_i = f^eq_i(rho, u + F/2rho) + (1 - lambda+) (f - f^eq(rho, u))^even_i
//                                  + (1 - lambda-) (f - f^eq(rho, u))^odd_i
// with even/odd parts taken over the opposite pairs (1,2), (3,4), ...; BGK is
// the case lambda- = lambda+.  All equilibria are formed directly in storage
// units, split into the parts even and odd in c: with A = w S drho,
// B = w S rho, B0 = w S rho0,
//   even: A + B (9/2 (c.u)^2 - 3/2 u.u) - B0 (9/2 (c.U)^2 - 3/2 U.U)
//   odd:  3 B (c.u) - 3 B0 (c.U)
// so neither the loads nor the stores need the scale; the U terms are
// per-pass constants (comoving_terms).
// With NS the thermal noise of site_noise is added to every stored value.
template <int S, bool CM, bool NS = false, bool SG = false>
__device__ __forceinline__ void fused_site(const typename Store<S>::R f[Q], typename Store<S>::R Fx,
                                           typename Store<S>::R Fy, typename Store<S>::R Fz,
                                           const PassK<typename Store<S>::R>& k,
                                           typename Store<S>::T* __restrict__ fo, size_t P,
                                           size_t own,
                                           typename Store<S>::R* __restrict__ sgo = nullptr,
                                           size_t sN = 0, typename Store<S>::R sp = 0) {
  using St = Store<S>;
  using R = typename St::R;
  R d = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    d += f[i];
    if (CX[i]) jx += R(CX[i]) * f[i];
    if (CY[i]) jy += R(CY[i]) * f[i];
    if (CZ[i]) jz += R(CZ[i]) * f[i];
  }
  const R rho = k.rho0 + d * k.inv;  // the references carry no density
  const R ir = R(1) / rho;
  const R js = k.inv * ir;
  R ux = jx * js, uy = jy * js, uz = jz * js;
  if (CM) {  // sum_i c_i e_i(U) = rho0 U
    const R r0 = k.rho0 * ir;
    ux += r0 * k.ui[0];
    uy += r0 * k.ui[1];
    uz += r0 * k.ui[2];
  }
  const R hf = R(0.5) * ir;
  const R hx = ux + hf * Fx, hy = uy + hf * Fy, hz = uz + hf * Fz;
  const R usq = ux * ux + uy * uy + uz * uz, hsq = hx * hx + hy * hy + hz * hz;
  const R rs = rho * k.sc;
  R nz[Q];
  if (NS) site_noise<R>(k, (uint32_t)own, rho, nz);
  R pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;  // non-equilibrium stress (SG)
  {
    const R w = wgt<R>(0);
    R eb = w * (d - R(1.5) * rs * usq), eh = w * (d - R(1.5) * rs * hsq);
    if (CM) {
      eb -= k.cm[0];
      eh -= k.cm[20];
    }
    R v = eh + R(2) * k.hp * (f[0] - eb);
    if (NS) v += nz[0];
    St::st_raw(fo + own, v);
  }
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    const R w = wgt<R>(i);
    const R A = w * d, B = w * rs;
    const R cb = R(CX[i]) * ux + R(CY[i]) * uy + R(CZ[i]) * uz;
    const R ch = R(CX[i]) * hx + R(CY[i]) * hy + R(CZ[i]) * hz;
    R Eb = A + B * (R(4.5) * cb * cb - R(1.5) * usq), Ob = R(3) * B * cb;
    R Eh = A + B * (R(4.5) * ch * ch - R(1.5) * hsq), Oh = R(3) * B * ch;
    if (CM) {
      const int q = (i + 1) / 2;
      Eb -= k.cm[q];
      Ob -= k.cm[10 + q];
      Eh -= k.cm[20 + q];
      Oh -= k.cm[30 + q];
    }
    const R ni = f[i] - Eb - Ob, nj = f[i + 1] - Eb + Ob;
    const R sym = k.hp * (ni + nj), anti = k.hm * (ni - nj);
    R vi = Eh + Oh + sym + anti, vj = Eh - Oh + sym - anti;
    if (NS) {
      vi += nz[i];
      vj += nz[i + 1];
    }
    if (SG) {  // sum_i (f_i - f^eq_i) c_i c_i over the opposite pair (c_j = -c_i)
      const R s2 = ni + nj;
      if (CX[i]) pxx += s2;
      if (CY[i]) pyy += s2;
      if (CZ[i]) pzz += s2;
      if (CX[i] && CY[i]) pxy += R(CX[i] * CY[i]) * s2;
      if (CX[i] && CZ[i]) pxz += R(CX[i] * CZ[i]) * s2;
      if (CY[i] && CZ[i]) pyz += R(CY[i] * CZ[i]) * s2;
    }
    St::st_raw(fo + (size_t)i * P + own, vi);
    St::st_raw(fo + (size_t)(i + 1) * P + own, vj);
  }
  if (SG) {  // viscous stress of the state this pass started from (Eq. viscstress)
    const R pf = sp * k.inv;
    sgo[own] = pf * pxx;
    sgo[sN + own] = pf * pyy;
    sgo[2 * sN + own] = pf * pzz;
    sgo[3 * sN + own] = pf * pxy;
    sgo[4 * sN + own] = pf * pxz;
    sgo[5 * sN + own] = pf * pyz;
  }
}

// ------------------------------------------------------------- general MRT
// Moment rows of the general MRT collision (Eq. mrt-coll with a rate per
// moment group): the D3Q19 polynomials of Duenweg, Schiller and Ladd (2007),
// w-orthogonal, each group spanning a subspace the cubic symmetry leaves
// invariant.  Rows 0..3 (density, momentum) are conserved; row k >= 4 belongs
// to group mrt_group(k): 0 bulk, 1 shear, 2 vector ghosts, 3 pseudo-vector
// ghosts, 4 scalar ghost, 5 tensor ghosts.  Evaluated at compile time.
constexpr int mrt_row(int k, int i) {
  const int x = CX[i], y = CY[i], z = CZ[i], c2 = x * x + y * y + z * z;
  switch (k) {
    case 4: return c2 - 1;
    case 5: return 3 * x * x - c2;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return z * x;
    case 10: return x * (3 * c2 - 5);
    case 11: return y * (3 * c2 - 5);
    case 12: return z * (3 * c2 - 5);
    case 13: return x * (y * y - z * z);
    case 14: return y * (z * z - x * x);
    case 15: return z * (x * x - y * y);
    case 16: return 3 * c2 * c2 - 6 * c2 + 1;
    case 17: return (2 * c2 - 3) * (3 * x * x - c2);
    case 18: return (2 * c2 - 3) * (y * y - z * z);
  }
  return 0;
}
constexpr int mrt_group(int k) {
  return k == 4 ? 0 : (k <= 9 ? 1 : (k <= 12 ? 2 : (k <= 15 ? 3 : (k == 16 ? 4 : 5))));
}
constexpr bool mrt_odd(int k) { return k >= 10 && k <= 15; }
// 1 / b_k with b_k = sum_i w_i e_k(c_i)^2
constexpr double mrt_inv_b(int k) {
  double b = 0.0;
  for (int i = 0; i < Q; ++i) {
    const double w = WCLASS[i] == 0 ? 1.0 / 3.0 : (WCLASS[i] == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    b += w * mrt_row(k, i) * mrt_row(k, i);
  }
  return 1.0 / b;
}

// One site of the fused pass with the general MRT collision (no comoving
// frame):
//   f*_i = f^eq_i(rho, u + F/2rho) + n_i - w_i sum_k e_k(c_i) (lambda_k m_k - xi_k) / b_k
// with n = f - f^eq(rho, u), m_k = sum_i e_k(c_i) n_i over the non-conserved
// rows and, with NS, the thermal noise xi_k = sqrt(rho) S sqrt(mu lambda_k
// (2 - lambda_k)) m_k(z) of z_i = sqrt(w_i) g_i (Eq. mrt-fluct).  Sums run
// over the opposite pairs: even rows see n_i + n_j, odd rows n_i - n_j.  The
// row coefficients are compile-time integers, so only their nonzero terms
// are formed.
template <int S, bool NS>
__device__ __forceinline__ void fused_site_mrt(const typename Store<S>::R f[Q],
                                               typename Store<S>::R Fx, typename Store<S>::R Fy,
                                               typename Store<S>::R Fz,
                                               const PassK<typename Store<S>::R>& k,
                                               typename Store<S>::T* __restrict__ fo, size_t P,
                                               size_t own) {
  using St = Store<S>;
  using R = typename St::R;
  R d = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    d += f[i];
    if (CX[i]) jx += R(CX[i]) * f[i];
    if (CY[i]) jy += R(CY[i]) * f[i];
    if (CZ[i]) jz += R(CZ[i]) * f[i];
  }
  const R rho = k.rho0 + d * k.inv;
  const R ir = R(1) / rho;
  const R js = k.inv * ir;
  const R ux = jx * js, uy = jy * js, uz = jz * js;
  const R hf = R(0.5) * ir;
  const R hx = ux + hf * Fx, hy = uy + hf * Fy, hz = uz + hf * Fz;
  const R usq = ux * ux + uy * uy + uz * uz, hsq = hx * hx + hy * hy + hz * hz;
  const R rs = rho * k.sc;
  // equilibria (storage units) and non-equilibrium parts; pair p = (2p+1, 2p+2)
  R n0, eh0, Eh[9], Oh[9], nI[9], nJ[9], sp[9], ap[9];
  {
    const R w = wgt<R>(0);
    n0 = f[0] - w * (d - R(1.5) * rs * usq);
    eh0 = w * (d - R(1.5) * rs * hsq);
  }
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    const int i = 2 * p + 1;
    const R w = wgt<R>(i);
    const R A = w * d, B = w * rs;
    const R cb = R(CX[i]) * ux + R(CY[i]) * uy + R(CZ[i]) * uz;
    const R ch = R(CX[i]) * hx + R(CY[i]) * hy + R(CZ[i]) * hz;
    const R Eb = A + B * (R(4.5) * cb * cb - R(1.5) * usq), Ob = R(3) * B * cb;
    Eh[p] = A + B * (R(4.5) * ch * ch - R(1.5) * hsq);
    Oh[p] = R(3) * B * ch;
    nI[p] = f[i] - Eb - Ob;
    nJ[p] = f[i + 1] - Eb + Ob;
    sp[p] = nI[p] + nJ[p];
    ap[p] = nI[p] - nJ[p];
  }
  // noise moments m_k(z), z_i = sqrt(w_i) g_i, paired like n
  R zs[9], za[9], z0 = 0;
  if (NS) {
    R g[20];
#pragma unroll
    for (int b = 0; b < 5; ++b)
      normals4<R>(philox(make_uint4((uint32_t)own, k.t0, b, k.t1), k.k0, k.k1), g + 4 * b);
    const R s0 = sqrt(R(1) / R(3)), s1 = sqrt(R(1) / R(18)), s2 = sqrt(R(1) / R(36));
    z0 = s0 * g[kVelRank.r[0]];
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      const int i = 2 * p + 1;
      const R sw = WCLASS[i] == 1 ? s1 : s2;
      const R zi = sw * g[kVelRank.r[i]], zj = sw * g[kVelRank.r[i + 1]];
      zs[p] = zi + zj;
      za[p] = zi - zj;
    }
  }
  const R sr = NS ? sqrt(rho) : R(0);
  // relaxation amounts D_k = (lambda_k m_k - xi_k) / b_k
  R D[Q];
#pragma unroll
  for (int q = 4; q < Q; ++q) {
    R m = 0, mz = 0;
    if (!mrt_odd(q) && mrt_row(q, 0) != 0) {
      m += R(mrt_row(q, 0)) * n0;
      if (NS) mz += R(mrt_row(q, 0)) * z0;
    }
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      const int c = mrt_row(q, 2 * p + 1);
      if (c != 0) {
        m += R(c) * (mrt_odd(q) ? ap[p] : sp[p]);
        if (NS) mz += R(c) * (mrt_odd(q) ? za[p] : zs[p]);
      }
    }
    R v = k.lg[mrt_group(q)] * m;
    if (NS) v -= sr * k.ag[mrt_group(q)] * mz;
    D[q] = v * R(mrt_inv_b(q));
  }
  {
    R c = 0;
#pragma unroll
    for (int q = 4; q < Q; ++q)
      if (!mrt_odd(q) && mrt_row(q, 0) != 0) c += R(mrt_row(q, 0)) * D[q];
    St::st_raw(fo + own, eh0 + n0 - wgt<R>(0) * c);
  }
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    const int i = 2 * p + 1;
    R ce = 0, co = 0;
#pragma unroll
    for (int q = 4; q < Q; ++q) {
      const int c = mrt_row(q, i);
      if (c == 0) continue;
      if (mrt_odd(q))
        co += R(c) * D[q];
      else
        ce += R(c) * D[q];
    }
    const R w = wgt<R>(i);
    St::st_raw(fo + (size_t)i * P + own, Eh[p] + Oh[p] + nI[p] - w * (ce + co));
    St::st_raw(fo + (size_t)(i + 1) * P + own, Eh[p] - Oh[p] + nJ[p] - w * (ce - co));
  }
}

// ---------------------------------------------------------- delta functions
// One-dimensional weights of a delta-function stencil (Appendix A kernels).
// Returns the first node j0; weights for nodes j0 .. j0+K-1.
template <typename T>
__device__ __forceinline__ T phi_eval_t(int K, T r) {
  const T a = fabs(r);
  if (K == 2) return a < T(1) ? T(1) - a : T(0);
  if (K == 3) {
    if (a <= T(0.5)) return (T(1) + sqrt(T(1) - T(3) * r * r)) / T(3);
    if (a <= T(1.5)) return (T(5) - T(3) * a - sqrt(fmax(T(0), T(6) * a - T(2) - T(3) * r * r))) / T(6);
    return T(0);
  }
  if (a <= T(1)) return (T(3) - T(2) * a + sqrt(T(1) + T(4) * a - T(4) * r * r)) / T(8);
  if (a <= T(2)) return (T(5) - T(2) * a - sqrt(fmax(T(0), T(-7) + T(12) * a - T(4) * r * r))) / T(8);
  return T(0);
}

__device__ __forceinline__ double phi_eval(int K, double r) { return phi_eval_t<double>(K, r); }

// floor(X) as an int for any X: the argument is first clamped to [-2^30, 2^30]
// (a NaN becomes -2^30), so a non-finite or runaway position (an unstable run,
// an over-stretched FENE bond) still maps to an in-range integer that the
// periodic wrap or the wall test below can handle; its weights stay NaN.
__device__ __forceinline__ int safe_floor(double X) {
  return (int)floor(fmin(fmax(X, -1073741824.0), 1073741824.0));
}

// First node of the K-point stencil of X: nodes j0 .. j0+K-1.
template <int K>
__device__ __forceinline__ int first_node(double X) {
  return K == 3 ? safe_floor(X + 0.5) - 1 : (K == 2 ? safe_floor(X) : safe_floor(X) - 1);
}

__device__ __forceinline__ int stencil(int K, double X, double w[4]) {
  const int j0 = K == 3 ? safe_floor(X + 0.5) - 1 : (K == 2 ? safe_floor(X) : safe_floor(X) - 1);
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = k < K ? phi_eval(K, (double)(j0 + k) - X) : 0.0;
  return j0;
}

__device__ __forceinline__ int wrap_idx(int j, int n) {
  int r = j % n;
  return r < 0 ? r + n : r;
}

// x - L floor(x/L); for x in [-L, 2L) (every drift of less than a box length)
// the compare-and-add below performs the same single rounding operation.
__device__ __forceinline__ double wrap_pos(double x, double L) {
  if (x >= 0.0 && x < L) return x;
  if (x >= -L && x < 0.0) return x + L;
  if (x >= L && x < 2.0 * L) return x - L;
  return x - L * floor(x / L);
}

// ------------------------------------------------------------- reductions
// Lanes per particle for a K-point stencil: one lane per stencil node (K^3),
// rounded up to a power of two that divides the wavefront.
template <int K>
struct Lanes {
  static constexpr int L = K == 2 ? 8 : (K == 3 ? 32 : 64);
};

// Sum over an aligned group of L lanes (butterfly; every lane gets the sum).
template <int L, typename T>
__device__ __forceinline__ T group_sum_t(T v) {
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int L>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over an aligned group of G = 4 or 16 lanes with DPP moves (every lane
// gets the sum): pairs and quads by quad permutations, then the two quads of
// each 8-lane half by a half-row mirror and the two halves by a row mirror.
template <int ctrl>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xf, 0xf, false));
}
template <int ctrl>
__device__ __forceinline__ double dpp_add(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, ctrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), ctrl, 0xf, 0xf, false);
  return v + __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int G, typename T>
__device__ __forceinline__ T group_sum_dpp(T v) {
  static_assert(G == 4 || G == 16, "DPP group sums cover 4 or 16 lanes");
  v = dpp_add<0xB1>(v);  // quad_perm [1,0,3,2]
  v = dpp_add<0x4E>(v);  // quad_perm [2,3,0,1]
  if (G == 16) {
    v = dpp_add<0x141>(v);  // row_half_mirror
    v = dpp_add<0x140>(v);  // row_mirror
  }
  return v;
}

// Sum over the 64 lanes of a wavefront, every lane getting it: the DPP sum of
// each 16-lane row, then the four row sums read from lanes 0, 16, 32, 48.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v = group_sum_dpp<16, double>(v);
  auto lane_value = [&](int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  };
  return (lane_value(0) + lane_value(16)) + (lane_value(32) + lane_value(48));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Position of the n-th set bit (n < popcount) of v.
__device__ __forceinline__ int nth_set_bit(uint64_t v, int n) {
  int pos = 0;
#pragma unroll
  for (int half = 32; half > 0; half >>= 1) {
    const int c = __popcll(v & ((1ull << half) - 1ull));
    if (n >= c) {
      n -= c;
      v >>= half;
      pos += half;
    }
  }
  return pos;
}

// Each wavefront reads WORDS (at most 64) words of the force mask and hands
// their flagged sites out one per lane (a scan of the words' bit counts and a
// binary search in it); f(x, y, z) runs once for every flagged site, up to 64
// sites at a time per wavefront.  Few words per wavefront suit a densely
// flagged mask, 64 a sparse one.
constexpr int kFlagWords = 16;

template <int WORDS = kFlagWords, typename F>
__device__ __forceinline__ void for_flagged_sites(const Geo& g, const uint64_t* __restrict__ mask,
                                                  long long nwords, F&& f) {
  static_assert(WORDS >= 1 && WORDS <= 64, "one word per lane at most");
  const int lane = (int)threadIdx.x & 63;
  const long long chunk = (long long)WORDS * gridDim.x * (blockDim.x / 64);
  for (long long base = (long long)WORDS * (blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64);
       base < nwords; base += chunk) {
    const long long w = base + lane;
    const uint64_t word = (lane < WORDS && w < nwords) ? mask[w] : 0ull;
    const int c = __popcll(word);
    int incl = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int u = __shfl_up(incl, d, 64);
      if (lane >= d) incl += u;
    }
    const int excl = incl - c;
    const int total = __shfl(incl, 63, 64);
    for (int k0 = 0; k0 < total; k0 += 64) {
      const int k = k0 + lane;
      int lo = 0;  // the last word whose first flagged site is at or before k
#pragma unroll
      for (int step = 32; step > 0; step >>= 1) {
        const int mid = lo + step;
        if (__shfl(excl, mid, 64) <= k) lo = mid;
      }
      const uint64_t wl = __shfl(word, lo, 64);
      const int nth = k - __shfl(excl, lo, 64);
      if (k >= total) continue;
      const int bit = nth_set_bit(wl, nth);
      const long long wi = base + lo;
      int x, y, z;
      if (g.wpr) {
        const long long row = wi / g.wpr;
        x = (int)(wi % g.wpr) * 64 + bit;
        y = (int)(row % g.ny);
        z = (int)(row / g.ny);
      } else {
        const long long site = wi * 64 + bit;
        x = (int)(site % g.nx);
        y = (int)((site / g.nx) % g.ny);
        z = (int)(site / ((long long)g.nx * g.ny));
      }
      f(x, y, z);
    }
  }
}

// Mask words of a box: rows of 64-site words, or a linear bit array.
__host__ __device__ inline long long mask_nwords(const Geo& g) {
  return g.wpr ? (long long)g.ny * g.nz * g.wpr : (g.N + 63) / 64;
}

}  // namespace lbc
