/*
 * lbo.c -- plain FP64 CPU oracle of the operator-split lattice Boltzmann step
 * with fluid-particle coupling (Schiller, "A unified operator splitting
 * approach for multi-scale fluid-particle coupling in the lattice Boltzmann
 * method", arXiv:1406.2211).
 *
 * TEST INFRASTRUCTURE ONLY: it is the reference the GPU library is checked
 * against, and nothing on the product path may call it.  It is deliberately
 * unfused: every operator of the splitting is a separate pass over full
 * arrays, in the order the paper composes them.
 *
 * Readings taken where the paper leaves a choice open (each is repeated at the
 * function it affects):
 *   R1  D3Q19 with the usual weights; f^eq is the second-order Hermite
 *       polynomial and G_i the second-order Hermite force term with the
 *       moments of Eq. force-moments (the paper names neither explicitly).
 *   R2  tau is the lattice relaxation time (tau_paper + h/2, Sec. 3.2), so the
 *       Crank-Nicolson full-step rate is lambda = 1/tau.
 *   R3  The time step is F^1/2 C S F^1/2 with the full collision C; by
 *       Eq. LB-splitting-combined this is the C^1/2 S C^1/2 core up to the
 *       end half-collisions.
 *   R4  Each F^1/2 uses the midpoint rule with G evaluated at the half-step
 *       midpoint velocity u + (h/4) F / rho (Eq. LB-force-moments, and the
 *       G(t +- h/4) arguments of Eq. force-first-halfstep).
 *   R5  Coupling half steps use h' = h/2 in alpha and beta (Sec. 5.2).
 *   R6  The second coupling half uses the post-stream velocity before that
 *       half's force (Alg. 3 computes the coupling right after the LB update).
 *   R7  The particle velocity kick carries 1/m (Eq. for d v / d t in Sec. 5.2).
 *   R8  IB: the final position half step uses the interpolated physical
 *       velocity after the second half force (Sec. 5.1 position equations).
 *   R9  Halfway bounce-back at y walls on post-collision populations; delta
 *       stencil sites beyond a wall carry no weight.
 *   R10 Populations are kept as deviations df = f - w rho0 (a change of
 *       variables that avoids cancellation).
 */
#include "lbo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* D3Q19 lattice (R1): rest, 6 face and 12 edge velocities.                 */
/* ------------------------------------------------------------------------ */
static int C[LBO_Q][3];
static double W[LBO_Q];
static int OPP[LBO_Q];
static int RANK[LBO_Q]; /* order of c in increasing 9(cx+1) + 3(cy+1) + (cz+1) */
static int lattice_ready = 0;

static void lattice_init(void) {
  if (lattice_ready) return;
  int n = 0;
  C[n][0] = C[n][1] = C[n][2] = 0;
  W[n++] = 1.0 / 3.0;
  for (int a = 0; a < 3; ++a)
    for (int s = 1; s >= -1; s -= 2) {
      C[n][0] = C[n][1] = C[n][2] = 0;
      C[n][a] = s;
      W[n++] = 1.0 / 18.0;
    }
  const int pa[3][2] = {{0, 1}, {1, 2}, {2, 0}};
  for (int p = 0; p < 3; ++p)
    for (int s = 1; s >= -1; s -= 2)
      for (int t = 1; t >= -1; t -= 2) {
        C[n][0] = C[n][1] = C[n][2] = 0;
        C[n][pa[p][0]] = s;
        C[n][pa[p][1]] = t;
        W[n++] = 1.0 / 36.0;
      }
  for (int i = 0; i < LBO_Q; ++i)
    for (int j = 0; j < LBO_Q; ++j)
      if (C[j][0] == -C[i][0] && C[j][1] == -C[i][1] && C[j][2] == -C[i][2])
        OPP[i] = j;
  for (int i = 0; i < LBO_Q; ++i) {
    const int ki = 9 * (C[i][0] + 1) + 3 * (C[i][1] + 1) + (C[i][2] + 1);
    RANK[i] = 0;
    for (int j = 0; j < LBO_Q; ++j)
      if (9 * (C[j][0] + 1) + 3 * (C[j][1] + 1) + (C[j][2] + 1) < ki) ++RANK[i];
  }
  lattice_ready = 1;
}

int lbo_d3q19(int32_t c[LBO_Q * 3], double w[LBO_Q], int32_t opp[LBO_Q]) {
  lattice_init();
  for (int i = 0; i < LBO_Q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = C[i][a];
    w[i] = W[i];
    opp[i] = OPP[i];
  }
  return LBO_Q;
}

int lbo_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static inline long site(const lbo_cfg *g, int x, int y, int z) {
  return ((long)z * g->ny + y) * g->nx + x;
}
static inline int wrapi(int j, int n) {
  int r = j % n;
  return r < 0 ? r + n : r;
}
static inline double wrapd(double x, double L) {
  return x - L * floor(x / L);
}
static inline long nsites(const lbo_cfg *g) { return (long)g->nx * g->ny * g->nz; }

/* ------------------------------------------------------------------------ */
/* Equilibrium and force term (Sec. 2 moments; Eq. force-moments; R1, R10)  */
/* ------------------------------------------------------------------------ */

/* f^eq_i(rho,u) - w_i rho0 with f^eq = w rho [1 + c.u/cs2 + (c.u)^2/(2 cs4)
 * - u.u/(2 cs2)], cs2 = 1/3, written so that the rest part w drho,
 * drho = rho - rho0, is separated from the velocity part.  drho is passed in
 * directly (R10): forming it as (rho0 + sum df) - rho0 would drop its low bits. */
void lbo_feq_dev(double drho, double rho, const double u[3], double out[LBO_Q]) {
  lattice_init();
  const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < LBO_Q; ++i) {
    const double cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
    out[i] = W[i] * drho + W[i] * rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
  }
}

/* G_i = w_i [ c.F/cs2 + (c.u)(c.F)/cs4 - u.F/cs2 ]: zeroth moment 0, first
 * moment F, second moment F u + u F (Eq. force-moments). */
void lbo_force_term(const double u[3], const double F[3], double G[LBO_Q]) {
  lattice_init();
  const double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
  for (int i = 0; i < LBO_Q; ++i) {
    const double cF = C[i][0] * F[0] + C[i][1] * F[1] + C[i][2] * F[2];
    const double cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
    G[i] = W[i] * (3.0 * cF + 9.0 * cu * cF - 3.0 * uF);
  }
}

/* ------------------------------------------------------------------------ */
/* Moment basis for the MRT collision (Eq. mrt-coll).  The paper leaves the */
/* basis open; any w-orthogonal basis works.  This one is Gram-Schmidt on   */
/* 19 monomials of c ordered by degree, with <a,b> = sum_i w_i a_i b_i, so  */
/* rows 0..3 are 1, cx, cy, cz; rows 4..9 span the stress; 10..15 are the   */
/* odd (third-order) ghosts and 16..18 the even (fourth-order) ghosts.      */
/* ------------------------------------------------------------------------ */
void lbo_mrt_basis(double E[LBO_Q * LBO_Q], double b[LBO_Q]) {
  lattice_init();
  for (int i = 0; i < LBO_Q; ++i) {
    const double x = C[i][0], y = C[i][1], z = C[i][2];
    const double mono[LBO_Q] = {1.0,         x,           y,           z,           x * x,
                                y * y,       z * z,       x * y,       y * z,       z * x,
                                x * y * y,   x * z * z,   y * x * x,   y * z * z,   z * x * x,
                                z * y * y,   x * x * y * y, y * y * z * z, z * z * x * x};
    for (int k = 0; k < LBO_Q; ++k) E[k * LBO_Q + i] = mono[k];
  }
  for (int k = 0; k < LBO_Q; ++k) {
    for (int l = 0; l < k; ++l) {
      double num = 0.0;
      for (int i = 0; i < LBO_Q; ++i) num += W[i] * E[k * LBO_Q + i] * E[l * LBO_Q + i];
      const double p = num / b[l];
      for (int i = 0; i < LBO_Q; ++i) E[k * LBO_Q + i] -= p * E[l * LBO_Q + i];
    }
    double nrm = 0.0;
    for (int i = 0; i < LBO_Q; ++i) nrm += W[i] * E[k * LBO_Q + i] * E[k * LBO_Q + i];
    b[k] = nrm;
  }
}

/* Moment basis of the general MRT collision (Eq. mrt-coll with a rate per
 * moment group): the polynomials of the D3Q19 basis of Duenweg, Schiller and
 * Ladd (2007), w-orthogonal, whose rows span the subspaces that the cubic
 * symmetry leaves invariant: 1; c_a; bulk c^2 - 1; shear 3cx^2 - c^2,
 * cy^2 - cz^2, cx cy, cy cz, cz cx; vector ghosts c_a (3c^2 - 5); pseudo-vector
 * ghosts cx (cy^2 - cz^2) and cyclic; scalar ghost 3c^4 - 6c^2 + 1; tensor
 * ghosts (2c^2 - 3)(3cx^2 - c^2), (2c^2 - 3)(cy^2 - cz^2).  A rate per group
 * keeps the collision isotropic. */
void lbo_group_basis(double E[LBO_Q * LBO_Q], double b[LBO_Q]) {
  lattice_init();
  for (int i = 0; i < LBO_Q; ++i) {
    const double x = C[i][0], y = C[i][1], z = C[i][2];
    const double c2 = x * x + y * y + z * z, c4 = c2 * c2;
    const double row[LBO_Q] = {1.0,
                               x,
                               y,
                               z,
                               c2 - 1.0,
                               3.0 * x * x - c2,
                               y * y - z * z,
                               x * y,
                               y * z,
                               z * x,
                               x * (3.0 * c2 - 5.0),
                               y * (3.0 * c2 - 5.0),
                               z * (3.0 * c2 - 5.0),
                               x * (y * y - z * z),
                               y * (z * z - x * x),
                               z * (x * x - y * y),
                               3.0 * c4 - 6.0 * c2 + 1.0,
                               (2.0 * c2 - 3.0) * (3.0 * x * x - c2),
                               (2.0 * c2 - 3.0) * (y * y - z * z)};
    for (int k = 0; k < LBO_Q; ++k) E[k * LBO_Q + i] = row[k];
  }
  for (int k = 0; k < LBO_Q; ++k) {
    double nrm = 0.0;
    for (int i = 0; i < LBO_Q; ++i) nrm += W[i] * E[k * LBO_Q + i] * E[k * LBO_Q + i];
    b[k] = nrm;
  }
}

/* The basis a configuration relaxes in: the group basis for the general MRT,
 * the Gram-Schmidt basis otherwise (any w-orthogonal basis with the same
 * even and odd subspaces gives the same two-rate collision). */
static void basis_for(const lbo_cfg *cfg, double *E, double *b) {
  if (cfg->collision == LBO_MRT)
    lbo_group_basis(E, b);
  else
    lbo_mrt_basis(E, b);
}

/* Relaxation rates per basis row.  BGK: lambda = 1/tau for every row (R2).
 * Two-rate MRT: even rows at lp = 1/tau, odd rows at lm from the magic
 * parameter (1/lp - 1/2)(1/lm - 1/2) = magic.  Rows 0..3 are conserved, so
 * their rate is irrelevant. */
void lbo_rates(const lbo_cfg *cfg, double lam[LBO_Q]) {
  const double lp = 1.0 / cfg->tau;
  if (cfg->collision == LBO_MRT) { /* rows of lbo_group_basis */
    const double *r = cfg->mrt_rates;
    for (int k = 0; k < LBO_Q; ++k) lam[k] = lp; /* conserved rows and shear */
    lam[4] = r[0];
    for (int k = 10; k < 13; ++k) lam[k] = r[1];
    for (int k = 13; k < 16; ++k) lam[k] = r[2];
    lam[16] = r[3];
    lam[17] = lam[18] = r[4];
    return;
  }
  double lm = lp;
  if (cfg->collision == LBO_TRT) lm = 1.0 / (0.5 + cfg->magic / (cfg->tau - 0.5));
  for (int k = 0; k < LBO_Q; ++k) {
    const int odd = (k >= 1 && k <= 3) || (k >= 10 && k <= 15);
    lam[k] = odd ? lm : lp;
  }
}

static void site_rho_u(const lbo_cfg *cfg, const double df[LBO_Q], double *drho, double *rho,
                       double u[3]) {
  double d = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  for (int i = 0; i < LBO_Q; ++i) {
    d += df[i];
    jx += df[i] * C[i][0];
    jy += df[i] * C[i][1];
    jz += df[i] * C[i][2];
  }
  *drho = d;
  *rho = cfg->rho0 + d;
  u[0] = jx / *rho;
  u[1] = jy / *rho;
  u[2] = jz / *rho;
}

/* ------------------------------------------------------------------------ */
/* Random numbers.  Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel */
/* random numbers: as easy as 1, 2, 3", SC 2011): ten rounds, each taking   */
/* the two 32x32 -> 64-bit products of words 0 and 2 with the published     */
/* multipliers and mixing their halves with words 1 and 3 and the key; the  */
/* key advances by the published Weyl increments between rounds.  Normal    */
/* deviates by the Box-Muller transform (Box and Muller 1958) of uniforms   */
/* u = (x / 2^9 + 1/2) / 2^23 in (0, 1) made from the top 23 bits (a value */
/* with 24 significant bits, exact in single precision as well).            */
/* ------------------------------------------------------------------------ */
void lbo_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

static double unit23(uint32_t x) { return ((double)(x >> 9) + 0.5) / 8388608.0; }

void lbo_normals4(const uint32_t ctr[4], const uint32_t key[2], double g[4]) {
  uint32_t x[4];
  lbo_philox(ctr, key, x);
  for (int p = 0; p < 2; ++p) {
    const double r = sqrt(-2.0 * log(unit23(x[2 * p])));
    const double th = 6.283185307179586 * unit23(x[2 * p + 1]);
    g[2 * p] = r * cos(th);
    g[2 * p + 1] = r * sin(th);
  }
}

/* The 19 normal deviates of one site in one step: five Philox blocks with
 * counter (site, step low word, block, step high word), stream 0; deviate
 * RANK[i] belongs to velocity c_i. */
void lbo_site_normals(const lbo_cfg *cfg, int64_t step, uint32_t site, double g[LBO_Q]) {
  lattice_init();
  const uint32_t key[2] = {(uint32_t)cfg->seed, (uint32_t)(cfg->seed >> 32)};
  double all[20];
  for (int k = 0; k < 5; ++k) {
    const uint32_t ctr[4] = {site, (uint32_t)step, (uint32_t)k, (uint32_t)((uint64_t)step >> 32)};
    lbo_normals4(ctr, key, all + 4 * k);
  }
  for (int i = 0; i < LBO_Q; ++i) g[i] = all[RANK[i]];
}

/* Three normal deviates of particle p for coupling step j of a step:
 * counter (p, step low word, 2^16 + j, step high word). */
static void particle_normals(const lbo_cfg *cfg, int64_t step, int p, int j, double g[3]) {
  const uint32_t key[2] = {(uint32_t)cfg->seed, (uint32_t)(cfg->seed >> 32)};
  const uint32_t ctr[4] = {(uint32_t)p, (uint32_t)step, 65536u + (uint32_t)j,
                           (uint32_t)((uint64_t)step >> 32)};
  double all[4];
  lbo_normals4(ctr, key, all);
  g[0] = all[0];
  g[1] = all[1];
  g[2] = all[2];
}

/* Noise of the fluctuating collision (Eq. mrt-fluct) in population form:
 * sqrt(rho) phi_k r_k added to every non-conserved moment (rows 4..18),
 * phi_k = sqrt(mu b_k lambda_k (2 - lambda_k)), mu = k_B T / c_s^2 (a = 1),
 * then f_i = w_i sum_k E_ki m_k / b_k.  The amplitude keeps the variance of
 * each non-conserved moment at its equilibrium value mu rho b_k under
 * m <- (1 - lambda) m + phi r (the fluctuation-dissipation relation of the
 * cited fluctuating LB).  The standard normal r_k are the normalised
 * moments m_k(z)/sqrt(b_k) of z_i = sqrt(w_i) g_i, g_i iid standard normal
 * (independent because the basis is w-orthogonal). */
static void collision_noise(const lbo_cfg *cfg, double rho, const double *g, const double *E,
                            const double *b, const double *lam, double out[LBO_Q]) {
  const double mu = 3.0 * cfg->kT;
  double z[LBO_Q], add[LBO_Q];
  for (int i = 0; i < LBO_Q; ++i) z[i] = sqrt(W[i]) * g[i];
  for (int k = 0; k < LBO_Q; ++k) {
    add[k] = 0.0;
    if (k < 4) continue; /* density and momentum are conserved */
    double m = 0.0;
    for (int i = 0; i < LBO_Q; ++i) m += E[k * LBO_Q + i] * z[i];
    const double r = m / sqrt(b[k]);
    add[k] = sqrt(rho) * sqrt(mu * b[k] * lam[k] * (2.0 - lam[k])) * r;
  }
  for (int i = 0; i < LBO_Q; ++i) {
    double s2 = 0.0;
    for (int k = 4; k < LBO_Q; ++k) s2 += E[k * LBO_Q + i] * add[k] / b[k];
    out[i] = W[i] * s2;
  }
}

/* Collision C (Eq. CN-coll / collision-operator, Eq. mrt-coll) on one site.
 * BGK: f <- f^eq + (1 - lambda)(f - f^eq).  Two-rate MRT: the same relaxation
 * applied row by row in moment space, m_k <- m_k^eq + (1 - lambda_k)(m_k - m_k^eq),
 * followed by f_i = w_i sum_k E_ki m_k / b_k. */
static void collide_site_with(const lbo_cfg *cfg, double df[LBO_Q], const double *E,
                              const double *b, const double *lam) {
  double drho, rho, u[3], feq[LBO_Q];
  site_rho_u(cfg, df, &drho, &rho, u);
  lbo_feq_dev(drho, rho, u, feq);
  if (cfg->collision == LBO_BGK) {
    const double om = 1.0 - lam[4]; /* every non-conserved row relaxes at the same rate */
    for (int i = 0; i < LBO_Q; ++i) df[i] = feq[i] + om * (df[i] - feq[i]);
    return;
  }
  double m[LBO_Q], meq[LBO_Q];
  for (int k = 0; k < LBO_Q; ++k) {
    double s = 0.0, se = 0.0;
    for (int i = 0; i < LBO_Q; ++i) {
      s += E[k * LBO_Q + i] * df[i];
      se += E[k * LBO_Q + i] * feq[i];
    }
    m[k] = se + (1.0 - lam[k]) * (s - se);
    meq[k] = se;
  }
  (void)meq;
  for (int i = 0; i < LBO_Q; ++i) {
    double s = 0.0;
    for (int k = 0; k < LBO_Q; ++k) s += E[k * LBO_Q + i] * m[k] / b[k];
    df[i] = W[i] * s;
  }
}

void lbo_collide_site(const lbo_cfg *cfg, double df[LBO_Q]) {
  double E[LBO_Q * LBO_Q], b[LBO_Q], lam[LBO_Q];
  basis_for(cfg, E, b);
  lbo_rates(cfg, lam);
  collide_site_with(cfg, df, E, b, lam);
}

/* ------------------------------------------------------------------------ */
/* Lattice-wide passes                                                      */
/* ------------------------------------------------------------------------ */

void lbo_init_fluid(const lbo_cfg *cfg, double *df, const double *rho, const double *u) {
  lattice_init();
  const long N = nsites(cfg);
#pragma omp parallel for schedule(static)
  for (long s = 0; s < N; ++s) {
    double uu[3] = {0.0, 0.0, 0.0}, feq[LBO_Q];
    if (u) {
      uu[0] = u[s];
      uu[1] = u[N + s];
      uu[2] = u[2 * N + s];
    }
    const double r = rho ? rho[s] : cfg->rho0;
    lbo_feq_dev(r - cfg->rho0, r, uu, feq);
    for (int i = 0; i < LBO_Q; ++i) df[i * N + s] = feq[i];
  }
}

/* rho = sum_i f_i, u = sum_i f_i c_i / rho (Sec. 2).  In the oracle the
 * stored populations are always physical, so these are the physical fields. */
void lbo_moments(const lbo_cfg *cfg, const double *df, double *rho, double *u) {
  lattice_init();
  const long N = nsites(cfg);
#pragma omp parallel for schedule(static)
  for (long s = 0; s < N; ++s) {
    double f[LBO_Q], d, r, uu[3];
    for (int i = 0; i < LBO_Q; ++i) f[i] = df[i * N + s];
    site_rho_u(cfg, f, &d, &r, uu);
    rho[s] = r;
    u[s] = uu[0];
    u[N + s] = uu[1];
    u[2 * N + s] = uu[2];
  }
}

/* Force operator over a time dt (Eq. force-midpoint with h -> dt; R4):
 * f <- f + dt G(F, u_mid), u_mid = u + (dt/2) F/rho, F = F_ext + Fc(x).  The
 * half step F^1/2 is dt = h/2; the sub-steps of Eq. multistep take dt = h/2n. */
void lbo_force_dt(const lbo_cfg *cfg, double *df, const double *Fc, double dt) {
  lattice_init();
  const long N = nsites(cfg);
#pragma omp parallel for schedule(static)
  for (long s = 0; s < N; ++s) {
    double f[LBO_Q], d, r, uu[3], F[3], G[LBO_Q];
    for (int i = 0; i < LBO_Q; ++i) f[i] = df[i * N + s];
    for (int a = 0; a < 3; ++a) F[a] = cfg->fext[a] + (Fc ? Fc[a * N + s] : 0.0);
    site_rho_u(cfg, f, &d, &r, uu);
    double um[3];
    for (int a = 0; a < 3; ++a) um[a] = uu[a] + 0.5 * dt * F[a] / r;
    lbo_force_term(um, F, G);
    for (int i = 0; i < LBO_Q; ++i) df[i * N + s] = f[i] + dt * G[i];
  }
}

void lbo_force_half(const lbo_cfg *cfg, double *df, const double *Fc) {
  lbo_force_dt(cfg, df, Fc, 0.5);
}

/* Collision of every site; with kT > 0 the fluctuating collision of Eq.
 * mrt-fluct, its random numbers drawn for the given step.  The noise uses the
 * site density before the collision (which the collision conserves). */
void lbo_collide_noisy(const lbo_cfg *cfg, double *df, int64_t step) {
  lattice_init();
  double E[LBO_Q * LBO_Q], b[LBO_Q], lam[LBO_Q];
  basis_for(cfg, E, b);
  lbo_rates(cfg, lam);
  const long N = nsites(cfg);
#pragma omp parallel for schedule(static)
  for (long s = 0; s < N; ++s) {
    double f[LBO_Q], d, r, u[3];
    for (int i = 0; i < LBO_Q; ++i) f[i] = df[i * N + s];
    site_rho_u(cfg, f, &d, &r, u);
    collide_site_with(cfg, f, E, b, lam);
    if (cfg->kT > 0.0) {
      double g[LBO_Q], n[LBO_Q];
      lbo_site_normals(cfg, step, (uint32_t)s, g);
      collision_noise(cfg, r, g, E, b, lam, n);
      for (int i = 0; i < LBO_Q; ++i) f[i] += n[i];
    }
    for (int i = 0; i < LBO_Q; ++i) df[i * N + s] = f[i];
  }
}

void lbo_collide(const lbo_cfg *cfg, double *df) { lbo_collide_noisy(cfg, df, cfg->step0); }

/* Half-step collision C^1/2 of the collide-stream-collide form (Sec. 4):
 * the same relaxation with 1 - lambda_1/2 = sqrt(1 - lambda) for every
 * eigenvalue (Sec. 3.2, the exact half step), so that C^1/2 C^1/2 = C.  Real
 * only for lambda <= 1. */
void lbo_collide_half(const lbo_cfg *cfg, double *df) {
  lattice_init();
  double E[LBO_Q * LBO_Q], b[LBO_Q], lam[LBO_Q];
  basis_for(cfg, E, b);
  lbo_rates(cfg, lam);
  for (int k = 0; k < LBO_Q; ++k) lam[k] = 1.0 - sqrt(1.0 - lam[k]);
  const long N = nsites(cfg);
#pragma omp parallel for schedule(static)
  for (long s = 0; s < N; ++s) {
    double f[LBO_Q];
    for (int i = 0; i < LBO_Q; ++i) f[i] = df[i * N + s];
    collide_site_with(cfg, f, E, b, lam);
    for (int i = 0; i < LBO_Q; ++i) df[i * N + s] = f[i];
  }
}

/* Non-equilibrium second moment Pi_ab = sum_i (f_i - f^eq_i(rho, u)) c_ia c_ib
 * of the given populations, u their own velocity (the stress of Eq. viscstress
 * before its prefactor). */
void lbo_stress(const lbo_cfg *cfg, const double *df, double *pi) {
  lattice_init();
  const long N = nsites(cfg);
  static const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
#pragma omp parallel for schedule(static)
  for (long s = 0; s < N; ++s) {
    double f[LBO_Q], d, r, uu[3], feq[LBO_Q];
    for (int i = 0; i < LBO_Q; ++i) f[i] = df[i * N + s];
    site_rho_u(cfg, f, &d, &r, uu);
    lbo_feq_dev(d, r, uu, feq);
    for (int q = 0; q < 6; ++q) {
      double acc = 0.0;
      for (int i = 0; i < LBO_Q; ++i) acc += (f[i] - feq[i]) * C[i][A[q]] * C[i][B[q]];
      pi[q * N + s] = acc;
    }
  }
}

/* Streaming S (Sec. 3.1): f_i(x + c_i) <- f_i(x), written in pull form
 * dst_i(x) = src_i(x - c_i), periodic in every direction without a wall; with
 * y walls (R9) a population whose source lies beyond a wall is the reflected
 * opposite population of the same site, dst_i(x) = src_opp(i)(x). */
void lbo_stream(const lbo_cfg *cfg, const double *src, double *dst) {
  lattice_init();
  const long N = nsites(cfg);
#pragma omp parallel for schedule(static)
  for (int z = 0; z < cfg->nz; ++z)
    for (int y = 0; y < cfg->ny; ++y)
      for (int x = 0; x < cfg->nx; ++x) {
        const long s = site(cfg, x, y, z);
        for (int i = 0; i < LBO_Q; ++i) {
          const int ys = y - C[i][1];
          if (cfg->wall_y && (ys < 0 || ys >= cfg->ny)) {
            dst[i * N + s] = src[OPP[i] * N + s];
          } else {
            const long t = site(cfg, wrapi(x - C[i][0], cfg->nx), wrapi(ys, cfg->ny),
                                wrapi(z - C[i][2], cfg->nz));
            dst[i * N + s] = src[i * N + t];
          }
        }
      }
}

/* ------------------------------------------------------------------------ */
/* Delta functions (Appendix A) and the interpolation / spreading pair      */
/* (Eq. IBM-interpolation, Eq. IBM-spreading).                              */
/* ------------------------------------------------------------------------ */

/* phi_2: linear interpolation.  phi_3: the closed form of Appendix A.
 * phi_4: Peskin's four-point function (cited by the paper, not printed). */
double lbo_phi(int kernel, double r) {
  const double a = fabs(r);
  switch (kernel) {
    case 2:
      return a < 1.0 ? 1.0 - a : 0.0;
    case 3:
      if (a <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * r * r)) / 3.0;
      if (a <= 1.5) return (5.0 - 3.0 * a - sqrt(6.0 * a - 2.0 - 3.0 * r * r)) / 6.0;
      return 0.0;
    case 4:
      if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * r * r)) / 8.0;
      if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * r * r)) / 8.0;
      return 0.0;
  }
  return 0.0;
}

/* Weights of every lattice node j in a window wide enough for any kernel;
 * nodes outside the support get weight 0.  Returns the first node. */
#define LBO_WIN 6
static int node_weights(const lbo_cfg *cfg, int dim, double X, double wgt[LBO_WIN],
                        int idx[LBO_WIN]) {
  const int n = dim == 0 ? cfg->nx : (dim == 1 ? cfg->ny : cfg->nz);
  const int j0 = (int)floor(X) - 2;
  for (int k = 0; k < LBO_WIN; ++k) {
    const int j = j0 + k;
    wgt[k] = lbo_phi(cfg->kernel, (double)j - X);
    if (dim == 1 && cfg->wall_y) {
      if (j < 0 || j >= n) wgt[k] = 0.0; /* R9 */
      idx[k] = j < 0 ? 0 : (j >= n ? n - 1 : j);
    } else {
      idx[k] = wrapi(j, n);
    }
  }
  return j0;
}

/* u(X) = sum_x u(x) delta(X - x) and likewise rho(X) (Eq. IBM-interpolation). */
void lbo_interp(const lbo_cfg *cfg, int np, const double *pos, const double *rho,
                const double *u, double *rho_p, double *u_p) {
  const long N = nsites(cfg);
  for (int p = 0; p < np; ++p) {
    double wx[LBO_WIN], wy[LBO_WIN], wz[LBO_WIN];
    int ix[LBO_WIN], iy[LBO_WIN], iz[LBO_WIN];
    node_weights(cfg, 0, pos[3 * p + 0], wx, ix);
    node_weights(cfg, 1, pos[3 * p + 1], wy, iy);
    node_weights(cfg, 2, pos[3 * p + 2], wz, iz);
    double r = 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
    for (int c = 0; c < LBO_WIN; ++c)
      for (int b = 0; b < LBO_WIN; ++b)
        for (int a = 0; a < LBO_WIN; ++a) {
          const double wt = wx[a] * wy[b] * wz[c];
          if (wt == 0.0) continue;
          const long s = site(cfg, ix[a], iy[b], iz[c]);
          r += wt * rho[s];
          ux += wt * u[s];
          uy += wt * u[N + s];
          uz += wt * u[2 * N + s];
        }
    rho_p[p] = r;
    u_p[3 * p + 0] = ux;
    u_p[3 * p + 1] = uy;
    u_p[3 * p + 2] = uz;
  }
}

/* F(x) += a^-3 sum_p F_p delta(X_p - x), a = 1 (Eq. IBM-spreading). */
void lbo_spread(const lbo_cfg *cfg, int np, const double *pos, const double *Fp,
                double *Fgrid) {
  const long N = nsites(cfg);
  for (int p = 0; p < np; ++p) {
    double wx[LBO_WIN], wy[LBO_WIN], wz[LBO_WIN];
    int ix[LBO_WIN], iy[LBO_WIN], iz[LBO_WIN];
    node_weights(cfg, 0, pos[3 * p + 0], wx, ix);
    node_weights(cfg, 1, pos[3 * p + 1], wy, iy);
    node_weights(cfg, 2, pos[3 * p + 2], wz, iz);
    for (int c = 0; c < LBO_WIN; ++c)
      for (int b = 0; b < LBO_WIN; ++b)
        for (int a = 0; a < LBO_WIN; ++a) {
          const double wt = wx[a] * wy[b] * wz[c];
          if (wt == 0.0) continue;
          const long s = site(cfg, ix[a], iy[b], iz[c]);
          Fgrid[s] += wt * Fp[3 * p + 0];
          Fgrid[N + s] += wt * Fp[3 * p + 1];
          Fgrid[2 * N + s] += wt * Fp[3 * p + 2];
        }
  }
}

/* ------------------------------------------------------------------------ */
/* Coupling forces for one half step of length hh (R5).                     */
/* ------------------------------------------------------------------------ */

/* Force coupling, Eq. modified-force:
 * F^h = -[gamma (v - u) + (alpha/2) F_int] / (1 + alpha/2 + beta/2),
 * alpha = gamma hh / m, beta = gamma hh / (rho a^3). */
void lbo_fc_force(double gamma, double m, double rho_p, double hh, const double v[3],
                  const double u_p[3], const double Fint[3], double Fh[3]) {
  const double alpha = gamma * hh / m, beta = gamma * hh / rho_p;
  const double den = 1.0 + 0.5 * alpha + 0.5 * beta;
  for (int a = 0; a < 3; ++a) Fh[a] = -(gamma * (v[a] - u_p[a]) + 0.5 * alpha * Fint[a]) / den;
}

/* Modified external boundary force, Eq. modified-ebf and the force before it:
 * F^h = -gamma/(alpha+beta) (v - u) - alpha/(alpha+beta) F_int,
 * v' = v - alpha/(alpha+beta) (v - u) + (hh/m) beta/(alpha+beta) F_int. */
void lbo_ebf_update(double gamma, double m, double rho_p, double hh, const double v[3],
                    const double u_p[3], const double Fint[3], double Fh[3],
                    double v_new[3]) {
  const double alpha = gamma * hh / m, beta = gamma * hh / rho_p;
  const double s = alpha + beta;
  for (int a = 0; a < 3; ++a) {
    const double d = v[a] - u_p[a];
    Fh[a] = -gamma / s * d - alpha / s * Fint[a];
    v_new[a] = v[a] - alpha / s * d + (hh / m) * (beta / s) * Fint[a];
  }
}

/* ------------------------------------------------------------------------ */
/* Intrinsic forces ("CalculateForces" in Alg. 2 and 3; the paper leaves    */
/* the model open).  Bonds: harmonic U = k/2 (|d| - r0)^2 or FENE           */
/* U = -k R0^2/2 ln(1 - |d|^2/R0^2).  Shells: each marker is tethered to a  */
/* rigid copy of the shell template placed at the shell centroid with the   */
/* least-squares rotation (Horn's unit-quaternion solution).                */
/* ------------------------------------------------------------------------ */
static void min_image(const lbo_cfg *cfg, double d[3]) {
  const double L[3] = {cfg->nx, cfg->ny, cfg->nz};
  for (int a = 0; a < 3; ++a) {
    if (a == 1 && cfg->wall_y) continue;
    d[a] -= L[a] * floor(d[a] / L[a] + 0.5);
  }
}

void lbo_bond_forces(const lbo_cfg *cfg, int np, const double *pos, double *F) {
  (void)np;
  for (int b = 0; b < cfg->nbond; ++b) {
    const int i = cfg->bond_pairs[2 * b], j = cfg->bond_pairs[2 * b + 1];
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = pos[3 * j + a] - pos[3 * i + a];
    min_image(cfg, d);
    const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double s; /* F_i = s d */
    if (cfg->bond_type == LBO_FENE) {
      /* U = -k r0^2/2 ln(1 - L^2/r0^2) is infinite from L = r0 on: the force
       * there is NaN, not the sign-flipped value of the formula */
      s = L < cfg->bond_r0 ? cfg->bond_k / (1.0 - L * L / (cfg->bond_r0 * cfg->bond_r0)) : NAN;
    } else {
      s = L > 0.0 ? cfg->bond_k * (L - cfg->bond_r0) / L : 0.0;
    }
    for (int a = 0; a < 3; ++a) {
      F[3 * i + a] += s * d[a];
      F[3 * j + a] -= s * d[a];
    }
  }
}

/* Cyclic Jacobi eigen-decomposition of a symmetric 4x4 matrix. */
static void jacobi4(double A[4][4], double V[4][4]) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        tot += A[i][j] * A[i][j];
        if (i != j) off += A[i][j] * A[i][j];
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 4; ++q) {
        if (A[p][q] == 0.0) continue;
        const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 4; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 4; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 4; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
}

void lbo_tether_forces(const lbo_cfg *cfg, const double *pos, double *F, double *rot) {
  const int M = cfg->shell_size;
  double *y = (double *)malloc(sizeof(double) * 3 * (M > 0 ? M : 1));
  for (int sh = 0; sh < cfg->nshell; ++sh) {
    const double *X = pos + 3L * sh * M;
    /* unwrap the shell around its first marker, then centre it */
    double cen[3] = {0, 0, 0};
    for (int j = 0; j < M; ++j) {
      double d[3];
      for (int a = 0; a < 3; ++a) d[a] = X[3 * j + a] - X[a];
      min_image(cfg, d);
      for (int a = 0; a < 3; ++a) {
        y[3 * j + a] = X[a] + d[a];
        cen[a] += y[3 * j + a];
      }
    }
    for (int a = 0; a < 3; ++a) cen[a] /= M;
    /* S_ab = sum_j t_a p_b with t the template and p the centred marker */
    double S[3][3] = {{0}};
    for (int j = 0; j < M; ++j)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          S[a][b] += cfg->shell_template[3 * j + a] * (y[3 * j + b] - cen[b]);
    double N[4][4] = {
        {S[0][0] + S[1][1] + S[2][2], S[1][2] - S[2][1], S[2][0] - S[0][2], S[0][1] - S[1][0]},
        {S[1][2] - S[2][1], S[0][0] - S[1][1] - S[2][2], S[0][1] + S[1][0], S[2][0] + S[0][2]},
        {S[2][0] - S[0][2], S[0][1] + S[1][0], -S[0][0] + S[1][1] - S[2][2], S[1][2] + S[2][1]},
        {S[0][1] - S[1][0], S[2][0] + S[0][2], S[1][2] + S[2][1], -S[0][0] - S[1][1] + S[2][2]}};
    double V[4][4];
    jacobi4(N, V);
    int best = 0;
    for (int k = 1; k < 4; ++k)
      if (N[k][k] > N[best][best]) best = k;
    const double q0 = V[0][best], qx = V[1][best], qy = V[2][best], qz = V[3][best];
    const double R[3][3] = {
        {q0 * q0 + qx * qx - qy * qy - qz * qz, 2 * (qx * qy - q0 * qz), 2 * (qx * qz + q0 * qy)},
        {2 * (qy * qx + q0 * qz), q0 * q0 - qx * qx + qy * qy - qz * qz, 2 * (qy * qz - q0 * qx)},
        {2 * (qz * qx - q0 * qy), 2 * (qz * qy + q0 * qx), q0 * q0 - qx * qx - qy * qy + qz * qz}};
    if (rot)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) rot[9 * sh + 3 * a + b] = R[a][b];
    for (int j = 0; j < M; ++j) {
      const double *t = cfg->shell_template + 3 * j;
      for (int a = 0; a < 3; ++a) {
        const double target = R[a][0] * t[0] + R[a][1] * t[1] + R[a][2] * t[2];
        F[3L * (sh * M + j) + a] += -cfg->tether_k * (y[3 * j + a] - cen[a] - target);
      }
    }
  }
  free(y);
}

void lbo_intrinsic(const lbo_cfg *cfg, int np, const double *pos, double *F) {
  memset(F, 0, sizeof(double) * 3 * np);
  if (cfg->nbond > 0) lbo_bond_forces(cfg, np, pos, F);
  if (cfg->nshell > 0) lbo_tether_forces(cfg, pos, F, NULL);
}

/* ------------------------------------------------------------------------ */
/* Full time steps                                                          */
/* ------------------------------------------------------------------------ */
typedef struct work {
  double *df2, *rho, *u, *Fc, *Fint, *rho_p, *u_p, *Fh, *X1;
  int64_t t; /* index of the current step in the random streams */
} work;

static int work_alloc(const lbo_cfg *cfg, int np, work *w) {
  const long N = nsites(cfg);
  const int n = np > 0 ? np : 1;
  w->df2 = (double *)malloc(sizeof(double) * LBO_Q * N);
  w->rho = (double *)malloc(sizeof(double) * N);
  w->u = (double *)malloc(sizeof(double) * 3 * N);
  w->Fc = (double *)malloc(sizeof(double) * 3 * N);
  w->Fint = (double *)malloc(sizeof(double) * 3 * n);
  w->rho_p = (double *)malloc(sizeof(double) * n);
  w->u_p = (double *)malloc(sizeof(double) * 3 * n);
  w->Fh = (double *)malloc(sizeof(double) * 3 * n);
  w->X1 = (double *)malloc(sizeof(double) * 3 * n);
  return w->df2 && w->rho && w->u && w->Fc && w->Fint && w->rho_p && w->u_p && w->Fh && w->X1;
}
static void work_free(work *w) {
  free(w->df2); free(w->rho); free(w->u); free(w->Fc); free(w->Fint);
  free(w->rho_p); free(w->u_p); free(w->Fh); free(w->X1);
}

static void wrap_positions(const lbo_cfg *cfg, int np, double *pos) {
  const double L[3] = {cfg->nx, cfg->ny, cfg->nz};
  for (int p = 0; p < np; ++p)
    for (int a = 0; a < 3; ++a) {
      if (a == 1 && cfg->wall_y) continue;
      pos[3 * p + a] = wrapd(pos[3 * p + a], L[a]);
    }
}

static void drift(const lbo_cfg *cfg, int np, double *pos, const double *vel, double dt) {
  for (int p = 0; p < np; ++p)
    for (int a = 0; a < 3; ++a) pos[3 * p + a] += dt * vel[3 * p + a];
  wrap_positions(cfg, np, pos);
}

/* The LB update between the two half forces: C S (Eq. LB-splitting-combined),
 * or C^1/2 S C^1/2 in the collide-stream-collide form (Eq. csc); streams into
 * the other buffer and returns it. */
static double *collide_stream(const lbo_cfg *cfg, double *df, work *w) {
  if (cfg->csc) {
    lbo_collide_half(cfg, df);
    lbo_stream(cfg, df, w->df2);
    lbo_collide_half(cfg, w->df2);
    return w->df2;
  }
  lbo_collide_noisy(cfg, df, w->t);
  lbo_stream(cfg, df, w->df2);
  return w->df2;
}

/* One coupling step of length hh (Alg. 3 CalculateCoupling, velocity kick
 * and SpreadForce; hh = h/2 for the half steps): computes F^h at every
 * particle from the current fluid fields (w->rho, w->u), kicks v by
 * (hh/m)(F^h + F_int) (R7), and writes the lattice force -I*[r] F^h into
 * w->Fc. */
static void coupling_step(const lbo_cfg *cfg, int np, const double *pos, double *vel,
                          const double *mass, const double *Fint, double hh, int j, work *w) {
  const long N = nsites(cfg);
  lbo_interp(cfg, np, pos, w->rho, w->u, w->rho_p, w->u_p);
  for (int p = 0; p < np; ++p) {
    double *Fh = w->Fh + 3 * p, *v = vel + 3 * p;
    if (cfg->coupling == LBO_FC) {
      lbo_fc_force(cfg->gamma, mass[p], w->rho_p[p], hh, v, w->u_p + 3 * p, Fint + 3 * p, Fh);
      {
        /* The fluid at the particle also feels the body force over the coupling
         * step: Eq. fc-vel with du/dt = [gamma (v - u) + F_ext] / (rho a^3).
         * The Crank-Nicolson solution then gains +(beta/2) F_ext in the bracket
         * of Eq. modified-force (R6b), which keeps the step second order under a
         * body force (it is first order when the body force stays outside). */
        const double al = cfg->gamma * hh / mass[p], be = cfg->gamma * hh / w->rho_p[p];
        for (int a = 0; a < 3; ++a)
          Fh[a] += 0.5 * be * cfg->fext[a] / (1.0 + 0.5 * al + 0.5 * be);
      }
      if (cfg->kT > 0.0) {
        /* random force zeta of Eq. viscous-coupling, variance 2 k_B T gamma / hh
         * per component over a coupling step of length hh, entering the implicit
         * solution like the drag: F^h gains zeta / (1 + alpha/2 + beta/2) */
        double g[3];
        particle_normals(cfg, w->t, p, j, g);
        const double al = cfg->gamma * hh / mass[p], be = cfg->gamma * hh / w->rho_p[p];
        const double sig = sqrt(2.0 * cfg->kT * cfg->gamma / hh);
        for (int a = 0; a < 3; ++a) Fh[a] += sig * g[a] / (1.0 + 0.5 * al + 0.5 * be);
      }
      for (int a = 0; a < 3; ++a) v[a] += hh / mass[p] * (Fh[a] + Fint[3 * p + a]);
    } else {
      double vn[3];
      lbo_ebf_update(cfg->gamma, mass[p], w->rho_p[p], hh, v, w->u_p + 3 * p, Fint + 3 * p,
                     Fh, vn);
      for (int a = 0; a < 3; ++a) v[a] = vn[a];
    }
    for (int a = 0; a < 3; ++a) Fh[a] = -Fh[a]; /* the fluid feels -F^h */
  }
  memset(w->Fc, 0, sizeof(double) * 3 * N);
  lbo_spread(cfg, np, pos, w->Fh, w->Fc);
}

/* Force coupling / modified EBF, Eq. fc-splitting in the ordering of Alg. 3:
 * P^1/2, F^1/2 (coupling + lattice), C, S, F^1/2 (coupling + lattice), P^1/2. */
static double *step_fc(const lbo_cfg *cfg, double *df, int np, double *pos, double *vel,
                       const double *mass, work *w) {
  const int part = cfg->coupling != LBO_NONE && np > 0;
  if (part) {
    drift(cfg, np, pos, vel, 0.5);
    lbo_intrinsic(cfg, np, pos, w->Fint);
    lbo_moments(cfg, df, w->rho, w->u);
    coupling_step(cfg, np, pos, vel, mass, w->Fint, 0.5, 0, w);
  }
  lbo_force_half(cfg, df, part ? w->Fc : NULL);
  df = collide_stream(cfg, df, w);
  const int planted = part && cfg->order == 2; /* TEST ONLY: final P^1/2 misplaced */
  if (planted) drift(cfg, np, pos, vel, 0.5);
  if (part) {
    lbo_moments(cfg, df, w->rho, w->u); /* post-stream, before the half force (R6) */
    coupling_step(cfg, np, pos, vel, mass, w->Fint, 0.5, 1, w);
  }
  lbo_force_half(cfg, df, part ? w->Fc : NULL);
  if (part && !planted) drift(cfg, np, pos, vel, 0.5);
  return df;
}

/* TEST ONLY (order = 1).  The first-order sequence P S C F of Sec. 5.1,
 * applied right to left: the force operator over a full step h (the coupling
 * of Sec. 5.2 with h' = h at the current positions, the kick, the lattice
 * force with the body force), the collision, streaming, then the full
 * position update with the new velocities.  The second-order pins measure the
 * splitting of Eq. fc-splitting against this sequence. */
static double *step_fc_first_order(const lbo_cfg *cfg, double *df, int np, double *pos,
                                   double *vel, const double *mass, work *w) {
  const int part = cfg->coupling != LBO_NONE && np > 0;
  if (part) {
    lbo_intrinsic(cfg, np, pos, w->Fint);
    lbo_moments(cfg, df, w->rho, w->u);
    coupling_step(cfg, np, pos, vel, mass, w->Fint, 1.0, 0, w);
  }
  lbo_force_dt(cfg, df, part ? w->Fc : NULL, 1.0);
  df = collide_stream(cfg, df, w);
  if (part) drift(cfg, np, pos, vel, 1.0);
  return df;
}

/* n velocity-Verlet sub-steps of length dt = h/(2n) with intrinsic forces only
 * (the [P^(1/4n) F_int^(1/2n) P^(1/4n)]^n factor of Sec. 6). */
static void substeps(const lbo_cfg *cfg, int np, double *pos, double *vel, const double *mass,
                     work *w) {
  const double dt = 1.0 / (2.0 * cfg->mts_n);
  for (int s = 0; s < cfg->mts_n; ++s) {
    drift(cfg, np, pos, vel, 0.5 * dt);
    lbo_intrinsic(cfg, np, pos, w->Fint);
    for (int p = 0; p < np; ++p)
      for (int a = 0; a < 3; ++a) vel[3 * p + a] += dt / mass[p] * w->Fint[3 * p + a];
    drift(cfg, np, pos, vel, 0.5 * dt);
  }
}

/* Multiple time-step splitting with the coupling outside (Sec. 6, second
 * decomposition): F_h^1/2 [P F_int P]^n (C S) [P F_int P]^n F_h^1/2.  The
 * coupling halves carry no intrinsic force (it has its own sub-steps). */
static double *step_mts(const lbo_cfg *cfg, double *df, int np, double *pos, double *vel,
                        const double *mass, work *w) {
  memset(w->X1, 0, sizeof(double) * 3 * (np > 0 ? np : 1));
  lbo_moments(cfg, df, w->rho, w->u);
  coupling_step(cfg, np, pos, vel, mass, w->X1, 0.5, 0, w);
  lbo_force_half(cfg, df, w->Fc);
  substeps(cfg, np, pos, vel, mass, w);
  df = collide_stream(cfg, df, w);
  substeps(cfg, np, pos, vel, mass, w);
  lbo_moments(cfg, df, w->rho, w->u);
  coupling_step(cfg, np, pos, vel, mass, w->X1, 0.5, 1, w);
  lbo_force_half(cfg, df, w->Fc);
  return df;
}

/* One sub-step P^(1/4n) F^(1/2n) P^(1/4n) of Eq. multistep, dt = h/2n: drift
 * dt/2, the intrinsic force at the midpoint, the coupling over dt (particles
 * and lattice, with the body force), drift dt/2.  The fluid velocity is that
 * of the populations as they stand, so each sub-step sees the forces of the
 * earlier ones; after the LB update the first sees the post-stream velocity
 * (R6). */
static void coupled_substep(const lbo_cfg *cfg, double *df, int np, double *pos, double *vel,
                            const double *mass, double dt, int j, work *w) {
  drift(cfg, np, pos, vel, 0.5 * dt);
  lbo_intrinsic(cfg, np, pos, w->Fint);
  lbo_moments(cfg, df, w->rho, w->u);
  coupling_step(cfg, np, pos, vel, mass, w->Fint, dt, j, w);
  lbo_force_dt(cfg, df, w->Fc, dt);
  drift(cfg, np, pos, vel, 0.5 * dt);
}

/* Multiple time-step splitting with the coupling inside (Eq. multistep):
 * [P^(1/4n) F^(1/2n) P^(1/4n)]^n (C S) [P^(1/4n) F^(1/2n) P^(1/4n)]^n, where
 * F holds every force (intrinsic, coupling, body force). */
static double *step_mts_inside(const lbo_cfg *cfg, double *df, int np, double *pos,
                               double *vel, const double *mass, work *w) {
  const double dt = 1.0 / (2.0 * cfg->mts_n);
  const int n = cfg->mts_n;
  for (int k = 0; k < n; ++k) coupled_substep(cfg, df, np, pos, vel, mass, dt, k, w);
  df = collide_stream(cfg, df, w);
  for (int k = 0; k < n; ++k) coupled_substep(cfg, df, np, pos, vel, mass, dt, n + k, w);
  return df;
}

/* Immersed boundary method, Eq. IBM-scheme with the predictor of Sec. 5.1
 * (Alg. 2): X~ = X + h/2 I[X]u(t); forces at X~; X += h/2 I[X~]u(t);
 * F^1/2 with I*[X~]F; C S; F^1/2 with the same force; X += h/2 I[X~]u(t+h) (R8). */
static double *step_ib(const lbo_cfg *cfg, double *df, int np, double *X, work *w) {
  const long N = nsites(cfg);
  double *Xt = w->X1;
  lbo_moments(cfg, df, w->rho, w->u);
  lbo_interp(cfg, np, X, w->rho, w->u, w->rho_p, w->u_p);
  /* order = 2 (TEST ONLY) plants a mistake: no predictor, X~ = X(t) */
  const double pred = cfg->order == 2 ? 0.0 : 0.5;
  for (int p = 0; p < 3 * np; ++p) Xt[p] = X[p] + pred * w->u_p[p];
  wrap_positions(cfg, np, Xt);
  lbo_intrinsic(cfg, np, Xt, w->Fint);
  lbo_interp(cfg, np, Xt, w->rho, w->u, w->rho_p, w->u_p);
  for (int p = 0; p < 3 * np; ++p) X[p] += 0.5 * w->u_p[p];
  wrap_positions(cfg, np, X);
  memset(w->Fc, 0, sizeof(double) * 3 * N);
  lbo_spread(cfg, np, Xt, w->Fint, w->Fc);
  lbo_force_half(cfg, df, w->Fc);
  df = collide_stream(cfg, df, w);
  lbo_force_half(cfg, df, w->Fc);
  lbo_moments(cfg, df, w->rho, w->u);
  lbo_interp(cfg, np, Xt, w->rho, w->u, w->rho_p, w->u_p);
  for (int p = 0; p < 3 * np; ++p) X[p] += 0.5 * w->u_p[p];
  wrap_positions(cfg, np, X);
  return df;
}

/* TEST ONLY (order = 1).  The first-order IB sequence P S C F of Sec. 5.1:
 * the intrinsic forces at X(t) spread and applied over a full step, the
 * collision, streaming, then X(t+h) = X(t) + h I[X(t)] u(t+h). */
static double *step_ib_first_order(const lbo_cfg *cfg, double *df, int np, double *X,
                                   work *w) {
  const long N = nsites(cfg);
  lbo_intrinsic(cfg, np, X, w->Fint);
  memset(w->Fc, 0, sizeof(double) * 3 * N);
  lbo_spread(cfg, np, X, w->Fint, w->Fc);
  lbo_force_dt(cfg, df, w->Fc, 1.0);
  df = collide_stream(cfg, df, w);
  lbo_moments(cfg, df, w->rho, w->u);
  lbo_interp(cfg, np, X, w->rho, w->u, w->rho_p, w->u_p);
  for (int p = 0; p < 3 * np; ++p) X[p] += w->u_p[p];
  wrap_positions(cfg, np, X);
  return df;
}

static int check_cfg(const lbo_cfg *cfg, int np, const double *mass) {
  if (cfg->nx <= 0 || cfg->ny <= 0 || cfg->nz <= 0) return -1;
  if (!(cfg->tau > 0.5)) return -1;
  if (cfg->csc) { /* the exact half step needs every rate <= 1 */
    double lam[LBO_Q];
    lbo_rates(cfg, lam);
    for (int k = 0; k < LBO_Q; ++k)
      if (lam[k] > 1.0) return -1;
  }
  if (cfg->kernel < 2 || cfg->kernel > 4) return -1;
  if (cfg->coupling == LBO_IB && cfg->mts_n > 0) return -1;
  if (cfg->mts_inside != 0 && cfg->mts_inside != 1) return -1;
  if (cfg->order < 0 || cfg->order > 2) return -1;
  if (cfg->order != 0 && (cfg->mts_n > 0 || cfg->csc || cfg->kT > 0.0)) return -1;
  if (!(cfg->kT >= 0.0)) return -1;
  if (cfg->collision == LBO_MRT)
    for (int k = 0; k < 5; ++k)
      if (!(cfg->mrt_rates[k] > 0.0 && cfg->mrt_rates[k] < 2.0)) return -1;
  if (cfg->kT > 0.0 && cfg->csc) return -1; /* C^1/2 of a fluctuating state is not the
                                               fluctuating half step (Sec. 3.2) */
  if ((cfg->coupling == LBO_FC || cfg->coupling == LBO_EBF) && np > 0 && !mass) return -1;
  if (cfg->nshell > 0 && cfg->nshell * cfg->shell_size > np) return -1;
  return 0;
}

int lbo_run(const lbo_cfg *cfg, int nsteps, double *df, int np, double *pos, double *vel,
            const double *mass) {
  lattice_init();
  if (check_cfg(cfg, np, mass)) return -1;
  work w;
  if (!work_alloc(cfg, np, &w)) {
    work_free(&w);
    return -2;
  }
  const long n = (long)LBO_Q * nsites(cfg);
  double *orig2 = w.df2;
  double *cur = df;
  for (int t = 0; t < nsteps; ++t) {
    double *out;
    w.t = cfg->step0 + t;
    if (cfg->coupling == LBO_IB)
      out = cfg->order == 1 ? step_ib_first_order(cfg, cur, np, pos, &w)
                            : step_ib(cfg, cur, np, pos, &w);
    else if (cfg->order == 1)
      out = step_fc_first_order(cfg, cur, np, pos, vel, mass, &w);
    else if (cfg->mts_n > 0 && cfg->coupling != LBO_NONE && np > 0)
      out = cfg->mts_inside ? step_mts_inside(cfg, cur, np, pos, vel, mass, &w)
                            : step_mts(cfg, cur, np, pos, vel, mass, &w);
    else
      out = step_fc(cfg, cur, np, pos, vel, mass, &w);
    /* out is the buffer that was w.df2; the old one becomes scratch */
    w.df2 = cur;
    cur = out;
  }
  if (cur != df) {
    memcpy(df, cur, sizeof(double) * n);
    w.df2 = cur;
  }
  (void)orig2;
  work_free(&w);
  return 0;
}

int lbo_step(const lbo_cfg *cfg, double *df, int np, double *pos, double *vel,
             const double *mass) {
  return lbo_run(cfg, 1, df, np, pos, vel, mass);
}

/* Totals in FP64: out[0] = sum_x rho - N rho0, out[1..3] = fluid momentum
 * sum_x sum_i f_i c_i, out[4..6] = sum_p m_p v_p.  Slab sums are added in a
 * fixed order so the result does not depend on the thread count. */
void lbo_totals(const lbo_cfg *cfg, const double *df, int np, const double *vel,
                const double *mass, double out[7]) {
  lattice_init();
  const long N = nsites(cfg);
  const long slab = (long)cfg->nx * cfg->ny;
  double *part = (double *)calloc(4 * (size_t)cfg->nz, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int z = 0; z < cfg->nz; ++z) {
    double m = 0, px = 0, py = 0, pz = 0;
    for (long s = z * slab; s < (z + 1) * slab; ++s)
      for (int i = 0; i < LBO_Q; ++i) {
        const double f = df[i * N + s];
        m += f;
        px += f * C[i][0];
        py += f * C[i][1];
        pz += f * C[i][2];
      }
    part[4 * z] = m;
    part[4 * z + 1] = px;
    part[4 * z + 2] = py;
    part[4 * z + 3] = pz;
  }
  for (int k = 0; k < 7; ++k) out[k] = 0.0;
  for (int z = 0; z < cfg->nz; ++z)
    for (int k = 0; k < 4; ++k) out[k] += part[4 * z + k];
  free(part);
  if (vel && mass)
    for (int p = 0; p < np; ++p)
      for (int a = 0; a < 3; ++a) out[4 + a] += mass[p] * vel[3 * p + a];
}
