/*
 * lbo.h -- plain FP64 CPU oracle of the operator-split lattice Boltzmann
 * step with fluid-particle coupling (Schiller, arXiv:1406.2211).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product path never calls it.  It shares no
 * code, header, table or constant with the HIP library.
 *
 * Conventions (lattice units, h = a = 1):
 *   - D3Q19 populations are stored as deviations df_i = f_i - w_i*rho0,
 *     structure-of-arrays df[i][z][y][x] (site s = (z*ny + y)*nx + x).
 *   - Vector fields are [3][N] (component-major).
 *   - Particle arrays are [np][3] (FP64).
 *   - tau is the lattice relaxation time tau_LB = tau_paper + h/2, so the
 *     full-step BGK rate is lambda = 1/tau (Sec. 3.2, Eq. collision-operator).
 *
 * The only readings of the paper this file takes are listed beside the
 * function they affect.
 */
#ifndef LBO_H
#define LBO_H
#include <stdint.h>

#define LBO_Q 19

enum { LBO_BGK = 0, LBO_TRT = 1, LBO_MRT = 2 };
enum { LBO_NONE = 0, LBO_FC = 1, LBO_EBF = 2, LBO_IB = 3 };
enum { LBO_HARMONIC = 0, LBO_FENE = 1 };

typedef struct lbo_cfg {
  int nx, ny, nz;
  int wall_y;            /* 1: halfway bounce-back walls at y=-1/2 and y=ny-1/2 */
  double tau;            /* tau_LB, must be > 1/2 */
  double rho0;
  double fext[3];        /* constant body-force density */
  int collision;         /* LBO_BGK, LBO_TRT (MRT with two rates) or LBO_MRT (a rate per
                            moment group, see mrt_rates) */
  double magic;          /* TRT magic parameter (1/lp - 1/2)(1/lm - 1/2) */
  int coupling;          /* LBO_NONE, LBO_FC, LBO_EBF (modified EBF), LBO_IB */
  double gamma;          /* friction for FC / EBF */
  int kernel;            /* 2, 3 or 4 point delta function */
  int mts_n;             /* 0: Alg. 3 ordering; n>0: n sub-steps per side (see mts_inside) */
  /* intrinsic forces */
  int nbond;
  const int32_t *bond_pairs;   /* [nbond][2] */
  double bond_k, bond_r0;
  int bond_type;               /* LBO_HARMONIC or LBO_FENE (r0 = maximum extension) */
  int nshell, shell_size;      /* markers i*shell_size .. (i+1)*shell_size-1 form shell i */
  const double *shell_template;/* [shell_size][3], centred on the origin */
  double tether_k;
  int csc;                     /* 1: collide-stream-collide form C^1/2 S C^1/2 with
                                  1 - lambda_1/2 = sqrt(1 - lambda) (needs all rates <= 1) */
  int mts_inside;              /* with mts_n > 0: 0 the coupling outside the sub-steps
                                  (Sec. 6, second decomposition); 1 the coupling inside every
                                  sub-step (Eq. multistep), 2n coupling evaluations per step */
  double kT;                   /* thermal energy k_B T; 0: no fluctuations.  > 0: the
                                  fluctuating collision (Eq. mrt-fluct) and, for FC, the random
                                  force zeta of Eq. viscous-coupling */
  uint64_t seed;               /* key of the counter-based generator */
  int64_t step0;               /* index of the first step of a run in the random streams */
  double mrt_rates[5];         /* LBO_MRT: rates of the bulk stress, the vector and the
                                  pseudo-vector third-order ghosts, the scalar and the tensor
                                  fourth-order ghosts (the shear stress relaxes at 1/tau) */
  int order;                   /* TEST ONLY, the orderings the second-order pins are checked
                                  against: 0 the second-order splitting (Eq. fc-splitting in
                                  the order of Alg. 3; Eq. IBM-scheme in the order of Alg. 2);
                                  1 the first-order sequence P S C F that Sec. 5.1 contrasts it
                                  with (full-step force and coupling, collision, streaming,
                                  full-step position update); 2 a planted mistake: FC/EBF with
                                  the final P^1/2 moved before the second coupling half, IB
                                  without the predictor (forces and interpolation at X(t)) */
} lbo_cfg;

/* lattice and local operators */
int lbo_d3q19(int32_t c[LBO_Q * 3], double w[LBO_Q], int32_t opp[LBO_Q]);
void lbo_feq_dev(double drho, double rho, const double u[3], double out[LBO_Q]);
void lbo_force_term(const double u[3], const double F[3], double G[LBO_Q]);
void lbo_mrt_basis(double E[LBO_Q * LBO_Q], double b[LBO_Q]);
void lbo_group_basis(double E[LBO_Q * LBO_Q], double b[LBO_Q]);
void lbo_rates(const lbo_cfg *cfg, double lam[LBO_Q]);
void lbo_collide_site(const lbo_cfg *cfg, double df[LBO_Q]);

/* lattice-wide operators */
void lbo_init_fluid(const lbo_cfg *cfg, double *df, const double *rho /*nullable*/,
                    const double *u /*nullable [3][N]*/);
void lbo_moments(const lbo_cfg *cfg, const double *df, double *rho, double *u);
void lbo_force_half(const lbo_cfg *cfg, double *df, const double *Fc /*nullable [3][N]*/);
void lbo_force_dt(const lbo_cfg *cfg, double *df, const double *Fc /*nullable*/, double dt);
void lbo_collide(const lbo_cfg *cfg, double *df);
void lbo_collide_half(const lbo_cfg *cfg, double *df);
void lbo_stress(const lbo_cfg *cfg, const double *df, double *pi /*[6][N]: xx yy zz xy xz yz*/);
void lbo_stream(const lbo_cfg *cfg, const double *src, double *dst);

/* delta functions, interpolation and spreading */
double lbo_phi(int kernel, double r);
void lbo_interp(const lbo_cfg *cfg, int np, const double *pos, const double *rho,
                const double *u, double *rho_p, double *u_p);
void lbo_spread(const lbo_cfg *cfg, int np, const double *pos, const double *Fp,
                double *Fgrid);

/* counter-based random numbers: Philox4x32-10 and Box-Muller normal deviates */
void lbo_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void lbo_normals4(const uint32_t ctr[4], const uint32_t key[2], double g[4]);
void lbo_site_normals(const lbo_cfg *cfg, int64_t step, uint32_t site, double g[LBO_Q]);
void lbo_collide_noisy(const lbo_cfg *cfg, double *df, int64_t step);

/* coupling forces (one half step of length hh) */
void lbo_fc_force(double gamma, double m, double rho_p, double hh, const double v[3],
                  const double u_p[3], const double Fint[3], double Fh[3]);
void lbo_ebf_update(double gamma, double m, double rho_p, double hh, const double v[3],
                    const double u_p[3], const double Fint[3], double Fh[3],
                    double v_new[3]);

/* intrinsic forces */
void lbo_bond_forces(const lbo_cfg *cfg, int np, const double *pos, double *F);
void lbo_tether_forces(const lbo_cfg *cfg, const double *pos, double *F,
                       double *rot /*nullable [nshell][9]*/);
void lbo_intrinsic(const lbo_cfg *cfg, int np, const double *pos, double *F);

/* one full time step and run of n steps */
int lbo_step(const lbo_cfg *cfg, double *df, int np, double *pos, double *vel,
             const double *mass);
int lbo_run(const lbo_cfg *cfg, int nsteps, double *df, int np, double *pos,
            double *vel, const double *mass);

/* physical moments and conserved totals (mass, fluid momentum, particle momentum) */
void lbo_totals(const lbo_cfg *cfg, const double *df, int np, const double *vel,
                const double *mass, double out[7]);
int lbo_threads(void);

#endif
