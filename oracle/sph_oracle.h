/*
 * sph_oracle.h -- interface of the FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle is the plain, slow, single-threaded
 * statement of what the total-Lagrangian SPH multi-time-step hot path
 * computes.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the GPU library never does, and the two share no
 * code, header, table or constant.
 *
 * Built twice from one source: `liboracle.so` with `real` = double, and
 * `liboracle_cs.so` with `real` = double _Complex (ORC_COMPLEX), which turns
 * the same code into a complex-step derivative oracle: perturb one parameter
 * by i*eps, and Im(result)/eps is its exact derivative (Squire & Trapp 1998).
 * Geometry (positions, volumes, kernel, correction matrices, schedules) is
 * always real; material parameters and the evolving state are `real`.
 *
 * All state arrays are structure-of-arrays, [component][n], in the
 * cell-sorted particle order the build defines (perm[s] = input id of
 * sorted particle s).
 */
#ifndef SPH_ORACLE_H
#define SPH_ORACLE_H
#include <stdint.h>

#ifdef ORC_COMPLEX
#include <complex.h>
typedef double _Complex real;
#else
typedef double real;
#endif

#define ORC_FIXED 1u  /* kinematically constrained: velocity held in the inner loop */
#define ORC_CDIR  2u  /* concentration Dirichlet particle                          */
#define ORC_GRIP  4u  /* receives prescribed displacement increments (loading)     */

enum { ORC_LE = 0, ORC_NH = 1, ORC_J2 = 2 };
enum { ORC_LOAD = 0, ORC_DIFFUSION = 1, ORC_DIFFUSION_COUPLED = 2 };

typedef struct {
  int32_t model;              /* ORC_LE / ORC_NH / ORC_J2 */
  int32_t pad_;
  real E;                     /* Young's modulus */
  double nu;                  /* Poisson ratio */
  double rho0;                /* reference density */
  real sigma0, sigma_inf, delta, H;  /* hardening law k(alpha) */
  real C_swell;               /* fluid-pressure coefficient C */
  double c0;                  /* initial saturation */
  double rho_l0;              /* fluid reference density (mixture momentum); 0: dry solid */
} orc_material;

typedef struct {
  int32_t n_slow;
  int32_t slow_kind;          /* ORC_LOAD / ORC_DIFFUSION / ORC_DIFFUSION_COUPLED */
  double dt_slow;             /* loading step; for diffusion <=0 means 0.5 h^2/D */
  double dt_s;                /* <=0 means 0.6 h / sqrt(K/rho0) */
  double eta;                 /* damping viscosity */
  int64_t k_max;              /* <=0 means k0 = floor(dt_slow/dt_s)+1 */
  int64_t fixed_inner;        /* >0: exactly this many inner steps per slow step */
  double ke_tol;              /* absolute kinetic-energy threshold */
  real D;                     /* diffusion coefficient */
  double c_bc;                /* Dirichlet saturation */
  int32_t nonlinear;          /* coupled diffusion: flux -D a grad a (1) or -D grad a (0) */
  int32_t pad2_;
} orc_cfg;

typedef struct orc_sys orc_sys;

/* kernel function (Wendland C2, support 2h) */
double orc_kernel_W(int dim, double h, double r);
double orc_kernel_dW_over_r(int dim, double h, double r);

/* build: grid, sort, neighbour lists, correction matrices, damping schedule */
orc_sys* orc_create(int dim, int64_t n, const double* X_id, const double* V_id, double h, int* err);
void orc_destroy(orc_sys* s);
/* sizes: n, n_pairs, n_upairs, n_cells, ncell[0..2], n_anchors, max_level, max_deg */
void orc_sizes(const orc_sys* s, int64_t out[10]);
void orc_grid(const orc_sys* s, double origin[3], double* inv_rc);
void orc_get_build(const orc_sys* s, uint32_t* key, uint32_t* perm, uint32_t* cell_start,
                   int64_t* nbr_off, uint32_t* nbr_idx, double* X, double* V, double* B0);
void orc_get_schedule(const orc_sys* s, uint32_t* pa, uint32_t* pb, uint32_t* plevel,
                      uint32_t* anchor_key, int64_t* anchor_off, uint32_t* anchor_nlev,
                      int64_t* color_off);

/* one-particle constitutive update from H = F - I (3x3 row-major); plastic7 =
 * (Cbar_p^-1 - I: xx yy zz xy yz xz, alpha); returns 0, or -4 if the
 * return-mapping Newton iteration fails */
int orc_constitutive(const orc_material* m, const real* H, real* plastic7, real p, real* P);

/* inner-step pieces */
void orc_displacement_gradient(const orc_sys* s, const real* u, real* H9);
int orc_stress(const orc_sys* s, const orc_material* m, const real* H9, real* plastic,
               const real* p, real* P9, real* PB);
/* mixture momentum flux (Sec. 2.2.1, Sec. 3.2): PB_a -= rho_l0 v^l_a (x) Q_a B0_a */
void orc_mixture_flux(const orc_sys* s, const orc_material* m, const real* H9, const real* v,
                      const real* c, const real* q, real* PB);
void orc_momentum(const orc_sys* s, const orc_material* m, const real* PB, const real* c, real* acc);
/* c, q (optional): content and reference flux of the last slow step; with
   m->rho_l0 > 0 they give the mixture terms */
int orc_solid_step(const orc_sys* s, const orc_material* m, double dt, const real* u, real* v,
                   real* plastic, const real* p, const uint8_t* flags, real* PB, real* acc,
                   const real* c, const real* q);
void orc_damping_sweep(const orc_sys* s, double rho0, double eta, double dt, real* v,
                       const uint8_t* flags, double rho_l0, const real* c);
real orc_drift_ke(const orc_sys* s, double rho0, double dt, real* u, const real* v,
                  const uint8_t* flags, double rho_l0, const real* c);
/* slow steps */
void orc_load_step(const orc_sys* s, double dt_l, real* u, const real* vgrip, const uint8_t* flags);
void orc_diffusion_step(const orc_sys* s, real D, double dt_d, double c_bc, real C_swell,
                        double c0, real* c, real* q, real* p, const uint8_t* flags);
/* two-way coupled form: c is the fluid content per reference volume, the
 * saturation a = c / J follows the deformation u; q receives the reference
 * flux J F^-1 q */
void orc_diffusion_step_coupled(const orc_sys* s, real D, double dt_d, double c_bc, real C_swell,
                                double c0, int nonlinear, const real* u, real* c, real* q, real* p,
                                const uint8_t* flags);
/* step sizes of Sec. 4.1: dt_s = 0.6 h / sqrt(K / rho0) (eq. dts-advection at
   rest) and dt_d = 0.5 h^2 / D (0 for D <= 0); either output may be NULL */
void orc_default_steps(const orc_sys* s, const orc_material* m, double D, double* dt_s,
                       double* dt_d);
/* multi-time-step driver; k_sched (optional) freezes the inner counts;
   acc_out (optional, [d][n]) receives the momentum sum per unit mass of the
   last inner step, fixed particles included (their reaction) */
int orc_advance(const orc_sys* s, const orc_material* m, const orc_cfg* cfg, real* u, real* v,
                real* plastic, real* c, real* q, real* p, const real* vgrip,
                const uint8_t* flags, const int64_t* k_sched, int64_t* k_out, double* ke_out,
                int32_t* conv_out, real* acc_out);
#endif
