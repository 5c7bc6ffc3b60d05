/*
 * sph.h -- C ABI of the MI355X (gfx950) library for the fast process of
 * total-Lagrangian SPH solid dynamic relaxation inside an explicit
 * multi-time-step scheme (Tang, Wu, Wang, Haidn, Hu, arXiv 2309.04010), with
 * the slow processes beside it: displacement loading, the SPH diffusion
 * update (one-way, or two-way coupled to the deformation), and, optionally,
 * the momentum of the fluid in a saturated solid (sph_material.rho_l0).
 *
 * Conventions
 *  - Every function returns int: SPH_OK (0), a negative SPH_E_* error, or the
 *    positive warning SPH_W_NOT_CONVERGED.  No exception crosses the ABI.
 *    sph_last_error() returns a thread-local description of the last error.
 *  - All array arguments are DEVICE pointers unless marked "host".  Arrays are
 *    structure-of-arrays [component][n], contiguous, in the cell-sorted
 *    particle order fixed by sph_build_neighbors (perm[s] = input index of
 *    sorted particle s).  Matrices per particle are row-major d x d.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on that stream unless stated otherwise.
 *  - Precision: sph_state.prec selects the element type (float or double) of
 *    v, PB, plastic, c, q, p, acc and vgrip.  Displacements u, the kinetic
 *    energy and all reductions are always double.
 *  - Ownership: the neighbour handle owns its device memory (allocated once,
 *    at build time).  State arrays belong to the caller.  Stepping functions
 *    allocate nothing.  Two calls that use the same handle must not overlap
 *    in time (they share the handle's small control block).
 *  - Device-side faults (non-finite kinetic energy, return-mapping Newton
 *    failure, singular correction matrix) are latched in the handle's status
 *    word and reported by the next synchronising call (sph_status,
 *    sph_advance_multirate, sph_build_neighbors) as SPH_E_NUMERIC.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPH_OK 0
#define SPH_E_ARG (-1)         /* invalid argument (null pointer, bad size) */
#define SPH_E_CAPACITY (-2)    /* a structural limit of the build was exceeded */
#define SPH_E_DEVICE (-3)      /* HIP runtime error */
#define SPH_E_NUMERIC (-4)     /* NaN/Inf, singular B0, Newton failure */
#define SPH_E_UNSUPPORTED (-5) /* unsupported dimension / model / precision */
#define SPH_W_NOT_CONVERGED 1  /* an inner loop hit its step cap */

#define SPH_F32 0
#define SPH_F64 1

#define SPH_MODEL_LE 0 /* small-strain linear elastic (plane strain in 2D) */
#define SPH_MODEL_NH 1 /* neo-Hookean, App. A.2 eq. (kirchoff_stress_equation) */
#define SPH_MODEL_J2 2 /* J2 return mapping, App. A.4 Algorithm 1 */

#define SPH_SLOW_LOAD 0      /* slow step = prescribed grip displacement increment */
#define SPH_SLOW_DIFFUSION 1 /* slow step = SPH diffusion of the saturation */
#define SPH_SLOW_DIFFUSION_COUPLED 2 /* slow step = two-way coupled diffusion (sph_diffusion_step_coupled) */

/* per-particle flag bits (uint8) */
#define SPH_FLAG_FIXED 1u /* velocity held (zero) in the inner loop; infinite mass in damping */
#define SPH_FLAG_CDIR 2u  /* saturation reset to c_bc after every diffusion step */
#define SPH_FLAG_GRIP 4u  /* u += dt_slow * vgrip at every loading step */

/* status bits latched on the device */
#define SPH_STATUS_NONFINITE 1
#define SPH_STATUS_NEWTON 2
#define SPH_STATUS_SINGULAR_B0 4

typedef struct sph_nbr sph_nbr; /* opaque: fixed neighbourhood + schedule */

/* Read-only view of a built neighbourhood (device pointers owned by the
 * handle; valid until sph_nbr_destroy). */
typedef struct {
  int32_t dim;
  int32_t n_colors;        /* 2^dim cell-parity colours of the damping sweep */
  int64_t n;               /* particles */
  int64_t n_pairs;         /* directed neighbour pairs (CSR length) */
  int64_t n_upairs;        /* undirected pairs = n_pairs / 2 */
  int64_t n_cells;         /* cells of edge 2h */
  int64_t ncell[3];        /* cells per axis (1 for unused axes) */
  int64_t n_anchors;       /* cells that anchor at least one pair */
  int64_t max_deg;         /* largest neighbour count */
  int64_t max_level;       /* largest number of levels of one anchor */
  int64_t color_off[9];    /* host: anchors of colour k are [color_off[k], color_off[k+1]) */
  double origin[3];        /* cell-grid origin (the cloud is centred in the grid) */
  double h;                /* smoothing length; support radius 2h */
  double inv_rc;           /* 1/(2h), as used for the cell keys */
  const uint32_t* key;     /* [n] cell key of each sorted particle */
  const uint32_t* perm;    /* [n] sorted position -> input index */
  const uint32_t* cell_start; /* [n_cells+1] first sorted particle of each cell */
  const int64_t* nbr_off;  /* [n+1] CSR offsets */
  const uint32_t* nbr_idx; /* [n_pairs] neighbours, ascending sorted position */
  const double* X;         /* [dim][n] sorted reference positions */
  const double* V;         /* [n] sorted reference volumes */
  const double* B0;        /* [dim*dim][n] correction matrices (FP64) */
  const uint32_t* sched_a; /* [n_upairs] damping pairs in canonical order: smaller index */
  const uint32_t* sched_b; /* [n_upairs] larger index */
  const uint32_t* sched_level; /* [n_upairs] level of the pair within its anchor */
  const uint32_t* anchor_key;  /* [n_anchors] anchor cells, by (colour, key) */
  const int64_t* anchor_off;   /* [n_anchors+1] pair range of each anchor */
  const uint32_t* anchor_nlev; /* [n_anchors] levels per anchor */
} sph_nbr_info;

typedef struct {
  int32_t model; /* SPH_MODEL_* */
  int32_t pad_;
  double E;      /* Young's modulus; mu = E/(2(1+nu)), K = E/(3(1-2nu)) (eq. relation-modulus) */
  double nu;     /* Poisson ratio */
  double rho0;   /* reference density (TL momentum uses rho0, eq. mechanical-mom) */
  double sigma0, sigma_inf, delta, H; /* hardening k(a) = s0 + (sinf-s0)(1-exp(-delta a)) + H a (App. A.3) */
  double C_swell; /* fluid-pressure coefficient: p = C (c - c0), eq. (fluid_pressure) */
  double c0;      /* initial saturation */
  double rho_l0;  /* fluid reference density (Sec. 2.2.1, rho^l = rho^l_0 times the content);
                     0: a dry solid.  > 0 turns on the mixture momentum of the inner step,
                     which needs the state's c and q (the content and the reference flux Q
                     the last slow step left):
                       PB_a -= rho_l0 v^l_a (x) Q_a B0_a,  v^l = v + F Q / c (c > 0),
                     the fluid's momentum flux v^l (x) q of eq. (totalmomentumupdatesph) as
                     a Piola tensor; the inertia of the kick, the damping sweep's masses
                     and the kinetic energy become (rho0 + rho_l0 c_a) V_a.  The time step
                     stays 0.6 h / sqrt(K / rho0).  The reverse pass refuses a
                     mixture (SPH_E_UNSUPPORTED). */
} sph_material;

typedef struct {
  int32_t prec;  /* SPH_F32 or SPH_F64: element type of the void* arrays below */
  int32_t pad_;
  double* u;     /* [dim][n] displacement, always FP64 */
  void* v;       /* [dim][n] velocity */
  void* PB;      /* [dim*dim][n] P B0 (written by the stress stage, read by momentum) */
  void* plastic; /* [7][n] J2 state: Cbar_p^-1 - I (xx,yy,zz,xy,yz,xz) and alpha (zeros = virgin
                    material); NULL unless J2 */
  void* c;       /* [n] saturation (diffusion) or NULL */
  void* q;       /* [dim][n] flux scratch of the diffusion step or NULL */
  void* p;       /* [n] fluid pressure used by the stress stage, or NULL (no swelling) */
  void* acc;     /* [dim][n] optional output: acceleration before the kick, or NULL */
  void* vgrip;   /* [dim][n] prescribed grip velocity for loading steps, or NULL */
  const uint8_t* flags; /* [n] SPH_FLAG_* bits, or NULL (all free) */
} sph_state;

typedef struct {
  int32_t n_slow;      /* outer (slow) steps */
  int32_t slow_kind;   /* SPH_SLOW_LOAD / SPH_SLOW_DIFFUSION / SPH_SLOW_DIFFUSION_COUPLED */
  double dt_slow;      /* loading step; diffusion: <= 0 selects 0.5 h^2 / D (Sec. 4.1) */
  double dt_s;         /* inner step; <= 0 selects 0.6 h / sqrt(K/rho0) (eq. dts-advection at rest) */
  double eta;          /* damping viscosity (eq. damping-sph) */
  int64_t k_max;       /* inner cap; <= 0 selects k0 = floor(dt_slow/dt_s) + 1 (Sec. 4.2) */
  int64_t fixed_inner; /* > 0: exactly this many inner steps, no kinetic-energy exit */
  double ke_tol;       /* absolute kinetic-energy threshold of the early exit */
  double D;            /* diffusion coefficient */
  double c_bc;         /* Dirichlet saturation */
  int32_t chunk;       /* most inner steps launched between host polls (<= 0: 64);
                          an adaptive run polls first after min(chunk, 16) steps and
                          doubles the interval after each poll, up to chunk */
  int32_t use_graph;   /* 1: replay the inner steps as a captured hipGraph of one
                          chunk, or in an adaptive run of min(chunk, 16) steps
                          launched as often as each interval needs; the graph
                          stays on the handle for later calls with the same
                          arguments */
  const int64_t* k_sched; /* host, optional [n_slow]: frozen inner counts */
  const struct sph_batch* batch; /* optional: per-specimen parameters (see sph_build_neighbors_batched) */
  int32_t diff_nonlinear; /* SPH_SLOW_DIFFUSION_COUPLED: flux -D a grad a (1) or -D grad a (0) */
  int32_t pad2_;
} sph_multirate_cfg;

typedef struct {
  int64_t* k;          /* host [n_slow] (or NULL): inner steps taken per slow step */
  double* ke;          /* host [n_slow] (or NULL): kinetic energy after the last inner step */
  int32_t* converged;  /* host [n_slow] (or NULL): 1 if ke <= ke_tol at the end */
  double dt_s;         /* out: inner step used */
  double dt_slow;      /* out: slow step used */
  int64_t k_max;       /* out: inner cap used */
  int64_t total_inner; /* out: sum of k */
} sph_report;

/* ------------------------------------------------------------------------
 * Fixed neighbourhood (Sec. 3.1: in the total-Lagrangian form the neighbour
 * set and the correction matrix B0 of eq. (sph-correctmatrix) are built once
 * in the initial configuration).
 *   X [dim][n], V [n]: device FP64 reference positions and volumes, input order.
 *   h: smoothing length; neighbours are b != a with |X_a - X_b|^2 < (2h)^2
 *      (FP64, no fused multiply-add), found in cells of edge 2h: per axis
 *      nc = floor(extent / 2h) + 1 cells, the cloud centred in the grid,
 *      cell index floor((X - origin) / 2h) clamped to [0, nc-1].  Particles
 *      are stably sorted by cell key (x fastest); lists are in ascending
 *      sorted position.
 *   Damping schedule: each unordered pair {a < b} is anchored at a cell A
 *   whose block A .. A+1 holds both particles: per axis, the lower of the two
 *   cells where they differ; where both sit in cell c, c - 1 if c >= 1 and
 *   bit k (the axis index) of a + b is set, else c (a, b counted from the
 *   specimen's first sorted position); along an axis only two cells deep,
 *   the first cell (the block then spans that axis, and the colours odd
 *   along it stay empty).  The pair is coloured by the parity of
 *   its anchor (2^dim colours, so anchors of one colour touch disjoint
 *   2^dim-cell blocks); within an anchor, pairs in ascending (a, b) take the
 *   smallest level not used by an earlier pair sharing a particle.
 *   Synchronous.  On success *out receives a new handle.
 *   Errors: SPH_E_ARG, SPH_E_UNSUPPORTED (dim not 2/3), SPH_E_CAPACITY (more
 *   than 2^32-16 cells, 2^31 pairs, or an anchor block too dense for the level
 *   builder), SPH_E_NUMERIC (singular correction matrix), SPH_E_DEVICE. */
int sph_build_neighbors(int dim, int64_t n, const double* X, const double* V, double h,
                        void* stream, sph_nbr** out);
int sph_nbr_destroy(sph_nbr* nbr);
int sph_nbr_query(const sph_nbr* nbr, sph_nbr_info* info);

/* Device scratch of the per-step calls (the boundary's workspace): the
 * per-run damping records and inverse masses of both precisions (Sec. 4.3),
 * the block partials of the kinetic-energy reduction (Sec. 4.2) and of the
 * parameter gradients.  The handle allocates it when it is built; no
 * per-step call allocates.  A caller that manages device memory itself (a
 * pool, memory shared with other work) can hand its own in:
 * sph_workspace_size writes the bytes needed to *bytes (fixed for the
 * handle); sph_set_workspace makes the handle use [ws, ws + bytes) from then
 * on and frees the handle's own block, or, with ws = NULL, allocates a block
 * of its own again.  ws: device memory on the handle's device, 256-byte
 * aligned, at least sph_workspace_size bytes, not used by anything else
 * (another handle included) while this handle uses it, and kept until the
 * handle is destroyed or given another workspace; its contents are the
 * library's.  The call waits for `stream`, and for the device, so no call of
 * the handle may still run; it zeroes the gradient partials, marks the
 * damping records for re-computation (the next damping call lays them out)
 * and drops the cached graphs (the whole-run graph and the chunk graph of
 * sph_advance_multirate), which point into the old block.  Synchronous.
 * Errors: SPH_E_ARG
 * (NULL handle or bytes, ws misaligned or smaller than needed),
 * SPH_E_DEVICE. */
int sph_workspace_size(const sph_nbr* nbr, int64_t* bytes);
int sph_set_workspace(sph_nbr* nbr, void* ws, int64_t bytes, void* stream);

/* ------------------------------------------------------------------------
 * One solid stage of an inner step (Sec. 3.1): deformation gradient from u
 *   F_a = I + (sum_b V_b (u_b - u_a) (x) grad_a W_ab) B0_a
 * (eq. deformationtensor-displacement with the corrected gradient; the exact
 * time integral of eq. rate_F), the first Piola-Kirchhoff stress of the
 * material model with the fluid-pressure term P -= J p F^-T (App. B.2),
 * PB = P B0, the pair-averaged momentum sum of eq. (sph-mechanical-mom)
 *   a_a = (1/rho0) sum_b V_b (PB_a + PB_b) grad_a W_ab,
 * and the kick v += dt_s a for particles without SPH_FLAG_FIXED.
 * J2 state in `plastic` is committed.  Asynchronous. */
int sph_solid_relax_step(const sph_nbr* nbr, const sph_material* mat, const sph_state* st,
                         double dt_s, void* stream);

/* Implicit pairwise-splitting sweep of the viscous damping term (Sec. 4.3,
 * eq. damping-sph): for every pair in canonical order (colour, anchor, level)
 *   beta = 2 eta V_a V_b (dW/dr / r) dt_s,
 *   delta = beta (v_a - v_b) / (m_a m_b - beta (m_a + m_b)),
 *   v_a += m_b delta, v_b -= m_a delta,
 * with a fixed particle acting as infinite mass.  Pairs of one level of one
 * anchor are disjoint and anchors of one colour touch disjoint particles, so
 * the parallel sweep equals the sequential canonical order.  The per-pair
 * coefficients are recomputed by every call (a multi-time-step run computes
 * them once); calls on one handle must not overlap.  Asynchronous. */
int sph_damping_sweep(const sph_nbr* nbr, const sph_material* mat, const sph_state* st,
                      double eta, double dt_s, void* stream);

/* Drift and kinetic energy (Sec. 4.2): u += dt_s v for free particles, then
 * E_k = sum 1/2 rho0 V |v|^2 reduced in a fixed order (deterministic) into
 * the device double *ke_out (may be NULL).  On sets of at most 65,536
 * particles the last block of the drift kernel reduces E_k (elected through
 * a counter in the handle's control block), else a second kernel does; the
 * order of the sum, and so E_k, is the same either way.  Calls on one handle
 * must not overlap.  Asynchronous. */
int sph_drift_ke(const sph_nbr* nbr, const sph_material* mat, const sph_state* st, double dt_s,
                 double* ke_out, void* stream);

/* sph_drift_ke for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results (bitwise) as sph_drift_ke; the block
 * partials of the kinetic-energy reduction live in a static device array of
 * the library (512 KiB per GPU, kept until the process ends) instead of the
 * handle's buffer, so the call allocates nothing, and it is never timed by
 * sph_profile_enable.  Call it with the handle's device current.  Every
 * partial is written before it is read, so calls need no clearing between
 * them, but calls that overlap in time on one GPU race on that array (and,
 * on one handle, on its control block, as sph_drift_ke's do).
 * Errors: as sph_drift_ke, plus SPH_E_CAPACITY for more than 2^26
 * particles (the array's limit) and SPH_E_ARG when the current device is
 * not the handle's.  Asynchronous. */
int sph_drift_ke_noalloc(const sph_nbr* nbr, const sph_material* mat, const sph_state* st,
                         double dt_s, double* ke_out, void* stream);

/* Loading slow step: u += dt_l * vgrip for SPH_FLAG_GRIP particles.  Async. */
int sph_load_step(const sph_nbr* nbr, const sph_state* st, double dt_l, void* stream);

/* Diffusion slow step (Fick's law, eqs. grad_q and fluid_mass_der, SPH form
 * of Sec. 3.2 read as linear in the saturation c with constant D):
 *   q_a = -D B0_a sum_b V_b (c_b - c_a) grad_a W_ab,
 *   c_a += dt_d (- sum_b V_b (B0_a q_a + B0_b q_b) . grad_a W_ab),
 * then c = c_bc on SPH_FLAG_CDIR particles and p = C_swell (c - c0)
 * (eq. fluid_pressure) when st->p is not NULL.  Needs st->c and st->q.  Async. */
int sph_diffusion_step(const sph_nbr* nbr, const sph_material* mat, const sph_state* st,
                       double D, double dt_d, double c_bc, void* stream);

/* Two-way coupled diffusion slow step: the reading of eqs. grad_q,
 * fluid_mass_der, fluid_mass_sph and ralative_velocity_sph (Sec. 2.2.2, 3.2)
 * with the updated-Lagrangian kernel gradient stated after fluid_mass_sph.
 * st->c holds the fluid content per reference volume (over the reference
 * fluid density); the saturation is a = c / J, J = det F, F = I + H(st->u)
 * (eq. deformationtensor-displacement).  Then
 *   q_a = -D w_a F_a^-T B0_a sum_b V_b (a_b - a_a) grad0_a W_ab,
 *         w_a = a_a if nonlinear (eq. grad_q with rho^l = rho^l_0 a), else 1,
 *   st->q <- Q_a = J_a F_a^-1 q_a (the reference flux),
 *   c_a  += dt_d (- sum_b V_b (B0_a Q_a + B0_b Q_b) . grad0_a W_ab),
 * c = c_bc J on SPH_FLAG_CDIR particles (saturation c_bc) and
 * p = C_swell (c / J - c0).  Needs st->u, c, q, p; uses st->PB as scratch
 * (overwritten: F^-1).  With u = 0 and nonlinear = 0 it is
 * sph_diffusion_step.  Its reverse: sph_diffusion_step_coupled_vjp, and
 * inside sph_advance_multirate_backward.  Asynchronous. */
int sph_diffusion_step_coupled(const sph_nbr* nbr, const sph_material* mat, const sph_state* st,
                               double D, double dt_d, double c_bc, int32_t nonlinear, void* stream);

/* Recording of a forward multi-time-step run for the reverse pass
 * (sph_advance_multirate_backward).  All arrays are caller-owned DEVICE
 * memory except k_rec (host).  Slice l of a checkpoint array holds the state
 * at the start of slow step l (before its load or diffusion update); slice
 * n_slow holds the final state.  hist_H receives, for every inner step of one
 * slow step (the last one of the forward run, when it fits, and each slow
 * step again while the reverse pass recomputes it), the displacement gradient
 * H = F - I the stress stage formed (row-major dim x dim), hist_plastic the
 * J2 state before the step; the reverse pass differentiates the constitutive
 * update at exactly these values.  Sizes: ck_u [n_slow_cap+1][dim][n] f64,
 * ck_v [n_slow_cap+1][dim][n], ck_plastic [n_slow_cap+1][7][n] (J2 only, else
 * NULL), ck_c [n_slow_cap+1][n] (diffusion only, else NULL),
 * hist_H [k_hist_cap][dim*dim][n], hist_plastic [k_hist_cap][7][n] (J2 only,
 * else NULL); prec-typed arrays follow sph_state.prec.
 * A slow step with more inner steps than k_hist_cap is reversed in segments
 * of k_hist_cap inner steps, last segment first (two-level checkpointing):
 * the reverse pass re-runs the slow step once to store the state at the
 * start of every segment but the first in seg_u [seg_cap][dim][n] f64,
 * seg_v [seg_cap][dim][n] and seg_plastic [seg_cap][7][n] (J2 only, else
 * NULL), then re-runs each segment from there with its inner states
 * recorded.  ceil(k / k_hist_cap) - 1 <= seg_cap is required (seg_cap = 0,
 * NULL arrays: no segments, k <= k_hist_cap); the cost is one more forward
 * run of the slow step, the memory (2 dim + 7) values per particle per
 * segment instead of dim^2 + 7 per inner step.  The results equal those of
 * an unsegmented reverse pass. */
typedef struct {
  int32_t n_slow_cap;  /* slow steps that fit */
  int32_t pad_;
  int64_t k_hist_cap;  /* inner steps of one slow step that fit in hist_H */
  double* ck_u;
  void* ck_v;
  void* ck_plastic;
  void* ck_c;
  void* hist_H;
  void* hist_plastic;
  int64_t* k_rec;      /* host [n_slow_cap]: inner steps taken per slow step (out) */
  int32_t n_rec;       /* out: slow steps recorded */
  int32_t hist_slow;   /* out: slow step whose inner states hist_H holds, -1 if none */
  double dt_s;         /* out: inner step used (frozen for the reverse pass) */
  double dt_slow;      /* out: slow step used */
  int64_t seg_cap;     /* inner checkpoints that fit in seg_u, seg_v, seg_plastic */
  double* seg_u;
  void* seg_v;
  void* seg_plastic;
} sph_tape;

/* Multi-time-step driver (Sec. 4.2): for l = 1..n_slow, one slow step (load
 * or diffusion), then inner steps {solid stage, damping sweep, drift + E_k}
 * until E_k <= ke_tol, or k = k_max (warning), or exactly fixed_inner /
 * k_sched[l] steps.  The stop test runs on the device; the host polls once per
 * chunk of inner steps.  `tape` (may be NULL) records the run for the reverse
 * pass; it requires cfg->use_graph == 0 for the slow step whose inner states
 * are recorded.  Synchronous; fills the host report.  Returns SPH_OK,
 * SPH_W_NOT_CONVERGED, or an error (SPH_E_CAPACITY: n_slow > n_slow_cap). */
int sph_advance_multirate(const sph_nbr* nbr, const sph_material* mat, const sph_state* st,
                          const sph_multirate_cfg* cfg, sph_report* report, sph_tape* tape,
                          void* stream);

/* ------------------------------------------------------------------------
 * Reverse mode.  The pass runs the transposed linear maps of the inner step
 * in reverse order -- drift, damping sweep (colours, levels and pair maps
 * reversed), kick, momentum sum, stress (exact derivative of the constitutive
 * update, the J2 return mapping through the implicit-function theorem on its
 * scalar residual), displacement-gradient sum -- then the transposed slow
 * step.  The schedule (inner counts, dt_s, dt_slow) is held fixed: the
 * gradient is that of the discrete map the forward run executed.  Parameter
 * gradients accumulate in FP64, in a fixed order (deterministic). */
#define SPH_GRAD_E 0      /* Young's modulus (mu and K scale with E at fixed nu) */
#define SPH_GRAD_D 1      /* diffusion coefficient */
#define SPH_GRAD_C 2      /* fluid-pressure coefficient C_swell */
#define SPH_GRAD_S0 3     /* hardening sigma0 */
#define SPH_GRAD_SINF 4   /* hardening sigma_inf */
#define SPH_GRAD_DELTA 5  /* hardening delta */
#define SPH_GRAD_H 6      /* hardening H (linear term) */
#define SPH_NGRAD 7

/* Adjoint state: the derivative of a scalar objective with respect to each
 * state array.  Caller-owned device memory; prec as in sph_state. */
typedef struct {
  int32_t prec;
  int32_t pad_;
  double* u;      /* [dim][n] adjoint of u (FP64) */
  void* v;        /* [dim][n] adjoint of v */
  void* plastic;  /* [7][n] adjoint of the J2 state, NULL unless J2 */
  void* c;        /* [n] adjoint of the saturation, NULL without diffusion */
  double* p;      /* [n] adjoint of the fluid pressure, accumulated over the inner steps
                     of a slow step (FP64), or NULL */
  void* work;     /* [dim*dim][n] scratch */
  double* grad;   /* [SPH_NGRAD] parameter gradients, accumulated (+=) */
} sph_adjoint;

/* Reverse of sph_solid_relax_step.  Inputs: st->u and st->plastic as they
 * were BEFORE the forward step (neither is modified), st->p, st->flags;
 * adj->v = adjoint of v after the kick (unchanged: the kick passes it
 * through); adj->plastic = adjoint of the J2 state after the step, replaced
 * by the adjoint before it.  Accumulates: adj->u (+=), adj->p (+=, if not
 * NULL), adj->grad[E, S0, SINF, DELTA, H] (+=).  Uses adj->work.  Async. */
int sph_solid_relax_step_vjp(const sph_nbr* nbr, const sph_material* mat, const sph_state* st,
                             const sph_adjoint* adj, double dt_s, void* stream);

/* Reverse of sph_damping_sweep: adj->v <- S^T adj->v, S the (linear) sweep
 * map.  st supplies flags.  Async. */
int sph_damping_sweep_vjp(const sph_nbr* nbr, const sph_material* mat, const sph_state* st,
                          const sph_adjoint* adj, double eta, double dt_s, void* stream);

/* Reverse of the drift: adj->v += dt_s adj->u for free particles.  Async. */
int sph_drift_vjp(const sph_nbr* nbr, const sph_state* st, const sph_adjoint* adj, double dt_s,
                  void* stream);

/* Reverse of sph_diffusion_step.  st->c = saturation AFTER the forward step,
 * c_before = saturation before it (device, prec-typed [n]); adj->c = adjoint
 * of c after the step (replaced by the adjoint before it); adj->p = adjoint of
 * p after the step (consumed: zeroed).  Accumulates adj->grad[D, C].  Uses
 * adj->work ([dim][n]).  Async. */
int sph_diffusion_step_vjp(const sph_nbr* nbr, const sph_material* mat, const sph_state* st,
                           const void* c_before, const sph_adjoint* adj, double D, double dt_d,
                           double c_bc, void* stream);

/* Reverse of sph_diffusion_step_coupled (the same reading of Sec. 2.2.2 and
 * Sec. 3.2).  st->u = the step's displacement (the step leaves it as it is),
 * st->c = content AFTER the step, c_before = content before it (device,
 * prec-typed [n]).  adj->c = adjoint of c after the step (replaced by the
 * adjoint before it); adj->p = adjoint of p after the step (consumed:
 * zeroed); adj->u += the adjoint of u through F, J and F^-1;
 * adj->grad[D, C] accumulated.  Working storage, overwritten: st->PB, st->p,
 * st->q, the first two components of st->v and adj->work ([dim*dim][n]).
 * Errors: SPH_E_ARG (arrays missing), SPH_E_UNSUPPORTED (a mixture, or a
 * batched neighbourhood).  Async. */
int sph_diffusion_step_coupled_vjp(const sph_nbr* nbr, const sph_material* mat,
                                   const sph_state* st, const void* c_before,
                                   const sph_adjoint* adj, double D, double dt_d, double c_bc,
                                   int32_t nonlinear, void* stream);

/* Reverse pass of a taped sph_advance_multirate run with the same cfg.  On
 * entry adj->u, adj->v (and adj->plastic, adj->c) hold the adjoint of the
 * final state; on return they hold the adjoint of the initial state and
 * adj->grad has the parameter gradients added.  The pass re-runs each slow
 * step from its checkpoint (recording its inner states, in segments when
 * k_rec[l] > k_hist_cap) unless hist_H already holds it; st is used as working
 * storage and restored to the final state on return.  adj->p must be zero on
 * entry.  Slow steps: loading, diffusion, and the two-way coupled diffusion
 * (one specimen; its u-dependence through F, J and F^-1 goes to adj->u).
 * Synchronous.  Errors: SPH_E_ARG (tape incomplete), SPH_E_CAPACITY,
 * SPH_E_UNSUPPORTED (a mixture, or a batched coupled run). */
int sph_advance_multirate_backward(const sph_nbr* nbr, const sph_material* mat,
                                   const sph_state* st, const sph_multirate_cfg* cfg,
                                   sph_tape* tape, const sph_adjoint* adj, void* stream);

/* Point evaluation of the constitutive update (App. A) and its reverse, per
 * particle, for n independent particles: H [9][n] = F - I (row-major 3x3),
 * plastic [7][n] (J2, updated in place by sph_constitutive; read-only in the
 * vjp), p [n] or NULL, P [9][n] first Piola-Kirchhoff stress.  The vjp takes
 * Pbar [9][n] and plastic_bar [7][n] (adjoint of the updated state; replaced
 * by the adjoint of the state before) and writes Hbar [9][n], pbar [n] and
 * theta_bar [5][n] (per-particle derivatives with respect to E, sigma0,
 * sigma_inf, delta, H).  prec-typed arrays.  Async. */
int sph_constitutive(const sph_material* mat, int prec, int64_t n, const void* H, void* plastic,
                     const void* p, void* P, void* stream);
int sph_constitutive_vjp(const sph_material* mat, int prec, int64_t n, const void* H,
                         const void* plastic, const void* p, const void* Pbar, void* plastic_bar,
                         void* Hbar, void* pbar, void* theta_bar, void* stream);

/* ------------------------------------------------------------------------
 * Batches of independent specimens (parameter sweeps).  Several specimens
 * share one particle set and one neighbour handle, and every kernel runs over
 * all of them in a single launch.  Each specimen gets its own segment of the
 * cell grid -- its own origin and cell counts, cell keys offset by those of
 * the specimens before it -- so its cells, sorted order, neighbour lists,
 * correction matrices and damping order are exactly those it has when built
 * alone, and specimens may overlap in space.  Per-specimen scalars come from
 * small device tables indexed by each particle's specimen id.
 *
 * sph_build_neighbors_batched: as sph_build_neighbors, with spec_id [n]
 * (device int32, input order) assigning particles to specimens 0..n_spec-1 in
 * contiguous ascending runs.  Sorted positions then hold specimen after
 * specimen.  With n_spec == 1 it is sph_build_neighbors.  Errors as
 * sph_build_neighbors, plus SPH_E_ARG for ids that are not contiguous
 * ascending runs and SPH_E_CAPACITY for more than 65535 specimens. */
int sph_build_neighbors_batched(int dim, int64_t n, const double* X, const double* V, double h,
                                int32_t n_spec, const int32_t* spec_id, void* stream,
                                sph_nbr** out);

/* Per-specimen values that replace the uniform ones of sph_material (E) and
 * sph_multirate_cfg (D, dt_s, dt_slow) when cfg->batch is set.  Host arrays of
 * n_spec doubles, copied to the device at the start of each run; dt_s and
 * dt_slow may be NULL, and entries <= 0 take each specimen's
 * sph_default_steps (the diffusion step from its own D).  The other
 * material and schedule values are shared by all specimens.  A batched run
 * needs fixed inner counts (fixed_inner or k_sched): one specimen's kinetic
 * energy does not decide another's stop.  `grad` (device [n_spec][SPH_NGRAD],
 * may be NULL) receives the reverse pass's per-specimen gradients (+=). */
typedef struct sph_batch {
  int32_t n_spec;
  int32_t pad_;
  const double* E;
  const double* D;
  const double* dt_s;
  const double* dt_slow;
  double* grad;
} sph_batch;

/* Forward run, and the reverse pass when adj is not NULL, recorded as ONE
 * hipGraph and launched once; the instantiated graph is kept in the handle
 * and launched again while the arguments (the structures' contents) stay
 * the same -- per-specimen values may change between launches.  Needs fixed
 * inner counts and a tape whose k_hist_cap covers one slow step's inner
 * count.  Results equal the eager
 * sph_advance_multirate + sph_advance_multirate_backward bitwise.
 * Synchronous.  Fills the report's counts. */
int sph_advance_multirate_graph(const sph_nbr* nbr, const sph_material* mat, const sph_state* st,
                                const sph_multirate_cfg* cfg, sph_report* report, sph_tape* tape,
                                const sph_adjoint* adj, void* stream);

/* ------------------------------------------------------------------------
 * Launch shapes.  The tiled gather kernels split each particle's neighbour
 * list over 1, 2 or 4 lanes; the damping pass gives each anchor 8, 16, 32
 * or 64 lanes.  The fastest choice depends on the particle set and precision.
 * sph_autotune times every candidate on this handle's data (HIP events, a
 * few launches each, on scratch copies of v, PB and the J2 state: st is not
 * modified) and keeps the fastest for st->prec; later launches use them.
 * A damping width is timed on its own colour's pass, with events around that
 * pass inside whole sweeps, so that the other colours' records pass through
 * the caches between its timings as in a run.
 * with_adjoint also tunes the reverse kernels.  eta and dt_s are those of the
 * runs to come.  Synchronous; allocates scratch for its own duration.
 * sph_set_tuning / sph_get_tuning write and read the choices directly
 * (damp_lanes 0 = automatic: 16, widened while a wavefront's anchors would
 * exceed the LDS).  damp_idle chooses what the lanes of a damping row
 * without a pair do: 1 = update a spare slot with a zero coefficient (no
 * branch: shorter rows, for passes of few wavefronts), 2 = skip the row's LDS
 * work (a branch: less LDS traffic, for passes of many wavefronts), 0 =
 * automatic (2 from 512 wavefronts a pass up); the results are the same.
 * sph_autotune sets it to automatic: its repeated sweeps over the same data
 * keep the records in the last-level cache, where the two forms time alike. */
typedef struct {
  int32_t lpp_stress;      /* 1, 2, 4 */
  int32_t lpp_momentum;    /* 1, 2, 4 */
  int32_t lpp_adj_stress;  /* 1, 2, 4 */
  int32_t lpp_adj_gather;  /* 1, 2, 4 */
  int32_t damp_lanes[8];   /* per colour: 0, 8, 16, 32, 64 */
  int32_t damp_idle[8];    /* per colour: 0, 1, 2 */
  double ms_solid, ms_adjoint, ms_damping_sweep; /* out: best times of sph_autotune
                                                    (the sweep's: the sum of its passes') */
} sph_tuning;
int sph_autotune(sph_nbr* nbr, const sph_material* mat, const sph_state* st, double eta,
                 double dt_s, int with_adjoint, sph_tuning* out, void* stream);
int sph_set_tuning(sph_nbr* nbr, int prec, const sph_tuning* tuning);
int sph_get_tuning(const sph_nbr* nbr, int prec, sph_tuning* tuning);

/* Step sizes of Sec. 4.1 for smoothing length h and a material: the fast
 * (stress-relaxation) step of eq. (dts-advection) at rest, where only the
 * sound-speed term remains,
 *   dt_s = 0.6 h / sqrt(K / rho0),  K = E / (3 (1 - 2 nu))  (eq. relation-modulus),
 * and the explicit diffusion step dt_d = 0.5 h^2 / D (0 for D <= 0).  These
 * are the defaults sph_advance_multirate takes for cfg->dt_s <= 0 and
 * cfg->dt_slow <= 0, and the per-specimen defaults of sph_batch.  Host
 * outputs (either may be NULL); a pure host computation, no device call.
 * Errors: SPH_E_ARG (h <= 0, E <= 0, rho0 <= 0 or nu >= 1/2). */
int sph_default_steps(double h, const sph_material* mat, double D, double* dt_s, double* dt_d);

/* Synchronise `stream` and return (and clear) the latched status bits in
 * *status_bits (may be NULL): SPH_OK, or SPH_E_NUMERIC if any bit was set. */
int sph_status(const sph_nbr* nbr, void* stream, int32_t* status_bits);

/* Per-kernel timing with HIP events recorded on the launch stream around
 * every kernel the handle launches (eager launches only; launches replayed
 * from a captured graph are not timed).  sph_profile_enable resets the
 * counters; sph_profile_read synchronises on the recorded events and returns
 * the number of launches and their summed duration for one kernel class.
 * Timing adds two event records per timed launch, or per sweep for the
 * damping classes (a few microseconds of queue time each); sph_profile_classes limits it to the classes whose bit
 * (1 << class) is set in `mask` (all by default; kept across enables). */
#define SPH_KERNEL_STRESS 0    /* deformation gradient + stress + PB */
#define SPH_KERNEL_MOMENTUM 1  /* pair momentum sum + kick */
#define SPH_KERNEL_DAMPING 2   /* one colour pass of the damping sweep (timed per
                                  sweep: one event pair around its colour passes,
                                  which share its time) */
#define SPH_KERNEL_DRIFT_KE 3  /* drift + kinetic energy + stop test */
#define SPH_KERNEL_DIFF_GRAD 4 /* diffusion flux */
#define SPH_KERNEL_DIFF_DIV 5  /* diffusion divergence + Dirichlet + pressure */
#define SPH_KERNEL_LOAD 6      /* grip displacement increment */
#define SPH_KERNEL_ADJ_STRESS 7  /* reverse: stress + momentum transpose */
#define SPH_KERNEL_ADJ_GATHER 8  /* reverse: displacement-gradient transpose (+ drift) */
#define SPH_KERNEL_ADJ_DAMPING 9 /* reverse: one colour pass of the transposed sweep
                                    (timed per sweep, as SPH_KERNEL_DAMPING) */
#define SPH_KERNEL_COUNT 10
int sph_profile_enable(sph_nbr* nbr, int enable);
int sph_profile_classes(sph_nbr* nbr, uint32_t mask);
int sph_profile_read(sph_nbr* nbr, int kernel_class, int64_t* launches, double* total_ms);

/* Thread-local description of the last error ("" if none). */
const char* sph_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPH_H */
