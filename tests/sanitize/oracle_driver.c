/*
 * oracle_driver.c -- exercises the CPU oracle's build, stepping and
 * multi-time-step driver on small jittered lattices, for a run under the
 * address and undefined-behaviour sanitizers.  Built against sph_oracle.c as
 * it is (FP64, or the complex-step build with ORC_COMPLEX); prints "ok" when
 * every result is finite.  Test infrastructure: only the tests build it.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sph_oracle.h"

#ifdef ORC_COMPLEX
#define RE(x) creal(x)
#else
#define RE(x) (x)
#endif

static uint64_t lcg = 88172645463325252ull;
static double urand(void) {  /* xorshift64, uniform in [0, 1) */
  lcg ^= lcg << 13;
  lcg ^= lcg >> 7;
  lcg ^= lcg << 17;
  return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static void* xcalloc(size_t n, size_t sz) {
  void* p = calloc(n ? n : 1, sz);
  if (!p) {
    fprintf(stderr, "out of memory\n");
    exit(3);
  }
  return p;
}

/* lattice [dim][n] in id order, idx[0] fastest, jitter in units of dp */
static double* lattice(int dim, const int* shape, double dp, double jit, int64_t* n_out) {
  int64_t n = 1;
  for (int k = 0; k < dim; ++k) n *= shape[k];
  double* X = xcalloc((size_t)(dim * n), sizeof(double));
  for (int64_t i = 0; i < n; ++i) {
    int64_t r = i;
    for (int k = 0; k < dim; ++k) {
      const int64_t c = r % shape[k];
      r /= shape[k];
      X[k * n + i] = (c + 0.5) * dp + jit * dp * (2.0 * urand() - 1.0);
    }
  }
  *n_out = n;
  return X;
}

static int finite_all(const real* a, int64_t m) {
  for (int64_t i = 0; i < m; ++i)
    if (!isfinite(RE(a[i]))) return 0;
  return 1;
}

static int check_build(orc_sys* s, int dim) {
  int64_t sz[10];
  orc_sizes(s, sz);
  const int64_t n = sz[0], np = sz[1], nu = sz[2], nc = sz[3], na = sz[7];
  uint32_t* key = xcalloc((size_t)n, 4);
  uint32_t* perm = xcalloc((size_t)n, 4);
  uint32_t* cs = xcalloc((size_t)(nc + 1), 4);
  int64_t* off = xcalloc((size_t)(n + 1), 8);
  uint32_t* idx = xcalloc((size_t)np, 4);
  double* X = xcalloc((size_t)(dim * n), 8);
  double* V = xcalloc((size_t)n, 8);
  double* B0 = xcalloc((size_t)(dim * dim * n), 8);
  orc_get_build(s, key, perm, cs, off, idx, X, V, B0);
  uint32_t* pa = xcalloc((size_t)nu, 4);
  uint32_t* pb = xcalloc((size_t)nu, 4);
  uint32_t* pl = xcalloc((size_t)nu, 4);
  uint32_t* ak = xcalloc((size_t)na, 4);
  int64_t* ao = xcalloc((size_t)(na + 1), 8);
  uint32_t* an = xcalloc((size_t)na, 4);
  int64_t co[9];
  orc_get_schedule(s, pa, pb, pl, ak, ao, an, co);
  int ok = off[n] == np && co[1 << dim] == na && ao[na] == nu;
  for (int64_t i = 0; i < dim * dim * n; ++i) ok = ok && isfinite(B0[i]);
  free(key); free(perm); free(cs); free(off); free(idx); free(X); free(V); free(B0);
  free(pa); free(pb); free(pl); free(ak); free(ao); free(an);
  return ok;
}

/* 2D strip: NH, swelling, two-way coupled nonlinear diffusion, mixture momentum */
static int run_strip(void) {
  const int shape[2] = {24, 6};
  const double dp = 12.5e-6;
  int64_t n;
  double* X = lattice(2, shape, dp, 0.05, &n);
  double* V = xcalloc((size_t)n, 8);
  for (int64_t i = 0; i < n; ++i) V[i] = dp * dp;
  int err = 0;
  orc_sys* s = orc_create(2, n, X, V, 1.3 * dp, &err);
  if (!s || err) return 0;
  int ok = check_build(s, 2);
  /* the oracle's arrays are in its sorted order: flags by sorted position */
  int64_t sz[10];
  orc_sizes(s, sz);
  uint32_t* perm = xcalloc((size_t)n, 4);
  {
    uint32_t* key = xcalloc((size_t)n, 4);
    uint32_t* cs = xcalloc((size_t)(sz[3] + 1), 4);
    int64_t* off = xcalloc((size_t)(n + 1), 8);
    uint32_t* idx = xcalloc((size_t)sz[1], 4);
    double* Xs = xcalloc((size_t)(2 * n), 8);
    double* Vs = xcalloc((size_t)n, 8);
    double* B0 = xcalloc((size_t)(4 * n), 8);
    orc_get_build(s, key, perm, cs, off, idx, Xs, Vs, B0);
    free(key); free(cs); free(off); free(idx); free(Xs); free(Vs); free(B0);
  }
  uint8_t* flags = xcalloc((size_t)n, 1);
  real* c = xcalloc((size_t)n, sizeof(real));
  for (int64_t a = 0; a < n; ++a) {
    const int64_t id = perm[a];
    const int ix = (int)(id % shape[0]), iy = (int)(id / shape[0]);
    if (ix < 3 || ix >= shape[0] - 3) flags[a] |= ORC_FIXED;
    if (iy == shape[1] - 1) {
      flags[a] |= ORC_CDIR;
      c[a] = 0.4;
    }
  }
  orc_material m;
  memset(&m, 0, sizeof m);
  m.model = ORC_NH;
  m.E = 100.0e6;
  m.nu = 0.4;
  m.rho0 = 2000.0;
  m.C_swell = 3.0e6;
  m.rho_l0 = 1000.0;
  orc_cfg cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.n_slow = 3;
  cfg.slow_kind = ORC_DIFFUSION_COUPLED;
  cfg.eta = 10.0;
  cfg.fixed_inner = 25;
  cfg.D = 1.0e-10;
  cfg.c_bc = 0.4;
  cfg.nonlinear = 1;
  real* u = xcalloc((size_t)(2 * n), sizeof(real));
  real* v = xcalloc((size_t)(2 * n), sizeof(real));
  real* q = xcalloc((size_t)(2 * n), sizeof(real));
  real* p = xcalloc((size_t)n, sizeof(real));
  real* acc = xcalloc((size_t)(2 * n), sizeof(real));
  int64_t k[3];
  double ke[3];
  int32_t conv[3];
  const int rc = orc_advance(s, &m, &cfg, u, v, NULL, c, q, p, NULL, flags, NULL, k, ke, conv, acc);
  ok = ok && rc >= 0 && finite_all(u, 2 * n) && finite_all(c, n) && finite_all(p, n) &&
       finite_all(acc, 2 * n);
  /* the one-way step and the lone pieces */
  orc_diffusion_step(s, 1.0e-10, 1.0e-3, 0.4, 3.0e6, 0.0, c, q, p, flags);
  real* H9 = xcalloc((size_t)(9 * n), sizeof(real));
  real* P9 = xcalloc((size_t)(9 * n), sizeof(real));
  real* PB = xcalloc((size_t)(4 * n), sizeof(real));
  orc_displacement_gradient(s, u, H9);
  ok = ok && orc_stress(s, &m, H9, NULL, p, P9, PB) >= 0;
  orc_mixture_flux(s, &m, H9, v, c, q, PB);
  orc_momentum(s, &m, PB, c, acc);
  orc_damping_sweep(s, m.rho0, cfg.eta, 1.0e-9, v, flags, m.rho_l0, c);
  const real e = orc_drift_ke(s, m.rho0, 1.0e-9, u, v, flags, m.rho_l0, c);
  ok = ok && isfinite(RE(e)) && finite_all(PB, 4 * n) && finite_all(v, 2 * n);
  free(X); free(V); free(perm); free(flags); free(c); free(u); free(v); free(q); free(p);
  free(acc); free(H9); free(P9); free(PB);
  orc_destroy(s);
  return ok;
}

/* 2D bar: LE, loading steps, adaptive stop with a cap */
static int run_bar(void) {
  const int shape[2] = {20, 6};
  const double dp = 0.25e-3;
  int64_t n;
  double* X = lattice(2, shape, dp, 0.0, &n);
  double* V = xcalloc((size_t)n, 8);
  for (int64_t i = 0; i < n; ++i) V[i] = dp * dp;
  int err = 0;
  orc_sys* s = orc_create(2, n, X, V, 1.3 * dp, &err);
  if (!s || err) return 0;
  int ok = check_build(s, 2);
  orc_material m;
  memset(&m, 0, sizeof m);
  m.model = ORC_LE;
  m.E = 210.0e9;
  m.nu = 0.3;
  m.rho0 = 7850.0;
  /* a lattice without jitter keeps id order within cells; grips by position */
  int64_t sz[10];
  orc_sizes(s, sz);
  double* Xs = xcalloc((size_t)(2 * n), 8);
  {
    uint32_t* key = xcalloc((size_t)n, 4);
    uint32_t* perm = xcalloc((size_t)n, 4);
    uint32_t* cs = xcalloc((size_t)(sz[3] + 1), 4);
    int64_t* off = xcalloc((size_t)(n + 1), 8);
    uint32_t* idx = xcalloc((size_t)sz[1], 4);
    double* Vs = xcalloc((size_t)n, 8);
    double* B0 = xcalloc((size_t)(4 * n), 8);
    orc_get_build(s, key, perm, cs, off, idx, Xs, Vs, B0);
    free(key); free(perm); free(cs); free(off); free(idx); free(Vs); free(B0);
  }
  uint8_t* flags = xcalloc((size_t)n, 1);
  real* vgrip = xcalloc((size_t)(2 * n), sizeof(real));
  for (int64_t a = 0; a < n; ++a) {
    if (Xs[a] < 3 * dp) flags[a] |= ORC_FIXED;
    if (Xs[a] > (shape[0] - 3) * dp) {
      flags[a] |= ORC_FIXED | ORC_GRIP;
      vgrip[a] = 1.0e-3;
    }
  }
  orc_cfg cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.n_slow = 3;
  cfg.slow_kind = ORC_LOAD;
  cfg.dt_slow = 1.0e-3;
  cfg.eta = 1.0e4;
  cfg.k_max = 200;
  cfg.ke_tol = 1.0e-12;
  real* u = xcalloc((size_t)(2 * n), sizeof(real));
  real* v = xcalloc((size_t)(2 * n), sizeof(real));
  int64_t k[3];
  double ke[3];
  int32_t conv[3];
  const int rc = orc_advance(s, &m, &cfg, u, v, NULL, NULL, NULL, NULL, vgrip, flags, NULL, k, ke,
                             conv, NULL);
  ok = ok && rc >= 0 && finite_all(u, 2 * n) && k[0] > 0 && k[0] <= 200;
  double dts = 0.0, dtd = 0.0;
  orc_default_steps(s, &m, 1.0e-10, &dts, &dtd);
  ok = ok && dts > 0.0 && dtd > 0.0;
  free(X); free(V); free(Xs); free(flags); free(vgrip); free(u); free(v);
  orc_destroy(s);
  return ok;
}

/* 3D bar: J2 with nonlinear hardening, pulled into the plastic range */
static int run_neck(void) {
  const int shape[3] = {12, 5, 5};
  const double dp = 0.53334e-3;
  int64_t n;
  double* X = lattice(3, shape, dp, 0.01, &n);
  double* V = xcalloc((size_t)n, 8);
  for (int64_t i = 0; i < n; ++i) V[i] = dp * dp * dp;
  int err = 0;
  orc_sys* s = orc_create(3, n, X, V, 1.3 * dp, &err);
  if (!s || err) return 0;
  int ok = check_build(s, 3);
  int64_t sz[10];
  orc_sizes(s, sz);
  double* Xs = xcalloc((size_t)(3 * n), 8);
  {
    uint32_t* key = xcalloc((size_t)n, 4);
    uint32_t* perm = xcalloc((size_t)n, 4);
    uint32_t* cs = xcalloc((size_t)(sz[3] + 1), 4);
    int64_t* off = xcalloc((size_t)(n + 1), 8);
    uint32_t* idx = xcalloc((size_t)sz[1], 4);
    double* Vs = xcalloc((size_t)n, 8);
    double* B0 = xcalloc((size_t)(9 * n), 8);
    orc_get_build(s, key, perm, cs, off, idx, Xs, Vs, B0);
    free(key); free(perm); free(cs); free(off); free(idx); free(Vs); free(B0);
  }
  uint8_t* flags = xcalloc((size_t)n, 1);
  real* vgrip = xcalloc((size_t)(3 * n), sizeof(real));
  for (int64_t a = 0; a < n; ++a) {
    if (Xs[a] < 2 * dp) {
      flags[a] |= ORC_FIXED | ORC_GRIP;
      vgrip[a] = -0.02;
    }
    if (Xs[a] > (shape[0] - 2) * dp) {
      flags[a] |= ORC_FIXED | ORC_GRIP;
      vgrip[a] = 0.02;
    }
  }
  const double mu = 80.1938e9, K = 164.21e9;
  orc_material m;
  memset(&m, 0, sizeof m);
  m.model = ORC_J2;
  m.E = 9.0 * K * mu / (3.0 * K + mu);
  m.nu = (3.0 * K - 2.0 * mu) / (2.0 * (3.0 * K + mu));
  m.rho0 = 7850.0;
  m.sigma0 = 200.0e6;
  m.sigma_inf = 400.0e6;
  m.delta = 16.0;
  m.H = 1.0e8;
  orc_cfg cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.n_slow = 3;
  cfg.slow_kind = ORC_LOAD;
  cfg.dt_slow = 1.0e-3;
  cfg.eta = 1.0e4;
  cfg.fixed_inner = 20;
  real* u = xcalloc((size_t)(3 * n), sizeof(real));
  real* v = xcalloc((size_t)(3 * n), sizeof(real));
  real* pl = xcalloc((size_t)(7 * n), sizeof(real));
  real* acc = xcalloc((size_t)(3 * n), sizeof(real));
  int64_t k[3];
  double ke[3];
  int32_t conv[3];
  const int rc = orc_advance(s, &m, &cfg, u, v, pl, NULL, NULL, NULL, vgrip, flags, NULL, k, ke,
                             conv, acc);
  double amax = 0.0;
  for (int64_t a = 0; a < n; ++a) amax = fmax(amax, RE(pl[6 * n + a]));
  ok = ok && rc >= 0 && finite_all(u, 3 * n) && finite_all(pl, 7 * n) && amax > 0.0;
  free(X); free(V); free(Xs); free(flags); free(vgrip); free(u); free(v); free(pl); free(acc);
  orc_destroy(s);
  return ok;
}

int main(void) {
  const int a = run_strip(), b = run_bar(), c = run_neck();
  printf("strip %d bar %d neck %d\n", a, b, c);
  if (a && b && c) {
    printf("ok\n");
    return 0;
  }
  return 1;
}
