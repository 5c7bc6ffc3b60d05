// sph_tune.hip -- launch-shape autotuner.
//
// The best number of lanes per particle of the tiled gather kernels, and the
// best lane-group width of each damping colour pass, depend on the particle
// set (neighbour counts, tile windows, anchor block sizes) and on the
// precision.  sph_autotune times every candidate on the handle's own data,
// with HIP events, on scratch copies of the state, and keeps the fastest in
// the handle; later launches on that handle use them.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <vector>

#include "sph_common.h"

using namespace sph;

namespace {

struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) hipFree(p);
  }
  template <typename P>
  int alloc(P** p, size_t bytes) {
    if (bytes == 0) {
      *p = nullptr;
      return SPH_OK;
    }
    if (hipMalloc(reinterpret_cast<void**>(p), bytes) != hipSuccess) {
      set_error("autotune scratch allocation of %zu bytes failed", bytes);
      return SPH_E_DEVICE;
    }
    ptrs.push_back(*p);
    return SPH_OK;
  }
};

// mean milliseconds of `reps` calls of f, after one untimed call
template <typename F>
int time_ms(hipStream_t s, int reps, F&& f, double* ms) {
  int rc = f();
  if (rc) return rc;
  hipEvent_t a = nullptr, b = nullptr;
  SPH_HIP(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    hipEventDestroy(a);
    set_error("event creation failed");
    return SPH_E_DEVICE;
  }
  hipEventRecord(a, s);
  for (int i = 0; i < reps && rc == SPH_OK; ++i) rc = f();
  hipEventRecord(b, s);
  hipEventSynchronize(b);
  float t = 0.f;
  hipEventElapsedTime(&t, a, b);
  hipEventDestroy(a);
  hipEventDestroy(b);
  *ms = (double)t / reps;
  return rc;
}

}  // namespace

extern "C" int sph_set_tuning(sph_nbr* nb, int prec, const sph_tuning* t) {
  clear_error();
  if (!nb || !t || (prec != SPH_F32 && prec != SPH_F64)) {
    set_error("bad arguments");
    return SPH_E_ARG;
  }
  // a tile's workgroup is tile_tmax x lanes threads, at most 1024
  auto ok = [](int v) { return v == 1 || v == 2 || v == 4; };
  if (!ok(t->lpp_stress) || !ok(t->lpp_momentum) || !ok(t->lpp_adj_stress) ||
      !ok(t->lpp_adj_gather)) {
    set_error("lanes per particle of the tiled kernels: 1, 2 or 4");
    return SPH_E_ARG;
  }
  for (int c = 0; c < 8; ++c) {
    if (t->damp_lanes[c] != 0 && t->damp_lanes[c] != 8 && t->damp_lanes[c] != 16 &&
        t->damp_lanes[c] != 32 && t->damp_lanes[c] != 64) {
      set_error("damping lanes per anchor: 0 (automatic), 8, 16, 32 or 64");
      return SPH_E_ARG;
    }
    if (t->damp_idle[c] < 0 || t->damp_idle[c] > 2) {
      set_error("damping idle lanes: 0 (automatic), 1 (spare slot) or 2 (skip)");
      return SPH_E_ARG;
    }
  }
  nb->tune.lpp[TUNE_STRESS][prec] = t->lpp_stress;
  nb->tune.lpp[TUNE_MOMENTUM][prec] = t->lpp_momentum;
  nb->tune.lpp[TUNE_ADJ_STRESS][prec] = t->lpp_adj_stress;
  nb->tune.lpp[TUNE_ADJ_GATHER][prec] = t->lpp_adj_gather;
  for (int c = 0; c < 8; ++c) nb->tune.damp_g[prec][c] = t->damp_lanes[c];
  for (int c = 0; c < 8; ++c) nb->tune.damp_idle[prec][c] = t->damp_idle[c];
  return SPH_OK;
}

extern "C" int sph_get_tuning(const sph_nbr* nb, int prec, sph_tuning* t) {
  clear_error();
  if (!nb || !t || (prec != SPH_F32 && prec != SPH_F64)) {
    set_error("bad arguments");
    return SPH_E_ARG;
  }
  *t = sph_tuning{};
  t->lpp_stress = nb->tune.lpp[TUNE_STRESS][prec];
  t->lpp_momentum = nb->tune.lpp[TUNE_MOMENTUM][prec];
  t->lpp_adj_stress = nb->tune.lpp[TUNE_ADJ_STRESS][prec];
  t->lpp_adj_gather = nb->tune.lpp[TUNE_ADJ_GATHER][prec];
  for (int c = 0; c < 8; ++c) t->damp_lanes[c] = nb->tune.damp_g[prec][c];
  for (int c = 0; c < 8; ++c) t->damp_idle[c] = nb->tune.damp_idle[prec][c];
  return SPH_OK;
}

extern "C" int sph_autotune(sph_nbr* nb, const sph_material* m, const sph_state* st, double eta,
                            double dt_s, int with_adjoint, sph_tuning* out, void* stream) {
  clear_error();
  int rc = check_state(nb, st, true);
  if (rc) return rc;
  if (!m || !st->PB || (m->model == SPH_MODEL_J2 && !st->plastic)) {
    set_error("material, PB (and the J2 state) are required");
    return SPH_E_ARG;
  }
  if ((rc = check_mixture(m, st))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int prec = st->prec;
  const size_t n = (size_t)nb->n, d = (size_t)nb->dim, T = prec == SPH_F64 ? 8 : 4;
  const bool j2 = m->model == SPH_MODEL_J2;
  Scratch sc;
  sph_state w = *st;  // scratch copies of everything the kernels write
  w.acc = nullptr;
  if ((rc = sc.alloc(&w.v, d * n * T)) || (rc = sc.alloc(&w.PB, d * d * n * T))) return rc;
  SPH_HIP(hipMemcpyAsync(w.v, st->v, d * n * T, hipMemcpyDeviceToDevice, s));
  if (j2) {
    if ((rc = sc.alloc(&w.plastic, 7 * n * T))) return rc;
    SPH_HIP(hipMemcpyAsync(w.plastic, st->plastic, 7 * n * T, hipMemcpyDeviceToDevice, s));
  }
  sph_adjoint a{};
  a.prec = prec;
  if (with_adjoint) {
    if ((rc = sc.alloc(&a.u, d * n * 8)) || (rc = sc.alloc(&a.v, d * n * T)) ||
        (rc = sc.alloc(&a.work, d * d * n * T)) || (rc = sc.alloc(&a.grad, SPH_NGRAD * 8)) ||
        (rc = sc.alloc(&a.p, n * 8)))
      return rc;
    SPH_HIP(hipMemsetAsync(a.u, 0, d * n * 8, s));
    SPH_HIP(hipMemcpyAsync(a.v, st->v, d * n * T, hipMemcpyDeviceToDevice, s));
    SPH_HIP(hipMemsetAsync(a.p, 0, n * 8, s));
    SPH_HIP(hipMemsetAsync(a.grad, 0, SPH_NGRAD * 8, s));
    if (j2) {
      if ((rc = sc.alloc(&a.plastic, 7 * n * T))) return rc;
      SPH_HIP(hipMemsetAsync(a.plastic, 0, 7 * n * T, s));
    }
  }
  if ((rc = damp_prepare(nb, m, &w, eta, dt_s, s))) return rc;
  sph_tuning res{};
  const int reps = 3, trials = 3;
  Tune& tn = nb->tune;
  // tiled kernels: vary one kernel's lanes at a time (the other launch of
  // the pair is the same in every candidate, so the fastest sum picks it);
  // the candidates take turns over several trials and each keeps its best
  // time, so that a slow moment of the device does not decide
  auto pick = [&](int k, std::initializer_list<int> cands, auto&& run, double* best_ms) -> int {
    double bt[4] = {1e300, 1e300, 1e300, 1e300};
    if (cands.size() > 4) return SPH_E_ARG;
    for (int tr = 0; tr < trials; ++tr) {
      int i = 0;
      for (int c : cands) {
        tn.lpp[k][prec] = c;
        double ms = 0.0;
        int r = time_ms(s, reps, run, &ms);
        if (r) return r;
        bt[i] = std::min(bt[i], ms);
        ++i;
      }
    }
    int i = 0, best = tn.lpp[k][prec];
    *best_ms = 1e300;
    for (int c : cands) {
      if (bt[i] < *best_ms) {
        *best_ms = bt[i];
        best = c;
      }
      ++i;
    }
    tn.lpp[k][prec] = best;
    return SPH_OK;
  };
  auto solid = [&]() { return solid_stage(nb, m, &w, dt_s, s, false); };
  double ms = 0.0;
  if ((rc = pick(TUNE_STRESS, {1, 2, 4}, solid, &ms))) return rc;
  res.ms_solid = ms;
  if ((rc = pick(TUNE_MOMENTUM, {1, 2, 4}, solid, &ms))) return rc;
  res.ms_solid = ms;
  if (with_adjoint) {
    // the reverse takes the step's H, here that of st->u
    void* Hs = nullptr;
    if ((rc = sc.alloc(&Hs, d * d * n * T))) return rc;
    if ((rc = displacement_gradient(nb, st, Hs, s))) return rc;
    auto adjr = [&]() { return adj_solid(nb, m, Hs, w.plastic, &w, &a, dt_s, dt_s, s); };
    if ((rc = pick(TUNE_ADJ_STRESS, {1, 2, 4}, adjr, &ms))) return rc;
    if ((rc = pick(TUNE_ADJ_GATHER, {1, 2, 4}, adjr, &ms))) return rc;
    res.ms_adjoint = ms;
    if ((rc = grad_reduce(nb, a.grad, s))) return rc;  // clears the partials it accumulated
  }
  // damping: each colour's width by the time of its own pass (within a whole
  // sweep the widths of one colour differ by less than the sweep's noise),
  // timed inside whole sweeps: the other colours' passes run between its
  // timings as in a run, so its records are not left in the last-level
  // cache (a pass timed back to back on a large body then favours widths
  // that are slower in a run).  The idle lanes of a row follow the automatic
  // rule, for the same reason.
  for (int c = 0; c < 8; ++c) tn.damp_idle[prec][c] = 0;
  const int ncol = 1 << nb->dim;
  double sweep = 0.0;
  hipEvent_t ea = nullptr, eb = nullptr;
  SPH_HIP(hipEventCreate(&ea));
  if (hipEventCreate(&eb) != hipSuccess) {
    hipEventDestroy(ea);
    set_error("event creation failed");
    return SPH_E_DEVICE;
  }
  auto pass_in_sweep = [&](int col, double* ms) -> int {
    double tot = 0.0;
    for (int r = -1; r < reps; ++r) {  // r = -1: untimed
      for (int c = 0; c < ncol; ++c) {
        if (c == col) hipEventRecord(ea, s);
        int e = damping_pass(nb, &w, c, s);
        if (e) return e;
        if (c == col) hipEventRecord(eb, s);
      }
      if (hipEventSynchronize(eb) != hipSuccess) {
        set_error("timing the damping pass failed");
        return SPH_E_DEVICE;
      }
      float t = 0.f;
      hipEventElapsedTime(&t, ea, eb);
      if (r >= 0) tot += t;
    }
    *ms = tot / reps;
    return SPH_OK;
  };
  for (int col = 0; col < ncol; ++col) {
    if (nb->color_off[col + 1] <= nb->color_off[col]) continue;
    int best = 0;
    double bt = 1e300;
    for (int tr = 0; tr < trials && rc == SPH_OK; ++tr)
      for (int g : {8, 16, 32, 64}) {
        tn.damp_g[prec][col] = g;
        // the records laid out for this width, outside the timing
        if ((rc = damp_prepare(nb, m, &w, eta, dt_s, s))) break;
        double t = 0.0;
        if ((rc = pass_in_sweep(col, &t))) break;
        if (t < bt) {
          bt = t;
          best = g;
        }
      }
    if (rc) break;
    tn.damp_g[prec][col] = best;
    sweep += bt;
  }
  hipEventDestroy(ea);
  hipEventDestroy(eb);
  nb->damp_pre = false;
  if (rc) return rc;
  SPH_HIP(hipStreamSynchronize(s));
  res.ms_damping_sweep = sweep;
  res.lpp_stress = tn.lpp[TUNE_STRESS][prec];
  res.lpp_momentum = tn.lpp[TUNE_MOMENTUM][prec];
  res.lpp_adj_stress = tn.lpp[TUNE_ADJ_STRESS][prec];
  res.lpp_adj_gather = tn.lpp[TUNE_ADJ_GATHER][prec];
  for (int c = 0; c < 8; ++c) res.damp_lanes[c] = tn.damp_g[prec][c];
  for (int c = 0; c < 8; ++c) res.damp_idle[c] = tn.damp_idle[prec][c];
  if (out) *out = res;
  return SPH_OK;
}
