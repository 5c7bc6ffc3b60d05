// sph_driver.hip -- C ABI of the stepping functions and the multi-time-step
// driver (Sec. 4.2 of the paper): outer loop over slow steps (loading or
// diffusion), inner loop of damped solid relaxation steps until the kinetic
// energy falls to the threshold.  The stop test runs on the device (the
// drift/E_k kernel sets a flag that every later inner kernel checks), so the
// host only polls once per chunk of inner steps; a chunk can be replayed as a
// captured hipGraph to remove per-kernel launch cost on small problems.  In
// an adaptive run the first poll comes after a short chunk and each later one
// after twice as many steps, up to the configured chunk, so that a slow step
// that relaxes in a few inner steps does not launch a whole chunk after it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "sph_common.h"

using namespace sph;

namespace sph {

hipEvent_t prof_begin(const sph_nbr* nb, int kind, hipStream_t s) {
  Prof* p = nb->prof;
  if (!p || !p->on || p->suspend || !((p->mask >> kind) & 1u)) return nullptr;
  hipEvent_t e = nullptr;
  if (!p->pool.empty()) {
    e = p->pool.back();
    p->pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return nullptr;
  }
  if (hipEventRecord(e, s) != hipSuccess) {
    p->pool.push_back(e);
    return nullptr;
  }
  return e;
}

void prof_end(const sph_nbr* nb, int kind, hipEvent_t a, hipStream_t s, int launches) {
  Prof* p = nb->prof;
  if (!a || !p) return;
  hipEvent_t b = nullptr;
  if (!p->pool.empty()) {
    b = p->pool.back();
    p->pool.pop_back();
  } else if (hipEventCreate(&b) != hipSuccess) {
    p->pool.push_back(a);
    return;
  }
  hipEventRecord(b, s);
  p->pend.push_back(Prof::Pend{kind, a, b, launches});
  if (p->pend.size() > 65536) prof_resolve(nb);
}

int prof_resolve(const sph_nbr* nb) {
  Prof* p = nb->prof;
  if (!p) return SPH_OK;
  for (auto& q : p->pend) {
    SPH_HIP(hipEventSynchronize(q.b));
    float ms = 0.f;
    SPH_HIP(hipEventElapsedTime(&ms, q.a, q.b));
    p->count[q.kind] += q.launches;
    p->ms[q.kind] += ms;
    p->pool.push_back(q.a);
    p->pool.push_back(q.b);
  }
  p->pend.clear();
  return SPH_OK;
}

}  // namespace sph

extern "C" int sph_profile_enable(sph_nbr* nb, int enable) {
  clear_error();
  if (!nb) {
    set_error("null handle");
    return SPH_E_ARG;
  }
  if (!nb->prof) nb->prof = new Prof();
  int rc = prof_resolve(nb);
  for (int k = 0; k < SPH_KERNEL_COUNT; ++k) {
    nb->prof->count[k] = 0;
    nb->prof->ms[k] = 0.0;
  }
  nb->prof->on = enable != 0;
  return rc;
}

extern "C" int sph_profile_classes(sph_nbr* nb, uint32_t mask) {
  clear_error();
  if (!nb) {
    set_error("bad handle");
    return SPH_E_ARG;
  }
  if (!nb->prof) nb->prof = new Prof();
  nb->prof->mask = mask;
  return SPH_OK;
}

extern "C" int sph_profile_read(sph_nbr* nb, int kind, int64_t* launches, double* total_ms) {
  clear_error();
  if (!nb || kind < 0 || kind >= SPH_KERNEL_COUNT) {
    set_error("bad handle or kernel class");
    return SPH_E_ARG;
  }
  if (!nb->prof) {
    if (launches) *launches = 0;
    if (total_ms) *total_ms = 0.0;
    return SPH_OK;
  }
  int rc = prof_resolve(nb);
  if (launches) *launches = nb->prof->count[kind];
  if (total_ms) *total_ms = nb->prof->ms[kind];
  return rc;
}

namespace {

int inner_steps(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
                double eta, int count, hipStream_t s) {
  for (int i = 0; i < count; ++i) {
    int rc = solid_stage(nb, m, st, dt, s, true);
    if (rc) return rc;
    rc = damping_sweep(nb, m, st, eta, dt, s, true);
    if (rc) return rc;
    rc = drift_ke(nb, m, st, dt, nullptr, s, true);
    if (rc) return rc;
  }
  return SPH_OK;
}

struct GraphChunk {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~GraphChunk() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
  }
};

// the instantiated chunk of inner steps of sph_advance_multirate, kept with
// the arguments its launches were recorded with
struct ChunkGraph {
  std::vector<unsigned char> key;
  GraphChunk gc;
};

template <typename S>
void key_add(std::vector<unsigned char>& k, const S* p) {
  const unsigned char* b = reinterpret_cast<const unsigned char*>(p);
  if (p) k.insert(k.end(), b, b + sizeof(S));
  else k.push_back(0);
}

// checkpoint slice l of a tape <-> the state arrays
int tape_copy(const sph_nbr* nb, const sph_material* m, const sph_state* st, const sph_tape* tp,
              int l, bool to_tape, hipStream_t s) {
  const size_t n = (size_t)nb->n, d = (size_t)nb->dim;
  const size_t T = st->prec == SPH_F64 ? 8 : 4;
  auto cp = [&](void* tape_base, void* arr, size_t bytes) -> int {
    if (!tape_base || !arr || bytes == 0) return SPH_OK;
    char* t = (char*)tape_base + (size_t)l * bytes;
    SPH_HIP(hipMemcpyAsync(to_tape ? (void*)t : arr, to_tape ? arr : (void*)t, bytes,
                           hipMemcpyDeviceToDevice, s));
    return SPH_OK;
  };
  int rc = cp(tp->ck_u, st->u, d * n * 8);
  if (!rc) rc = cp(tp->ck_v, st->v, d * n * T);
  if (!rc && m->model == SPH_MODEL_J2) rc = cp(tp->ck_plastic, st->plastic, 7 * n * T);
  if (!rc) rc = cp(tp->ck_c, st->c, n * T);
  return rc;
}

// inner checkpoint j of the segmented reverse pass (the state at the start
// of segment j + 1 of a slow step): u, v and the J2 state
int seg_copy(const sph_nbr* nb, const sph_material* m, const sph_state* st, const sph_tape* tp,
             int64_t j, bool to_tape, hipStream_t s) {
  const size_t n = (size_t)nb->n, d = (size_t)nb->dim;
  const size_t T = st->prec == SPH_F64 ? 8 : 4;
  auto cp = [&](void* base, void* arr, size_t bytes) -> int {
    char* t = (char*)base + (size_t)j * bytes;
    SPH_HIP(hipMemcpyAsync(to_tape ? (void*)t : arr, to_tape ? arr : (void*)t, bytes,
                           hipMemcpyDeviceToDevice, s));
    return SPH_OK;
  };
  int rc = cp(tp->seg_u, st->u, d * n * 8);
  if (!rc) rc = cp(tp->seg_v, st->v, d * n * T);
  if (!rc && m->model == SPH_MODEL_J2) rc = cp(tp->seg_plastic, st->plastic, 7 * n * T);
  return rc;
}

// segments of k_hist_cap inner steps the reverse pass splits a slow step of
// kl inner steps into
int64_t n_segments(const sph_tape* tp, int64_t kl) {
  return kl <= 0 ? 0 : (kl + tp->k_hist_cap - 1) / tp->k_hist_cap;
}

// the tape can re-run and reverse slow steps of these inner counts
int check_segments(const sph_material* m, const sph_tape* tp, const int64_t* counts, int L) {
  const bool j2 = m->model == SPH_MODEL_J2;
  for (int l = 0; l < L; ++l) {
    const int64_t kl = counts[l];
    if (kl <= 0) continue;
    if (tp->k_hist_cap <= 0 || !tp->hist_H || (j2 && !tp->hist_plastic)) {
      set_error("slow step %d has %lld inner steps; the tape records none", l, (long long)kl);
      return SPH_E_CAPACITY;
    }
    const int64_t ns = n_segments(tp, kl);
    if (ns > 1 && (ns - 1 > tp->seg_cap || !tp->seg_u || !tp->seg_v || (j2 && !tp->seg_plastic))) {
      set_error("slow step %d has %lld inner steps: %lld segments of %lld need %lld inner "
                "checkpoints, the tape holds %lld", l, (long long)kl, (long long)ns,
                (long long)tp->k_hist_cap, (long long)(ns - 1), (long long)tp->seg_cap);
      return SPH_E_CAPACITY;
    }
  }
  return SPH_OK;
}

int check_tape(const sph_nbr* nb, const sph_material* m, const sph_state* st,
               const sph_multirate_cfg* cfg, const sph_tape* tp) {
  if (cfg->n_slow > tp->n_slow_cap) {
    set_error("tape holds %d slow steps, the run has %d", tp->n_slow_cap, cfg->n_slow);
    return SPH_E_CAPACITY;
  }
  if (!tp->ck_u || !tp->ck_v || !tp->k_rec || (m->model == SPH_MODEL_J2 && !tp->ck_plastic) ||
      (cfg->slow_kind != SPH_SLOW_LOAD && (!tp->ck_c || !st->c))) {
    set_error("tape checkpoint arrays missing");
    return SPH_E_ARG;
  }
  return SPH_OK;
}

struct RecGuard {  // inner-state recording is switched off on every exit
  const sph_nbr* nb;
  ~RecGuard() {
    nb->rec_H = nullptr;
    nb->rec_pl = nullptr;
  }
};

struct BatGuard {  // per-specimen lookups and per-run coefficients end with the run
  const sph_nbr* nb;
  ~BatGuard() {
    nb->bat_on = false;
    nb->damp_pre = false;
  }
};

int batch_begin(const sph_nbr* nb, const sph_material* m, const sph_multirate_cfg* cfg,
                hipStream_t s) {
  if (!cfg->batch) return SPH_OK;
  int rc = batch_check(nb, cfg);
  if (rc) return rc;
  if ((rc = batch_upload(nb, m, cfg, s))) return rc;
  nb->bat_on = true;
  return SPH_OK;
}

}  // namespace

extern "C" int sph_solid_relax_step(const sph_nbr* nb, const sph_material* mat,
                                    const sph_state* st, double dt_s, void* stream) {
  clear_error();
  int rc = check_state(nb, st, true);
  if (rc) return rc;
  if (!mat) {
    set_error("material is NULL");
    return SPH_E_ARG;
  }
  if ((rc = check_mixture(mat, st))) return rc;
  return solid_stage(nb, mat, st, dt_s, (hipStream_t)stream, false);
}

extern "C" int sph_damping_sweep(const sph_nbr* nb, const sph_material* mat, const sph_state* st,
                                 double eta, double dt_s, void* stream) {
  clear_error();
  int rc = check_state(nb, st, true);
  if (rc) return rc;
  if (!mat) {
    set_error("material is NULL");
    return SPH_E_ARG;
  }
  if ((rc = check_mixture(mat, st))) return rc;
  return damping_sweep(nb, mat, st, eta, dt_s, (hipStream_t)stream, false);
}

extern "C" int sph_drift_ke(const sph_nbr* nb, const sph_material* mat, const sph_state* st,
                            double dt_s, double* ke_out, void* stream) {
  clear_error();
  int rc = check_state(nb, st, true);
  if (rc) return rc;
  if (!mat) {
    set_error("material is NULL");
    return SPH_E_ARG;
  }
  if ((rc = check_mixture(mat, st))) return rc;
  return drift_ke(nb, mat, st, dt_s, ke_out, (hipStream_t)stream, false);
}

extern "C" int sph_drift_ke_noalloc(const sph_nbr* nb, const sph_material* mat,
                                    const sph_state* st, double dt_s, double* ke_out,
                                    void* stream) {
  clear_error();
  int rc = check_state(nb, st, true);
  if (rc) return rc;
  if (!mat) {
    set_error("material is NULL");
    return SPH_E_ARG;
  }
  if ((rc = check_mixture(mat, st))) return rc;
  return drift_ke_static(nb, mat, st, dt_s, ke_out, (hipStream_t)stream);
}

extern "C" int sph_load_step(const sph_nbr* nb, const sph_state* st, double dt_l, void* stream) {
  clear_error();
  int rc = check_state(nb, st, false);
  if (rc) return rc;
  return load_step(nb, st, dt_l, (hipStream_t)stream);
}

extern "C" int sph_diffusion_step_coupled(const sph_nbr* nb, const sph_material* mat,
                                          const sph_state* st, double D, double dt_d, double c_bc,
                                          int32_t nonlinear, void* stream) {
  clear_error();
  int rc = check_state(nb, st, true);
  if (rc) return rc;
  if (!mat) {
    set_error("material is NULL");
    return SPH_E_ARG;
  }
  return diffusion_step_coupled(nb, mat, st, D, dt_d, c_bc, nonlinear, (hipStream_t)stream);
}

extern "C" int sph_diffusion_step(const sph_nbr* nb, const sph_material* mat, const sph_state* st,
                                  double D, double dt_d, double c_bc, void* stream) {
  clear_error();
  int rc = check_state(nb, st, false);
  if (rc) return rc;
  if (!mat) {
    set_error("material is NULL");
    return SPH_E_ARG;
  }
  return diffusion_step(nb, mat, st, D, dt_d, c_bc, (hipStream_t)stream);
}

extern "C" int sph_default_steps(double h, const sph_material* mat, double D, double* dt_s,
                                 double* dt_d) {
  clear_error();
  if (!mat || !(h > 0.0) || !(mat->E > 0.0) || !(mat->rho0 > 0.0) || !(mat->nu < 0.5)) {
    set_error("need h > 0, a material with E > 0, rho0 > 0 and nu < 1/2");
    return SPH_E_ARG;
  }
  rest_steps(h, mat, D, dt_s, dt_d);
  return SPH_OK;
}

extern "C" int sph_status(const sph_nbr* nb, void* stream, int32_t* bits) {
  clear_error();
  if (!nb) {
    set_error("null handle");
    return SPH_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  SPH_HIP(hipMemcpyAsync(nb->ctrl_host, nb->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  int32_t st = nb->ctrl_host->status;
  if (bits) *bits = st;
  if (st) {
    int32_t zero = 0;
    SPH_HIP(hipMemcpy((char*)nb->ctrl + offsetof(Ctrl, status), &zero, sizeof(int32_t),
                      hipMemcpyHostToDevice));
    set_error("device status bits 0x%x", st);
    return SPH_E_NUMERIC;
  }
  return SPH_OK;
}

extern "C" int sph_advance_multirate(const sph_nbr* nb, const sph_material* m,
                                     const sph_state* st, const sph_multirate_cfg* cfg,
                                     sph_report* rep, sph_tape* tape, void* stream) {
  clear_error();
  int rc = check_state(nb, st, true);
  if (rc) return rc;
  if (!m || !cfg) {
    set_error("material or cfg is NULL");
    return SPH_E_ARG;
  }
  if ((rc = check_mixture(m, st))) return rc;
  if (cfg->n_slow < 0 || (cfg->slow_kind != SPH_SLOW_LOAD && cfg->slow_kind != SPH_SLOW_DIFFUSION &&
                           cfg->slow_kind != SPH_SLOW_DIFFUSION_COUPLED)) {
    set_error("bad n_slow or slow_kind");
    return SPH_E_ARG;
  }
  double dt_rest = 0.0, dt_diff = 0.0;
  rest_steps(nb->h, m, cfg->D, &dt_rest, &dt_diff);
  const double dt_s = cfg->dt_s > 0.0 ? cfg->dt_s : dt_rest;
  double dt_slow = cfg->dt_slow;
  if (cfg->slow_kind != SPH_SLOW_LOAD && !(dt_slow > 0.0)) {
    if (!(cfg->D > 0.0)) {
      set_error("diffusion needs D > 0");
      return SPH_E_ARG;
    }
    dt_slow = dt_diff;
  }
  const int64_t k_max = cfg->k_max > 0 ? cfg->k_max : (int64_t)std::floor(dt_slow / dt_s) + 1;
  const bool adaptive = cfg->k_sched == nullptr && cfg->fixed_inner <= 0;
  const int chunk = cfg->chunk > 0 ? cfg->chunk : 64;
  // inner steps of the first poll interval of an adaptive run, and of the
  // captured graph there (replayed to fill each interval)
  const int first = adaptive ? std::min(chunk, kPollFirst) : chunk;
  if (tape && (rc = check_tape(nb, m, st, cfg, tape))) return rc;
  RecGuard rec_guard{nb};
  bool recorded = false;
  if (rep) {
    rep->dt_s = dt_s;
    rep->dt_slow = dt_slow;
    rep->k_max = k_max;
    rep->total_inner = 0;
  }
  hipStream_t s = (hipStream_t)stream;
  hipGraphExec_t exec = nullptr;
  const bool graph = cfg->use_graph != 0;
  BatGuard bat_guard{nb};
  if ((rc = batch_begin(nb, m, cfg, s))) return rc;
  if ((rc = damp_prepare(nb, m, st, cfg->eta, dt_s, s))) return rc;
  if (graph) {
    // one chunk of inner steps as a graph, kept on the handle for later
    // calls with the same arguments
    std::vector<unsigned char> key;
    key_add(key, m);
    key_add(key, st);
    key_add(key, &dt_s);
    key_add(key, &cfg->eta);
    key_add(key, &first);
    key_add(key, &nb->tune);
    const Bat bv = bat_view(nb);
    key_add(key, &bv);
    ChunkGraph* cg = reinterpret_cast<ChunkGraph*>(nb->chunk_cache);
    if (!cg || cg->key != key) {
      delete cg;
      cg = new ChunkGraph();
      const_cast<sph_nbr*>(nb)->chunk_cache = cg;
      // capture needs a non-null stream: a private one, which runs nothing
      hipStream_t cap = nullptr;
      SPH_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      if (nb->prof) nb->prof->suspend = true;
      hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        rc = inner_steps(nb, m, st, dt_s, cfg->eta, first, cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cap, &g);
        cg->gc.graph = g;
      }
      if (nb->prof) nb->prof->suspend = false;
      hipStreamDestroy(cap);
      if (rc == SPH_OK && e != hipSuccess) {
        set_error("graph capture failed: %s", hipGetErrorString(e));
        rc = SPH_E_DEVICE;
      }
      if (rc == SPH_OK &&
          hipGraphInstantiate(&cg->gc.exec, cg->gc.graph, nullptr, nullptr, 0) != hipSuccess) {
        set_error("graph instantiation failed");
        rc = SPH_E_DEVICE;
      }
      if (rc) {
        delete cg;
        const_cast<sph_nbr*>(nb)->chunk_cache = nullptr;
        return rc;
      }
      cg->key = key;
    }
    exec = cg->gc.exec;
  }
  int warn = 0;
  for (int32_t l = 0; l < cfg->n_slow && rc == SPH_OK; ++l) {
    if (tape && (rc = tape_copy(nb, m, st, tape, l, true, s))) break;
    if (cfg->slow_kind == SPH_SLOW_LOAD)
      rc = load_step(nb, st, dt_slow, s);
    else if (cfg->slow_kind == SPH_SLOW_DIFFUSION_COUPLED)
      rc = diffusion_step_coupled(nb, m, st, cfg->D, dt_slow, cfg->c_bc, cfg->diff_nonlinear, s);
    else
      rc = diffusion_step(nb, m, st, cfg->D, dt_slow, cfg->c_bc, s);
    if (rc) break;
    // a mixture's masses follow the content the slow step has just changed
    if (m->rho_l0 > 0.0 && (rc = damp_prepare(nb, m, st, cfg->eta, dt_s, s))) break;
    const int64_t nk = cfg->k_sched ? cfg->k_sched[l] : (cfg->fixed_inner > 0 ? cfg->fixed_inner : k_max);
    Ctrl* hc = nb->ctrl_host;
    if (nk <= 0) {
      if (tape) tape->k_rec[l] = 0;
      if (rep && rep->k) rep->k[l] = 0;
      if (rep && rep->ke) rep->ke[l] = 0.0;
      if (rep && rep->converged) rep->converged[l] = 1;
      continue;
    }
    rc = reset_ctrl(nb, nk, adaptive ? cfg->ke_tol : -1.0, s);
    if (rc) break;
    // the last slow step's inner states go to the tape when they fit (eager launches only)
    const bool rec = tape && l == cfg->n_slow - 1 && !graph && tape->hist_H &&
                     nk <= tape->k_hist_cap &&
                     (m->model != SPH_MODEL_J2 || tape->hist_plastic);
    if (rec) {
      nb->rec_H = tape->hist_H;
      nb->rec_pl = tape->hist_plastic;
      recorded = true;
    }
    int64_t launched = 0;
    int64_t interval = first;
    for (;;) {
      int64_t mcount = std::min<int64_t>(interval, nk - launched);
      interval = std::min<int64_t>(2 * interval, chunk);
      if (graph) {
        // whole graphs: the steps past nk return at once on the device
        const int64_t reps = (mcount + first - 1) / first;
        for (int64_t r = 0; r < reps && rc == SPH_OK; ++r) {
          if (hipGraphLaunch(exec, s) != hipSuccess) {
            set_error("graph launch failed");
            rc = SPH_E_DEVICE;
          }
        }
        if (rc) break;
        mcount = reps * first;
      } else {
        rc = inner_steps(nb, m, st, dt_s, cfg->eta, (int)mcount, s);
        if (rc) break;
      }
      launched += mcount;
      if (hipMemcpyAsync(hc, nb->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        set_error("polling the inner-loop state failed");
        rc = SPH_E_DEVICE;
        break;
      }
      if (nb->prof) prof_resolve(nb);
      if (hc->done || launched >= nk) break;
    }
    nb->rec_H = nullptr;
    nb->rec_pl = nullptr;
    if (rc) break;
    if (tape) tape->k_rec[l] = hc->k;
    if (rep && rep->k) rep->k[l] = hc->k;
    if (rep && rep->ke) rep->ke[l] = hc->ke;
    const int conv = hc->ke <= cfg->ke_tol;
    if (rep && rep->converged) rep->converged[l] = conv;
    if (rep) rep->total_inner += hc->k;
    if (adaptive && !hc->stopped_by_ke) warn = 1;
    if (hc->status) {
      set_error("device status bits 0x%x at slow step %d", hc->status, l);
      rc = SPH_E_NUMERIC;
      break;
    }
  }
  if (rc) return rc;
  if (tape) {
    if ((rc = tape_copy(nb, m, st, tape, cfg->n_slow, true, s))) return rc;
    tape->n_rec = cfg->n_slow;
    tape->hist_slow = recorded ? cfg->n_slow - 1 : -1;
    tape->dt_s = dt_s;
    tape->dt_slow = dt_slow;
    SPH_HIP(hipStreamSynchronize(s));
  }
  return warn ? SPH_W_NOT_CONVERGED : SPH_OK;
}

namespace {

// Reverse pass: slow steps last to first; each is re-run from its checkpoint
// with its inner states recorded (unless the tape already holds them), then
// its inner steps are reversed, then its slow update.  A slow step longer
// than the tape's k_hist_cap goes in segments of that many inner steps, each
// re-run from an inner checkpoint the pass lays first.  Enqueues only (no
// host synchronisation), so that it can be captured in a graph.
int backward_enqueue(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                     const sph_multirate_cfg* cfg, sph_tape* tape, const sph_adjoint* adj,
                     hipStream_t s) {
  int rc = SPH_OK;
  const int L = cfg->n_slow;
  const double dt = tape->dt_s, dt_slow = tape->dt_slow;
  const size_t n = (size_t)nb->n, d = (size_t)nb->dim;
  const size_t T = st->prec == SPH_F64 ? 8 : 4;
  const int64_t K = tape->k_hist_cap;
  std::vector<int64_t> before(L + 1, 0);
  for (int l = 0; l < L; ++l) before[l + 1] = before[l] + tape->k_rec[l];
  if ((rc = check_segments(m, tape, tape->k_rec, L))) return rc;
  RecGuard rec_guard{nb};
  bool first = true;  // the next reversed inner step is the run's last one
  // slow step l from its checkpoint: the state its inner steps start from
  auto slow_update = [&](int l) -> int {
    int r = tape_copy(nb, m, st, tape, l, false, s);
    if (r) return r;
    return cfg->slow_kind == SPH_SLOW_LOAD ? load_step(nb, st, dt_slow, s)
           : cfg->slow_kind == SPH_SLOW_DIFFUSION_COUPLED
               ? diffusion_step_coupled(nb, m, st, cfg->D, dt_slow, cfg->c_bc, cfg->diff_nonlinear, s)
               : diffusion_step(nb, m, st, cfg->D, dt_slow, cfg->c_bc, s);
  };
  // `steps` inner steps from the current state; `record`: their H (and J2
  // state) to hist_H [0, steps)
  auto rerun = [&](int64_t steps, bool record) -> int {
    int r = reset_ctrl(nb, steps, -1.0, s);
    if (r) return r;
    nb->rec_H = record ? tape->hist_H : nullptr;
    nb->rec_pl = record ? tape->hist_plastic : nullptr;
    for (int64_t done = 0; done < steps && !r;) {
      const int c = (int)std::min<int64_t>(steps - done, 256);
      r = inner_steps(nb, m, st, dt, cfg->eta, c, s);
      done += c;
    }
    nb->rec_H = nullptr;
    nb->rec_pl = nullptr;
    return r;
  };
  // the transposed inner steps k1 - 1 .. k0 of slow step l, whose recorded
  // states hist_H holds from index 0 = step k0
  auto reverse = [&](int l, int64_t k0, int64_t k1) -> int {
    for (int64_t k = k1 - 1; k >= k0; --k) {
      int r;
      if (first) {
        if ((r = adj_drift(nb, st, adj, dt, s))) return r;
        first = false;
      }
      if ((r = adj_damping(nb, m, st, adj, cfg->eta, dt, s))) return r;
      const size_t i = (size_t)(k - k0);
      const void* Hk = (const char*)tape->hist_H + i * d * d * n * T;
      const void* plk = m->model == SPH_MODEL_J2
                            ? (const void*)((const char*)tape->hist_plastic + i * 7 * n * T)
                            : nullptr;
      const bool has_prev = before[l] + k > 0;
      if ((r = adj_solid(nb, m, Hk, plk, st, adj, dt, has_prev ? dt : 0.0, s))) return r;
    }
    return SPH_OK;
  };
  for (int l = L - 1; l >= 0; --l) {
    const int64_t kl = tape->k_rec[l];
    const int64_t ns = n_segments(tape, kl);
    if (tape->hist_slow == l) {
      if ((rc = reverse(l, 0, kl))) return rc;
    } else if (ns <= 1) {
      if ((rc = slow_update(l))) return rc;
      if (kl > 0) {
        tape->hist_slow = -1;
        if ((rc = rerun(kl, true))) return rc;
        tape->hist_slow = l;
        if ((rc = reverse(l, 0, kl))) return rc;
      }
    } else {
      // two-level checkpointing: store the start of segments 1 .. ns - 1,
      // then re-run and reverse the segments last to first
      tape->hist_slow = -1;
      if ((rc = slow_update(l))) return rc;
      for (int64_t j = 1; j < ns; ++j) {
        if ((rc = rerun(K, false))) return rc;
        if ((rc = seg_copy(nb, m, st, tape, j - 1, true, s))) return rc;
      }
      for (int64_t j = ns - 1; j >= 0; --j) {
        const int64_t k0 = j * K, k1 = std::min(kl, k0 + K);
        if (j < ns - 1)
          rc = j == 0 ? slow_update(l) : seg_copy(nb, m, st, tape, j - 1, false, s);
        if (rc || (rc = rerun(k1 - k0, true)) || (rc = reverse(l, k0, k1))) return rc;
      }
    }
    if (cfg->slow_kind == SPH_SLOW_DIFFUSION) {
      const void* c_before = (const char*)tape->ck_c + (size_t)l * n * T;
      if ((rc = adj_diffusion(nb, m, st, c_before, adj, cfg->D, dt_slow, s))) return rc;
    } else if (cfg->slow_kind == SPH_SLOW_DIFFUSION_COUPLED) {
      // the step's u is the checkpoint before it (the step leaves u as it is).
      // That u is also the one the previous inner step's drift produced; the
      // drift's transpose was folded into the next reversed gather already
      // (or, if no inner step has been reversed yet, is still to come in
      // adj_drift), so the u_bar added here reaches its velocity only in the
      // first case.
      const void* c_before = (const char*)tape->ck_c + (size_t)l * n * T;
      const double* u_before = tape->ck_u + (size_t)l * d * n;
      const double drift = (!first && before[l] > 0) ? dt : 0.0;
      if ((rc = adj_diffusion_coupled(nb, m, st, u_before, c_before, adj, cfg->D, dt_slow, cfg->c_bc,
                                      cfg->diff_nonlinear, drift, s)))
        return rc;
    }
  }
  if (cfg->batch)
    rc = grad_reduce_batched(nb, st->prec, cfg->batch->grad, s);
  else
    rc = grad_reduce(nb, adj->grad, s);
  if (rc) return rc;
  return tape_copy(nb, m, st, tape, L, false, s);
}

int check_backward_args(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                        const sph_multirate_cfg* cfg, const sph_tape* tape,
                        const sph_adjoint* adj) {
  int rc = check_state(nb, st, true);
  if (rc) return rc;
  if (!m || !cfg || !tape || !adj) {
    set_error("material, cfg, tape or adjoint is NULL");
    return SPH_E_ARG;
  }
  if (cfg->slow_kind == SPH_SLOW_DIFFUSION_COUPLED && cfg->batch) {
    set_error("the reverse of the two-way coupled slow step takes one specimen");
    return SPH_E_UNSUPPORTED;
  }
  if (m->rho_l0 != 0.0) {
    set_error("the reverse pass covers the dry solid only (rho_l0 = 0)");
    return SPH_E_UNSUPPORTED;
  }
  if (adj->prec != st->prec || !adj->u || !adj->v || !adj->work || !adj->grad ||
      (m->model == SPH_MODEL_J2 && !adj->plastic) ||
      (cfg->slow_kind != SPH_SLOW_LOAD && !adj->c)) {
    set_error("adjoint arrays missing or of the wrong precision");
    return SPH_E_ARG;
  }
  return check_tape(nb, m, st, cfg, tape);
}

int finish(const sph_nbr* nb, hipStream_t s, const char* what) {
  SPH_HIP(hipMemcpyAsync(nb->ctrl_host, nb->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  if (nb->prof) prof_resolve(nb);
  if (nb->ctrl_host->status) {
    set_error("device status bits 0x%x in %s", nb->ctrl_host->status, what);
    return SPH_E_NUMERIC;
  }
  return SPH_OK;
}

// Forward run with fixed inner counts, enqueued without host polling (the
// stop flag still ends each inner loop at its count on the device).
int forward_fixed_enqueue(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                          const sph_multirate_cfg* cfg, sph_tape* tape, double dt_s,
                          double dt_slow, std::vector<int64_t>& counts, hipStream_t s) {
  int rc = damp_prepare(nb, m, st, cfg->eta, dt_s, s);
  if (rc) return rc;
  RecGuard rec_guard{nb};
  bool recorded = false;
  for (int32_t l = 0; l < cfg->n_slow; ++l) {
    if (tape && (rc = tape_copy(nb, m, st, tape, l, true, s))) return rc;
    rc = cfg->slow_kind == SPH_SLOW_LOAD ? load_step(nb, st, dt_slow, s)
                                         : diffusion_step(nb, m, st, cfg->D, dt_slow, cfg->c_bc, s);
    if (rc) return rc;
    const int64_t nk = counts[l];
    if (tape) tape->k_rec[l] = nk;
    if (nk <= 0) continue;
    if ((rc = reset_ctrl(nb, nk, -1.0, s))) return rc;
    const bool rec = tape && l == cfg->n_slow - 1 && tape->hist_H && nk <= tape->k_hist_cap &&
                     (m->model != SPH_MODEL_J2 || tape->hist_plastic);
    if (rec) {
      nb->rec_H = tape->hist_H;
      nb->rec_pl = tape->hist_plastic;
      recorded = true;
    }
    if ((rc = inner_steps(nb, m, st, dt_s, cfg->eta, (int)nk, s))) return rc;
    nb->rec_H = nullptr;
    nb->rec_pl = nullptr;
  }
  if (tape) {
    if ((rc = tape_copy(nb, m, st, tape, cfg->n_slow, true, s))) return rc;
    tape->n_rec = cfg->n_slow;
    tape->hist_slow = recorded ? cfg->n_slow - 1 : -1;
    tape->dt_s = dt_s;
    tape->dt_slow = dt_slow;
  }
  return SPH_OK;
}

struct WholeGraph {
  std::vector<unsigned char> key;
  int32_t tape_n_rec = 0, tape_hist_slow = -1;  // the tape's host fields after a run
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~WholeGraph() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
  }
};

}  // namespace

void sph::free_graph_cache(sph_nbr* nb) {
  delete reinterpret_cast<WholeGraph*>(nb->graph_cache);
  nb->graph_cache = nullptr;
  delete reinterpret_cast<ChunkGraph*>(nb->chunk_cache);
  nb->chunk_cache = nullptr;
}

extern "C" int sph_advance_multirate_backward(const sph_nbr* nb, const sph_material* m,
                                              const sph_state* st, const sph_multirate_cfg* cfg,
                                              sph_tape* tape, const sph_adjoint* adj,
                                              void* stream) {
  clear_error();
  int rc = check_backward_args(nb, m, st, cfg, tape, adj);
  if (rc) return rc;
  if (tape->n_rec != cfg->n_slow) {
    set_error("the tape holds %d slow steps, cfg asks for %d", tape->n_rec, cfg->n_slow);
    return SPH_E_ARG;
  }
  if ((rc = check_segments(m, tape, tape->k_rec, cfg->n_slow))) return rc;
  hipStream_t s = (hipStream_t)stream;
  BatGuard bat_guard{nb};
  if ((rc = batch_begin(nb, m, cfg, s))) return rc;
  if ((rc = damp_prepare(nb, m, st, cfg->eta, tape->dt_s, s))) return rc;
  if ((rc = backward_enqueue(nb, m, st, cfg, tape, adj, s))) return rc;
  return finish(nb, s, "the reverse pass");
}

extern "C" int sph_advance_multirate_graph(const sph_nbr* nb, const sph_material* m,
                                           const sph_state* st, const sph_multirate_cfg* cfg,
                                           sph_report* rep, sph_tape* tape,
                                           const sph_adjoint* adj, void* stream) {
  clear_error();
  int rc = check_state(nb, st, true);
  if (rc) return rc;
  if (!m || !cfg || cfg->n_slow < 0 ||
      (cfg->slow_kind != SPH_SLOW_LOAD && cfg->slow_kind != SPH_SLOW_DIFFUSION)) {
    set_error("bad material or cfg (the whole-run graph takes loading and linear diffusion steps)");
    return SPH_E_ARG;
  }
  if (m->rho_l0 != 0.0) {
    set_error("the whole-run graph takes the dry solid only (rho_l0 = 0)");
    return SPH_E_UNSUPPORTED;
  }
  if (cfg->k_sched == nullptr && cfg->fixed_inner <= 0) {
    set_error("the whole-run graph needs fixed inner counts (fixed_inner or k_sched)");
    return SPH_E_ARG;
  }
  if (adj && (rc = check_backward_args(nb, m, st, cfg, tape, adj))) return rc;
  if (tape && (rc = check_tape(nb, m, st, cfg, tape))) return rc;
  std::vector<int64_t> counts(std::max(cfg->n_slow, 1));
  for (int l = 0; l < cfg->n_slow; ++l)
    counts[l] = cfg->k_sched ? cfg->k_sched[l] : cfg->fixed_inner;
  if (adj && (rc = check_segments(m, tape, counts.data(), cfg->n_slow))) return rc;
  double dt_rest = 0.0, dt_diff = 0.0;
  rest_steps(nb->h, m, cfg->D, &dt_rest, &dt_diff);
  const double dt_s = cfg->dt_s > 0.0 ? cfg->dt_s : dt_rest;
  double dt_slow = cfg->dt_slow;
  if (cfg->slow_kind == SPH_SLOW_DIFFUSION && !(dt_slow > 0.0)) {
    if (!(cfg->D > 0.0) && !cfg->batch) {
      set_error("diffusion needs D > 0");
      return SPH_E_ARG;
    }
    dt_slow = cfg->D > 0.0 ? dt_diff : 1.0;  // batched: per specimen
  }
  hipStream_t user = (hipStream_t)stream;
  BatGuard bat_guard{nb};
  if ((rc = batch_begin(nb, m, cfg, user))) return rc;
  // the key: every argument the recorded launches depend on
  std::vector<unsigned char> key;
  key_add(key, m);
  sph_multirate_cfg c2 = *cfg;
  c2.k_sched = nullptr;
  c2.batch = nullptr;
  key_add(key, &c2);
  for (int l = 0; l < cfg->n_slow; ++l) key_add(key, &counts[l]);
  if (cfg->batch) {
    key_add(key, &cfg->batch->n_spec);
    key_add(key, &cfg->batch->grad);
  }
  key_add(key, st);
  if (tape) {
    sph_tape t2 = *tape;
    t2.n_rec = 0;
    t2.hist_slow = 0;
    t2.dt_s = t2.dt_slow = 0.0;
    key_add(key, &t2);
  } else {
    key.push_back(0);
  }
  key_add(key, adj);
  WholeGraph* wg = reinterpret_cast<WholeGraph*>(nb->graph_cache);
  if (!wg || wg->key != key) {
    free_graph_cache(const_cast<sph_nbr*>(nb));
    wg = new WholeGraph();
    const_cast<sph_nbr*>(nb)->graph_cache = wg;
    hipStream_t cap = nullptr;
    SPH_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    if (nb->prof) nb->prof->suspend = true;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      rc = forward_fixed_enqueue(nb, m, st, cfg, tape, dt_s, dt_slow, counts, cap);
      if (rc == SPH_OK && adj) rc = backward_enqueue(nb, m, st, cfg, tape, adj, cap);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(cap, &g);
      wg->graph = g;
    }
    if (nb->prof) nb->prof->suspend = false;
    hipStreamDestroy(cap);
    if (rc == SPH_OK && e != hipSuccess) {
      set_error("graph capture failed: %s", hipGetErrorString(e));
      rc = SPH_E_DEVICE;
    }
    if (rc == SPH_OK && hipGraphInstantiate(&wg->exec, wg->graph, nullptr, nullptr, 0) != hipSuccess) {
      set_error("graph instantiation failed");
      rc = SPH_E_DEVICE;
    }
    if (rc) {
      free_graph_cache(const_cast<sph_nbr*>(nb));
      return rc;
    }
    wg->key = key;
    if (tape) {
      wg->tape_n_rec = tape->n_rec;
      wg->tape_hist_slow = tape->hist_slow;
    }
  } else if (tape) {
    // the host-side bookkeeping of the recorded run, the same on every launch
    for (int l = 0; l < cfg->n_slow; ++l) tape->k_rec[l] = counts[l];
    tape->n_rec = wg->tape_n_rec;
    tape->hist_slow = wg->tape_hist_slow;
    tape->dt_s = dt_s;
    tape->dt_slow = dt_slow;
  }
  SPH_HIP(hipGraphLaunch(wg->exec, user));
  if (rep) {
    rep->dt_s = dt_s;
    rep->dt_slow = dt_slow;
    rep->k_max = 0;
    rep->total_inner = 0;
    for (int l = 0; l < cfg->n_slow; ++l) {
      if (rep->k) rep->k[l] = counts[l];
      if (rep->ke) rep->ke[l] = 0.0;
      if (rep->converged) rep->converged[l] = 0;
      rep->total_inner += counts[l];
    }
  }
  return finish(nb, user, "the whole-run graph");
}
