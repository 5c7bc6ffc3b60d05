// sph_common.h -- internal declarations of the gfx950 SPH library.
// Not part of the C ABI (include/sph.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "sph.h"

namespace sph {

void set_error(const char* fmt, ...);
void clear_error();

#define SPH_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      ::sph::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call, hipGetErrorString(e_)); \
      return SPH_E_DEVICE;                                                              \
    }                                                                                   \
  } while (0)

#define SPH_LAUNCH_CHECK()                                                              \
  do {                                                                                  \
    hipError_t e_ = hipGetLastError();                                                  \
    if (e_ != hipSuccess) {                                                             \
      ::sph::set_error("%s:%d launch: %s", __FILE__, __LINE__, hipGetErrorString(e_));  \
      return SPH_E_DEVICE;                                                              \
    }                                                                                   \
  } while (0)

// Device control block of one handle: the inner-loop stop state.
struct Ctrl {
  int32_t done;      // 1 once the current inner loop has stopped
  int32_t status;    // SPH_STATUS_* bits (sticky until sph_status)
  int64_t k;         // inner steps taken in the current slow step
  int64_t k_limit;   // stop after this many steps
  double ke;         // kinetic energy after the last step
  double ke_tol;     // early-exit threshold (negative: never)
  uint32_t ticket;   // last-block election of the kinetic-energy reduction
  int32_t stopped_by_ke;
};

// per-kernel event timing (see sph_profile_enable)
struct Prof {
  bool on = false;
  uint32_t mask = 0xFFFFFFFFu;  // kernel classes timed while on
  bool suspend = false;  // set while a graph is being captured
  struct Pend {
    int kind;
    hipEvent_t a, b;
    int launches;  // kernels between the two events
  };
  std::vector<hipEvent_t> pool;
  std::vector<Pend> pend;
  int64_t count[SPH_KERNEL_COUNT] = {0};
  double ms[SPH_KERNEL_COUNT] = {0};
};

// one segment of the cell grid (one specimen): origin, cell counts, first key
struct GridSeg {
  int64_t nc0, nc1, nc2;
  double o0, o1, o2;
  int64_t koff;
};

// Per-specimen values of a batched run, one row per field, n_spec columns;
// kernels read them through each particle's specimen id.
enum BatchField { BT_MU = 0, BT_K, BT_LAM, BT_DT, BT_DTD, BT_D, BT_ETADT, BT_COUNT };
struct Bat {
  const uint16_t* spec = nullptr;  // [n] specimen of each sorted particle; nullptr: not batched
  const float* t32 = nullptr;      // [BT_COUNT][ns]
  const double* t64 = nullptr;     // [BT_COUNT][ns]
  int64_t ns = 0;
  template <typename T>
  __device__ __forceinline__ T get(int f, int s) const {
    if constexpr (sizeof(T) == 8) return t64[f * ns + s];
    else return t32[f * ns + s];
  }
};

// tuned launch shapes of one handle (sph_autotune): lanes per particle of the
// four tiled gather kernels, per precision, and the damping lane-group width
// per precision and colour (0: the automatic rule)
enum TuneKernel { TUNE_STRESS = 0, TUNE_MOMENTUM, TUNE_ADJ_STRESS, TUNE_ADJ_GATHER, TUNE_COUNT };
struct Tune {
  // [kernel][SPH_F32, SPH_F64]: the tuned choices on the 1M-particle plate
  int lpp[TUNE_COUNT][2] = {{1, 2}, {2, 4}, {1, 2}, {2, 4}};
  int damp_g[2][8] = {{0, 0, 0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0, 0, 0}};
  // idle lanes of a damping row: 0 automatic, 1 spare slot, 2 skip
  int damp_idle[2][8] = {{0, 0, 0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0, 0, 0}};
};

// reverse diffusion gathers (CSR lists): lanes per particle, threads per block
constexpr int kDiffLanes = 8;
constexpr int kDiffBlock = 1024;
constexpr int kDiffPerBlock = kDiffBlock / kDiffLanes;

constexpr int kPollFirst = 16;          // inner steps before an adaptive run's first poll
constexpr int kKeThreads = 256;
constexpr int kKeItems = 4;             // particles per thread in the drift kernel
constexpr int kKeFinishBlocks = 64;     // drift grids this small reduce E_k in their last block
constexpr int kKeMaxBlocks = 1 << 16;   // partial sums (67M particles)
constexpr int kStaticKeBlocks = 1 << 16;  // sph_drift_ke_noalloc: 512 KiB of partials per GPU

// A tile is a run of consecutive sorted particles inside one row of cells
// (fixed y, z).  Its neighbours all lie in the "window": the 3^(d-1) rows
// around it, each clipped to cells [x0-1, x1+1] -- contiguous particle runs,
// which a workgroup stages in LDS.  Neighbour lists of the tile are stored as
// window-local 16-bit indices in a blocked ELL layout: entries are grouped in
// fours, entry j of tile particle t is
//   ell[ell_off + (j / 4) * 4 * tmax + 4 * t + j % 4],
// so one lane loads four indices with one 8-byte load and a wavefront's loads
// are contiguous; entries past a particle's degree hold its own index (a zero
// contribution).  `width` is a multiple of 4.
// A tile's own particles are one run of a row of cells, or two runs (the same
// x-range of two stacked rows): own particle s < count0 is p0 + s at window
// position own_base + s, the others p1 + (s - count0) at own_base1 +
// (s - count0).  The window is the concatenation of nruns runs of sorted
// particles (the neighbouring rows' cells over the x-range widened by one).
// Thread slots take the own particles by descending neighbour count (stable),
// so that the lanes of a wavefront walk lists of about one length and stop
// at their own: tslot[tile][t] = s | (blocks of four entries of s's list)
// << 16 (0 for t >= count).
struct TileDesc {
  uint32_t p0, count, ell_off, width;
  uint32_t nruns, window, own_base, count0;
  uint32_t p1, own_base1, pad0, pad1;
  uint32_t run_start[9];
  uint32_t run_count[9];
};

struct Tiling {
  int tmax = 0;            // particles per tile (threads per particle x tmax = block)
  int64_t n_tiles = 0;
  int64_t window_max = 0;  // largest window, sizes the dynamic LDS
  int64_t ell_len = 0;
  TileDesc* tiles = nullptr;  // device
  uint16_t* ell = nullptr;    // device
  uint32_t* tslot = nullptr;  // device [n_tiles][tmax]
};

// damping pair word: a_loc | b_loc << 16 (locals inside the anchor's
// 2^d-cell block, in ascending sorted order); each anchor's level offsets sit
// in dloff; the joint rows of the wavefronts for lane-group width 8 << i
// (64 >> (3 + i) anchors per wavefront) in drow[i], dwave[i], ...
constexpr int kDampLocBits = 16;
constexpr int kDampWidths = 4;          // lane-group widths 8, 16, 32, 64
constexpr int kDampRowPad = 24;         // empty rows framing each wavefront's row list (3K)
constexpr int kDampMaxLocal = 1 << kDampLocBits;
constexpr int kDampMaxLevel = 255;      // levels of one anchor (offsets held in 4 registers)
constexpr int64_t kDampLdsBudget = 159 * 1024;  // gfx950: 160 KB of LDS per workgroup

}  // namespace sph

struct sph_nbr {
  int dim = 0;
  int64_t n = 0, n_pairs = 0, n_upairs = 0, n_cells = 0, n_anchors = 0, max_deg = 0, max_level = 0;
  int64_t nc[3] = {1, 1, 1};
  int64_t color_off[9] = {0};
  double origin[3] = {0, 0, 0};
  double h = 0, inv_rc = 0;
  double c5 = 0;     // (dW/dr)/r = c5 (1 - q/2)^3, c5 = -5 alpha_d / h^2
  double inv_h = 0;
  // device arrays
  uint32_t* key = nullptr;
  uint32_t* perm = nullptr;
  uint32_t* cell_start = nullptr;
  int64_t* nbr_off = nullptr;
  uint32_t* nbr_idx = nullptr;
  double* X = nullptr;
  double* V = nullptr;
  double* B0 = nullptr;
  float* Vf = nullptr;
  float* B0f = nullptr;
  double* gsum = nullptr;  // [dim][n] sum_b V_b grad_a W_ab (fixed reference configuration; tile_gsum)
  float* gsumf = nullptr;
  uint32_t* sa = nullptr;
  uint32_t* sb = nullptr;
  uint32_t* slev = nullptr;
  uint32_t* akey = nullptr;
  int64_t* aoff = nullptr;
  uint32_t* anlev = nullptr;
  uint32_t* dpair = nullptr;         // [n_upairs] packed damping pairs (canonical order)
  uint16_t* dloff = nullptr;         // level offsets of every anchor (relative to its first pair)
  uint32_t* dloff_base = nullptr;    // [n_anchors] start of each anchor's offsets in dloff
  uint32_t* ablk = nullptr;          // [n_anchors][8] anchor block runs (begin, count) x 4
  int64_t damp_block_max = 0;        // largest anchor block (particles)
  int64_t damp_pairs_max = 0;        // largest pair count of one anchor
  int64_t damp_bmax[8] = {0};        // the same, per colour (sizes each pass's LDS)
  int64_t damp_pmax[8] = {0};
  // joint rows of the damping sweep per lane-group width (build_joint_rows)
  uint32_t* drow[sph::kDampWidths] = {};       // row words first | end << 16, framed per wavefront
  int64_t* drow_base[sph::kDampWidths] = {};   // [n_waves + 1] start of each wavefront's framed list
  uint32_t* dwave[sph::kDampWidths] = {};      // [n_waves][64 / G][8] block runs of its anchors
  uint32_t* dwrec[sph::kDampWidths] = {};      // [n_waves] first record, from the colour's first pair
  uint32_t* djinfo[sph::kDampWidths] = {};     // [n_upairs] record position | group << 28
  int64_t dwave_off[sph::kDampWidths][9] = {}; // first wavefront of each colour
  bool dwidth_ok[sph::kDampWidths] = {};       // every wavefront's records fit the row words
  mutable int damp_g_used[2][8] = {};          // widths the per-run records were laid out for
  int64_t damp_pair_off[9] = {};               // first pair of each colour (canonical order)
  float* dgeo32 = nullptr;           // [n_upairs] 2 V_a V_b (dW/dr)/r per pair
  double* dgeo64 = nullptr;
  sph::Tiling tiling[2];             // [SPH_F32], [SPH_F64]
  // inner-loop control
  sph::Ctrl* ctrl = nullptr;         // device
  sph::Ctrl* ctrl_host = nullptr;    // pinned host mirror
  double* ke_partial = nullptr;      // device [kKeMaxBlocks]
  double* gpart = nullptr;           // device [gpart_slots][SPH_NGRAD] gradient partials
  int64_t gpart_slots = 0;
  // inner-step recording of a taped run (set by the driver while it runs)
  mutable void* rec_H = nullptr;     // [k][dim*dim][n]: H = F - I of inner step k
  mutable void* rec_pl = nullptr;    // [k][7][n]: J2 state before inner step k
  // cell-grid segments (one per specimen) and the segment of each cell
  std::vector<sph::GridSeg> segs;
  sph::GridSeg* dsegs = nullptr;
  uint16_t* cell_seg = nullptr;
  // specimen batch (sph_build_neighbors_batched); bat_on is set by the driver during a batched run
  int64_t n_spec = 0;
  uint16_t* spec = nullptr;          // [n] specimen of each sorted particle
  std::vector<int64_t> spec_off;     // host [n_spec+1] sorted-position ranges
  int64_t* spec_off_dev = nullptr;   // device copy
  float* bt32 = nullptr;             // [BT_COUNT][n_spec]
  double* bt64 = nullptr;
  double* gdiff = nullptr;           // [2][n] per-particle diffusion-gradient partials (batched)
  mutable bool bat_on = false;
  // per-run damping coefficients (k_damp_prep), [SPH_F32] float / [SPH_F64] double
  void* dwq[2] = {nullptr, nullptr};    // [n_upairs] PairQ: pair word and q of every pair
  void* imass[2] = {nullptr, nullptr};  // [n] inverse mass (0 for fixed particles)
  mutable bool damp_pre = false;        // set by the driver while they are valid
  void* graph_cache = nullptr;       // instantiated whole-run graph (sph_advance_multirate_graph)
  void* chunk_cache = nullptr;       // instantiated chunk of inner steps (sph_advance_multirate)
  // the per-step scratch (dwq, imass, ke_partial, gpart) is carved from one
  // block: the handle's own (ws_own) or the caller's (sph_set_workspace)
  void* ws_own = nullptr;
  sph::Tune tune;                    // launch shapes (sph_autotune)
  int device = 0;
  sph::Prof* prof = nullptr;         // host-side timing state
};

namespace sph {

inline Bat bat_view(const sph_nbr* nb) {
  Bat b;
  if (nb->bat_on) {
    b.spec = nb->spec;
    b.t32 = nb->bt32;
    b.t64 = nb->bt64;
    b.ns = nb->n_spec;
  }
  return b;
}

// ---- kernel function: Wendland C2, support 2h --------------------------------
// (dW/dr)/r = c5 (1 - q/2)^3 with q = r/h, c5 = -5 alpha_d / h^2.
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }  // 1 ulp
__device__ __forceinline__ double hw_sqrt(double x) { return sqrt(x); }

template <typename T>
__device__ __forceinline__ T dw_over_r(T r2, T inv_h, T c5) {
  T q = hw_sqrt(r2) * inv_h;
  T t = T(1) - T(0.5) * q;
  return c5 * t * t * t;
}

// ---- tiling parameters per precision -----------------------------------------
// LDS bytes per staged window particle of the widest tiled kernels: in 3D the
// momentum sum and its transpose (relative position and a 3 x 3 tensor, twelve
// values), in 2D the stress stages (two 4-vectors); the formula is
// ceil((dim + dim^2) / 4) 4-vectors, which covers both.
// Particles per tile: 256 in FP32 (a workgroup of 256 x lanes threads, the
// window's staging shared by more particles), 64 in FP64.
inline int tile_tmax(int prec) { return prec == SPH_F64 ? 64 : 256; }
inline int64_t tile_lds_bytes_per_particle(int prec, int dim) {
  const int t = prec == SPH_F64 ? 8 : 4;
  return (int64_t)t * 4 * ((dim + dim * dim + 3) / 4);
}
constexpr int64_t kTileLdsBudget = 80 * 1024;
inline int64_t tile_wmax(int prec, int dim) {
  return std::min<int64_t>(65535, kTileLdsBudget / tile_lds_bytes_per_particle(prec, dim));
}
constexpr int64_t kTileLdsHard = 159 * 1024;  // gfx950: 160 KB of LDS per workgroup
inline int64_t tile_wmax_hard(int prec, int dim) {
  return std::min<int64_t>(65535, kTileLdsHard / tile_lds_bytes_per_particle(prec, dim));
}

// ---- step sizes of Sec. 4.1 (sph_default_steps) -------------------------------
// dt_s = 0.6 h / sqrt(K / rho0), eq. (dts-advection) at rest; dt_d = 0.5 h^2 / D
// (0 for D <= 0); K from eq. (relation-modulus)
inline void rest_steps(double h, const sph_material* m, double D, double* dt_s, double* dt_d) {
  const double K = m->E / (3.0 * (1.0 - 2.0 * m->nu));
  if (dt_s) *dt_s = 0.6 * h / std::sqrt(K / m->rho0);
  if (dt_d) *dt_d = D > 0.0 ? 0.5 * h * h / D : 0.0;
}

// ---- event timing around launches --------------------------------------------
hipEvent_t prof_begin(const sph_nbr* nb, int kind, hipStream_t s);
void prof_end(const sph_nbr* nb, int kind, hipEvent_t a, hipStream_t s, int launches = 1);
int prof_resolve(const sph_nbr* nb);

// ---- host entry points implemented per translation unit ----------------------
int solid_stage(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
                hipStream_t s, bool gated);
// one colour pass of the forward sweep with the records already laid out
// (the tuner times passes one by one)
int damping_pass(const sph_nbr* nb, const sph_state* st, int col, hipStream_t s);
int damping_sweep(const sph_nbr* nb, const sph_material* m, const sph_state* st, double eta,
                  double dt, hipStream_t s, bool gated);
int damping_sweep_rev(const sph_nbr* nb, const sph_material* m, const sph_state* st, double eta,
                      double dt, hipStream_t s);
int damp_prepare(const sph_nbr* nb, const sph_material* m, const sph_state* st, double eta,
                 double dt, hipStream_t s);
int drift_ke(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
             double* ke_out, hipStream_t s, bool gated);
// drift_ke with its partials in a static device array (no library-owned scratch)
int drift_ke_static(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
                    double* ke_out, hipStream_t s);
int load_step(const sph_nbr* nb, const sph_state* st, double dt_l, hipStream_t s);
int diffusion_step_coupled(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                           double D, double dt, double c_bc, int nonlinear, hipStream_t s);
int diffusion_step(const sph_nbr* nb, const sph_material* m, const sph_state* st, double D,
                   double dt_d, double c_bc, hipStream_t s);
int reset_ctrl(const sph_nbr* nb, int64_t k_limit, double ke_tol, hipStream_t s);
int check_state(const sph_nbr* nb, const sph_state* st, bool need_v);
int check_mixture(const sph_material* m, const sph_state* st);
// H = F - I of st->u into H ([dim*dim][n], st->prec): the stress stage's gather
int displacement_gradient(const sph_nbr* nb, const sph_state* st, void* H, hipStream_t s);
// reverse mode (sph_adjoint.hip); H: the step's F - I ([dim*dim][n]), may
// alias adj->work (each particle's entries are read before its own are written)
int adj_solid(const sph_nbr* nb, const sph_material* m, const void* H, const void* plastic,
              const sph_state* st, const sph_adjoint* adj, double dt, double drift_dt,
              hipStream_t s);
int adj_damping(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                const sph_adjoint* adj, double eta, double dt, hipStream_t s);
int adj_drift(const sph_nbr* nb, const sph_state* st, const sph_adjoint* adj, double dt,
              hipStream_t s);
// g_a = sum_b V_b grad_a W_ab into nb->gsum (FP64) and nb->gsumf (FP32), each
// with the tiled gathers' arithmetic of its precision (needs both tilings)
int tile_gsum(const sph_nbr* nb, hipStream_t s);
int diffusion_F(const sph_nbr* nb, int prec, const double* u, const void* c, void* Fi, void* sat,
                hipStream_t s);
// drift_dt: the step of the inner step before the slow step when that inner
// step's drift transpose has already been taken (0 otherwise); the u_bar
// this reverse adds then also reaches that drift's velocity
int adj_diffusion_coupled(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                          const double* u_before, const void* c_before, const sph_adjoint* adj,
                          double D, double dt, double c_bc, int nonlinear, double drift_dt,
                          hipStream_t s);
int adj_diffusion(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                  const void* c_before, const sph_adjoint* adj, double Dc, double dt,
                  hipStream_t s);
int grad_reduce(const sph_nbr* nb, double* grad, hipStream_t s);
// specimen batches (sph_batch.hip)
int batch_check(const sph_nbr* nb, const sph_multirate_cfg* cfg);
int batch_finish(sph_nbr* nb, int32_t n_spec, const int32_t* spec_id, hipStream_t s);
int batch_upload(const sph_nbr* nb, const sph_material* m, const sph_multirate_cfg* cfg,
                 hipStream_t s);
int grad_reduce_batched(const sph_nbr* nb, int prec, double* out, hipStream_t s);
void free_graph_cache(sph_nbr* nb);

}  // namespace sph
