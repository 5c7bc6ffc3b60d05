// sph_common.h -- internal declarations of the gfx950 SPH library.
// Not part of the C ABI (include/sph.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstdio>
#include <string>

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

constexpr int kKeThreads = 256;
constexpr int kKeMaxBlocks = 2048;

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
  uint32_t* sa = nullptr;
  uint32_t* sb = nullptr;
  uint32_t* slev = nullptr;
  uint32_t* akey = nullptr;
  int64_t* aoff = nullptr;
  uint32_t* anlev = nullptr;
  // inner-loop control
  sph::Ctrl* ctrl = nullptr;         // device
  sph::Ctrl* ctrl_host = nullptr;    // pinned host mirror
  double* ke_partial = nullptr;      // device [kKeMaxBlocks]
  int device = 0;
};

namespace sph {

// ---- kernel function: Wendland C2, support 2h --------------------------------
// (dW/dr)/r = c5 (1 - q/2)^3 with q = r/h, c5 = -5 alpha_d / h^2.
template <typename T>
__device__ __forceinline__ T dw_over_r(T r2, T inv_h, T c5) {
  T q = sqrt(r2) * inv_h;
  T t = T(1) - T(0.5) * q;
  return c5 * t * t * t;
}

// ---- host entry points implemented per translation unit ----------------------
int solid_stage(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
                hipStream_t s, bool gated);
int damping_sweep(const sph_nbr* nb, const sph_material* m, const sph_state* st, double eta,
                  double dt, hipStream_t s, bool gated);
int drift_ke(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
             double* ke_out, hipStream_t s, bool gated);
int load_step(const sph_nbr* nb, const sph_state* st, double dt_l, hipStream_t s);
int diffusion_step(const sph_nbr* nb, const sph_material* m, const sph_state* st, double D,
                   double dt_d, double c_bc, hipStream_t s);
int reset_ctrl(const sph_nbr* nb, int64_t k_limit, double ke_tol, hipStream_t s);
int check_state(const sph_nbr* nb, const sph_state* st, bool need_v);

}  // namespace sph
