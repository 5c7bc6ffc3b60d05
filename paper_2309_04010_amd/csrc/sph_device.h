// sph_device.h -- device-side building blocks shared by the forward and
// adjoint kernels: geometry views, 3x3 algebra, the constitutive update,
// LDS tile staging helpers and the blocked-ELL neighbour walk.
#pragma once

#include <hip/hip_runtime.h>

#include "sph_common.h"

namespace sph {

template <typename T>
struct Geo {
  const double* X;
  const T* V;
  const T* B0;
  const int64_t* off;
  const uint32_t* idx;
  int64_t n;
  T inv_h, c5;
  const T* gsum;  // [dim][n] sum_b V_b grad_a W_ab
};

template <typename T>
static Geo<T> geo(const sph_nbr* nb) {
  if constexpr (sizeof(T) == 8)
    return Geo<T>{nb->X, nb->V, nb->B0, nb->nbr_off, nb->nbr_idx, nb->n, nb->inv_h, nb->c5,
                  nb->gsum};
  else
    return Geo<T>{nb->X, nb->Vf, nb->B0f, nb->nbr_off, nb->nbr_idx, nb->n, (float)nb->inv_h,
                  (float)nb->c5, nb->gsumf};
}

// ---------------------------------------------------------------------------
// 3x3 helpers (row-major)
template <typename T>
__device__ __forceinline__ T det3(const T* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}
template <typename T>
__device__ __forceinline__ void inv3(const T* A, T d, T* Ai) {
  T r = T(1) / d;
  Ai[0] = (A[4] * A[8] - A[5] * A[7]) * r;
  Ai[1] = (A[2] * A[7] - A[1] * A[8]) * r;
  Ai[2] = (A[1] * A[5] - A[2] * A[4]) * r;
  Ai[3] = (A[5] * A[6] - A[3] * A[8]) * r;
  Ai[4] = (A[0] * A[8] - A[2] * A[6]) * r;
  Ai[5] = (A[2] * A[3] - A[0] * A[5]) * r;
  Ai[6] = (A[3] * A[7] - A[4] * A[6]) * r;
  Ai[7] = (A[1] * A[6] - A[0] * A[7]) * r;
  Ai[8] = (A[0] * A[4] - A[1] * A[3]) * r;
}
template <typename T>
__device__ __forceinline__ void mul3(const T* A, const T* B, T* C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[i * 3 + j] = A[i * 3] * B[j] + A[i * 3 + 1] * B[3 + j] + A[i * 3 + 2] * B[6 + j];
}
template <typename T>
__device__ __forceinline__ void mul3_bt(const T* A, const T* B, T* C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C[i * 3 + j] = A[i * 3] * B[j * 3] + A[i * 3 + 1] * B[j * 3 + 1] + A[i * 3 + 2] * B[j * 3 + 2];
}

template <typename T>
struct MatP {
  int model;
  T mu, K, lam;
  T s0, sinf, delta, H;
  T newton_tol;  // relative tolerance of the return-mapping residual
  T dmu_dE, dK_dE;  // mu and K are proportional to E (nu fixed)
};

template <typename T>
__device__ __forceinline__ T hardening(const MatP<T>& m, T a) {
  return m.s0 + (m.sinf - m.s0) * (T(1) - exp(-m.delta * a)) + m.H * a;
}
template <typename T>
__device__ __forceinline__ T hardening_slope(const MatP<T>& m, T a) {
  return (m.sinf - m.s0) * m.delta * exp(-m.delta * a) + m.H;
}

// S = A + A^T + A A^T  (= (I+A)(I+A)^T - I)
template <typename T>
__device__ __forceinline__ void sym_sum(const T* A, T* S) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      S[i * 3 + j] = A[i * 3 + j] + A[j * 3 + i] + A[i * 3] * A[j * 3] + A[i * 3 + 1] * A[j * 3 + 1] +
                     A[i * 3 + 2] * A[j * 3 + 2];
}

// First Piola-Kirchhoff stress of one particle from H = F - I; returns
// SPH_STATUS_NEWTON on a failed return mapping.  App. A.2-A.4 and B.2 of the
// paper (LE is the small-strain reading).  Strain measures come from H by
// exact identities (det(I+H) - 1, F F^T - I) so FP32 keeps small strains.
// pl: Cbar_p^-1 - I (xx,yy,zz,xy,yz,xz) and alpha.
// MODEL >= 0 fixes the material model at compile time (a kernel specialised
// for one model carries only that model's code and registers); -1 reads it
// from m at run time
template <int MODEL, typename T>
__device__ __forceinline__ bool model_is(const MatP<T>& m, int k) {
  if constexpr (MODEL >= 0) return MODEL == k;
  else return m.model == k;
}

template <typename T, int MODEL = -1>
__device__ int constitutive(const MatP<T>& m, const T* H, T* pl, T p, T* P) {
  T trH = H[0] + H[4] + H[8];
  T trH2 = H[0] * H[0] + H[4] * H[4] + H[8] * H[8] + T(2) * (H[1] * H[3] + H[2] * H[6] + H[5] * H[7]);
  T jm1 = trH + T(0.5) * (trH * trH - trH2) + det3(H);
  T J = T(1) + jm1;
  T F[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) F[i] = H[i];
  F[0] += T(1);
  F[4] += T(1);
  F[8] += T(1);
  T Fi[9];
  inv3(F, J, Fi);
  int st = 0;
  T tau[9];
  const T vol = T(0.5) * m.K * jm1 * (T(2) + jm1);
  if (model_is<MODEL>(m, SPH_MODEL_LE)) {
    T tm = T(2) * m.mu;
    P[0] = tm * H[0] + m.lam * trH;
    P[4] = tm * H[4] + m.lam * trH;
    P[8] = tm * H[8] + m.lam * trH;
    P[1] = P[3] = m.mu * (H[1] + H[3]);
    P[2] = P[6] = m.mu * (H[2] + H[6]);
    P[5] = P[7] = m.mu * (H[5] + H[7]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) P[i * 3 + j] -= J * p * Fi[j * 3 + i];
    return 0;
  }
  if (model_is<MODEL>(m, SPH_MODEL_NH)) {
    T Bm[9];
    sym_sum(H, Bm);
    T cb = cbrt(J);
    T s23 = T(1) / (cb * cb);
    T tr3 = (Bm[0] + Bm[4] + Bm[8]) * (T(1) / T(3));
    T ms = m.mu * s23;
#pragma unroll
    for (int i = 0; i < 9; ++i) tau[i] = ms * Bm[i];
    tau[0] += vol - ms * tr3;
    tau[4] += vol - ms * tr3;
    tau[8] += vol - ms * tr3;
  } else {
    // Algorithm 1 with Fbar = c F, c = J^(-1/3); Hb = Fbar - I; E = bbar_pre - I
    T c = T(1) / cbrt(J);
    T cm1 = expm1(log1p(jm1) * T(-1.0 / 3.0));
    T Hb[9], Fb[9], Y[9], FFm[9], tmp[9], E[9], s[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Hb[i] = c * H[i];
    Hb[0] += cm1;
    Hb[4] += cm1;
    Hb[8] += cm1;
#pragma unroll
    for (int i = 0; i < 9; ++i) Fb[i] = Hb[i];
    Fb[0] += T(1);
    Fb[4] += T(1);
    Fb[8] += T(1);
    Y[0] = pl[0]; Y[4] = pl[1]; Y[8] = pl[2];
    Y[1] = Y[3] = pl[3];
    Y[5] = Y[7] = pl[4];
    Y[2] = Y[6] = pl[5];
    T alpha = pl[6];
    sym_sum(Hb, FFm);
    mul3(Fb, Y, tmp);
    mul3_bt(tmp, Fb, E);
#pragma unroll
    for (int i = 0; i < 9; ++i) E[i] += FFm[i];
    T trE3 = (E[0] + E[4] + E[8]) * (T(1) / T(3));
    T n2 = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      s[i] = m.mu * E[i];
      if (i == 0 || i == 4 || i == 8) s[i] -= m.mu * trE3;
      n2 += s[i] * s[i];
    }
    T sn = sqrt(n2);
    const T r23 = T(0.816496580927726);  // sqrt(2/3)
    T f = sn - r23 * hardening(m, alpha);
    if (f > T(0)) {
      T mub = m.mu * (T(1) + trE3);
      T dg = 0;
      T tol = m.newton_tol * (sn > T(1) ? sn : T(1));
      bool ok = false;
      for (int it = 0; it < 50; ++it) {
        T a1 = alpha + r23 * dg;
        T fh = sn - r23 * hardening(m, a1) - T(2) * mub * dg;
        if (fabs(fh) <= tol) {
          ok = true;
          break;
        }
        T dfh = -(T(2) / T(3)) * hardening_slope(m, a1) - T(2) * mub;
        dg -= fh / dfh;
      }
      if (!ok) st = SPH_STATUS_NEWTON;
      T fac = T(1) - T(2) * mub * dg / sn;
#pragma unroll
      for (int i = 0; i < 9; ++i) s[i] *= fac;
      alpha += r23 * dg;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) tau[i] = s[i];
    tau[0] += vol;
    tau[4] += vol;
    tau[8] += vol;
    // Y = Fbar^-1 ((bbar_e - I) - (Fbar Fbar^T - I)) Fbar^-T, bbar_e = s/mu + tr(bbar_pre)/3 I
    T Dm[9], Fbi[9], t2[9], Yn[9];
    T imu = T(1) / m.mu;
#pragma unroll
    for (int i = 0; i < 9; ++i) Dm[i] = s[i] * imu - FFm[i];
    Dm[0] += trE3;
    Dm[4] += trE3;
    Dm[8] += trE3;
    inv3(Fb, det3(Fb), Fbi);
    mul3(Fbi, Dm, t2);
    mul3_bt(t2, Fbi, Yn);
    pl[0] = Yn[0]; pl[1] = Yn[4]; pl[2] = Yn[8];
    pl[3] = Yn[1]; pl[4] = Yn[5]; pl[5] = Yn[2];
    pl[6] = alpha;
  }
  // P = (tau - J p I) F^-T
  tau[0] -= J * p;
  tau[4] -= J * p;
  tau[8] -= J * p;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      P[i * 3 + j] = tau[i * 3] * Fi[j * 3] + tau[i * 3 + 1] * Fi[j * 3 + 1] + tau[i * 3 + 2] * Fi[j * 3 + 2];
  return st;
}

// ---------------------------------------------------------------------------
// LDS-staged tile kernels.  One workgroup per tile; LPP lanes per particle
// (adjacent lanes of one wavefront) split its neighbour list and reduce with
// lane shuffles.  Tiles are taken in an XCD-aware order: workgroup b runs on
// XCD (b mod 8) and gets a tile from a contiguous eighth of the tile list, so
// neighbouring tiles -- which share most of their windows -- hit one L2.
template <typename T>
using vec4 = T __attribute__((ext_vector_type(4)));

// lanes per particle of the tile kernels (1, 2 or 4; a workgroup is
// tile_tmax x lanes threads, at most 256 x 4): per-handle choices (Tune), set
// by sph_autotune, else the defaults (in FP32 1 for the stress kernels, 2 for
// the momentum-shaped ones, which read more LDS per pair; twice that in FP64)

template <typename T>
struct TileGeo {
  const TileDesc* tiles;
  const uint16_t* ell;
  const uint32_t* tslot;
  int tmax;
  int64_t n_tiles;
  const double* X;
  const T* V;
  const T* B0;
  int64_t n;
  T inv_h, c5;
  const T* gsum;  // [dim][n] sum_b V_b grad_a W_ab
};

template <typename T>
static TileGeo<T> tile_geo(const sph_nbr* nb, int prec) {
  const Tiling& t = nb->tiling[prec];
  Geo<T> g = geo<T>(nb);
  return TileGeo<T>{t.tiles, t.ell, t.tslot, t.tmax, t.n_tiles, g.X, g.V, g.B0, g.n, g.inv_h, g.c5,
                    g.gsum};
}

// N values per window particle as N/4 arrays of 4-vectors ([N/4][window])
// and a remainder array ([window] of 1 or 2 values) after them, so that every
// LDS read is aligned, no padding is read, and every array has a 16-byte
// stride (window slots distinct mod 8 fall on distinct banks): 6 values are
// one 16-byte and one 8-byte read, 9 values two 16-byte reads and one 4-byte
// read.
template <typename T, int N>
struct Pk {
  static constexpr int Q = N / 4, R = N % 4;
  static_assert(R != 3, "a remainder of three values is not packed");
  static constexpr size_t bytes = Q * sizeof(vec4<T>) + R * sizeof(T);  // per particle
  __device__ static __forceinline__ void store(unsigned char* lds, uint32_t window, uint32_t l,
                                               const T* v) {
    vec4<T>* q = reinterpret_cast<vec4<T>*>(lds) + l;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      vec4<T> pv;
      pv.x = v[4 * j];
      pv.y = v[4 * j + 1];
      pv.z = v[4 * j + 2];
      pv.w = v[4 * j + 3];
      q[(size_t)j * window] = pv;
    }
    unsigned char* rb = lds + (size_t)window * Q * sizeof(vec4<T>);
    if constexpr (R == 2) {
      using v2 = T __attribute__((ext_vector_type(2)));
      v2 r;
      r.x = v[4 * Q];
      r.y = v[4 * Q + 1];
      reinterpret_cast<v2*>(rb)[l] = r;
    } else if constexpr (R == 1) {
      reinterpret_cast<T*>(rb)[l] = v[4 * Q];
    }
  }
  __device__ static __forceinline__ void load(const unsigned char* lds, uint32_t window,
                                              uint32_t l, T* v) {
    const vec4<T>* q = reinterpret_cast<const vec4<T>*>(lds) + l;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const vec4<T> pv = q[(size_t)j * window];
      v[4 * j] = pv.x;
      v[4 * j + 1] = pv.y;
      v[4 * j + 2] = pv.z;
      v[4 * j + 3] = pv.w;
    }
    const unsigned char* rb = lds + (size_t)window * Q * sizeof(vec4<T>);
    if constexpr (R == 2) {
      using v2 = T __attribute__((ext_vector_type(2)));
      const v2 r = reinterpret_cast<const v2*>(rb)[l];
      v[4 * Q] = r.x;
      v[4 * Q + 1] = r.y;
    } else if constexpr (R == 1) {
      v[4 * Q] = reinterpret_cast<const T*>(rb)[l];
    }
  }
};

// own particle t of a tile: its sorted index and its window position
// the own particle of thread slot t of a tile, its window position la and
// the blocks of four entries of its neighbour list
__device__ __forceinline__ int64_t tile_own(const uint32_t* __restrict__ tslot, int tmax,
                                            int64_t tile, const TileDesc& td, uint32_t t,
                                            uint32_t& la, uint32_t& nb4) {
  const uint32_t info = tslot[tile * tmax + t];
  const uint32_t s = info & 0xFFFFu;
  nb4 = info >> 16;
  if (s < td.count0) {
    la = td.own_base + s;
    return (int64_t)td.p0 + s;
  }
  la = td.own_base1 + (s - td.count0);
  return (int64_t)td.p1 + (s - td.count0);
}

__device__ __forceinline__ int64_t xcd_tile(int64_t n_tiles) {
  const int64_t per = (n_tiles + 7) / 8;
  return (int64_t)(blockIdx.x & 7u) * per + (blockIdx.x >> 3);
}

// value of the lane that the DPP control CTRL selects (within a row of 16)
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF,
                                                            0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// sum over the LPP consecutive lanes of one particle (every lane gets it), by
// lane swaps within the row: quad_perm [1,0,3,2], quad_perm [2,3,0,1], then
// the mirror within each half row (lane i <-> 7 - i), which pairs the two
// quads of a group of eight.  All lanes of a group are active together.
template <int LPP, typename T>
__device__ __forceinline__ T lane_sum(T x) {
  static_assert(LPP == 1 || LPP == 2 || LPP == 4 || LPP == 8, "lanes per particle");
  if constexpr (LPP >= 2) x += dpp_mov<0xB1>(x);
  if constexpr (LPP >= 4) x += dpp_mov<0x4E>(x);
  if constexpr (LPP >= 8) x += dpp_mov<0x141>(x);
  return x;
}

// window index -> global particle index: the window is the concatenation of
// the tile's runs (uniform data, kept in scalar registers)
struct WinMap {
  uint32_t start[9];
  uint32_t lend[9];  // exclusive end of each run in window numbering
  uint32_t nruns;
  __device__ __forceinline__ int64_t operator()(uint32_t l) const {
    uint32_t b = 0;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      if (r < (int)nruns && l >= b && l < lend[r]) return (int64_t)start[r] + (l - b);
      b = r < (int)nruns ? lend[r] : b;
    }
    return (int64_t)start[0];
  }
};

__device__ __forceinline__ WinMap win_map(const TileDesc& td) {
  WinMap m;
  m.nruns = td.nruns;
  uint32_t acc = 0;
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    m.start[r] = td.run_start[r];
    acc += r < (int)td.nruns ? td.run_count[r] : 0u;
    m.lend[r] = acc;
  }
  return m;
}

// Blocked-ELL walk: lane h of a particle takes the blocks of four neighbour
// indices c = h, h + LPP, ...; three registers rotate so that the loads of
// the next three blocks are in flight while one is applied.  Every load is
// unconditional (clamped to the particle's last block, which is always in its
// row), so the wait before a block's use is an exact count of the loads
// issued after it.
template <int LPP, typename F>
__device__ __forceinline__ void ell_walk(const uint16_t* ell, uint32_t ell_off, int tmax, int t,
                                         int h, uint32_t blocks, F&& f) {
  const uint2* e = reinterpret_cast<const uint2*>(ell + ell_off) + t;
  const int nb4 = (int)blocks;
  if (h >= nb4) return;
  const int last = nb4 - 1;
  auto ld = [&](int c) -> uint2 { return e[(int64_t)(c < last ? c : last) * tmax]; };
  auto apply = [&](uint2 b) {
    f(b.x & 0xFFFFu);
    f(b.x >> 16);
    f(b.y & 0xFFFFu);
    f(b.y >> 16);
  };
  // the blocks this lane takes, in full rounds of three and a remainder; the
  // remainder reads the registers the last round loaded, so the loads stay
  // at the top of each round
  const int cnt = (nb4 - h + LPP - 1) / LPP;
  const int full = cnt / 3, rem = cnt - 3 * full;
  uint2 b0 = ld(h), b1 = ld(h + LPP), b2 = ld(h + 2 * LPP);
  int c = h;
  for (int i = 0; i < full; ++i, c += 3 * LPP) {
    apply(b0);
    b0 = ld(c + 3 * LPP);
    apply(b1);
    b1 = ld(c + 4 * LPP);
    apply(b2);
    b2 = ld(c + 5 * LPP);
  }
  if (rem >= 1) apply(b0);
  if (rem >= 2) apply(b1);
}

template <typename T>
struct PairQ;
template <>
struct alignas(8) PairQ<float> {
  uint32_t w;
  float q;
};
template <>
struct alignas(16) PairQ<double> {
  uint32_t w, pad;
  double q;
};

static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <typename T>
static MatP<T> matp(const sph_material* m) {
  MatP<T> r;
  r.model = m->model;
  double mu = m->E / (2.0 * (1.0 + m->nu));
  double K = m->E / (3.0 * (1.0 - 2.0 * m->nu));
  r.mu = (T)mu;
  r.K = (T)K;
  r.lam = (T)(K - 2.0 * mu / 3.0);
  r.s0 = (T)m->sigma0;
  r.sinf = (T)m->sigma_inf;
  r.delta = (T)m->delta;
  r.H = (T)m->H;
  r.newton_tol = sizeof(T) == 8 ? (T)1e-13 : (T)2e-6;
  r.dmu_dE = (T)(1.0 / (2.0 * (1.0 + m->nu)));
  r.dK_dE = (T)(1.0 / (3.0 * (1.0 - 2.0 * m->nu)));
  return r;
}

template <typename K>
static int lds_attr(K kernel, size_t bytes) {
  if (bytes > 64 * 1024) {
    SPH_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  }
  return SPH_OK;
}

}  // namespace sph
