// sph_step.hip -- inner-step and slow-step kernels of the TL-SPH path on gfx950.
//
// Layout: structure-of-arrays [component][n] in cell-sorted order, so that a
// wavefront of 64 consecutive particles reads 64 consecutive words of every
// component, and the neighbours it gathers sit in the same few cells.
// Reference geometry (X) and displacement (u) are FP64; pair geometry and
// displacement differences are formed in FP64 and then rounded to the working
// type T (float or double), so the FP32 path loses nothing to cancellation.
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
};

template <typename T>
static Geo<T> geo(const sph_nbr* nb);
template <>
Geo<double> geo<double>(const sph_nbr* nb) {
  return Geo<double>{nb->X, nb->V, nb->B0, nb->nbr_off, nb->nbr_idx, nb->n, nb->inv_h, nb->c5};
}
template <>
Geo<float> geo<float>(const sph_nbr* nb) {
  return Geo<float>{nb->X, nb->Vf, nb->B0f, nb->nbr_off, nb->nbr_idx, nb->n, (float)nb->inv_h,
                    (float)nb->c5};
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
};

template <typename T>
__device__ __forceinline__ T hardening(const MatP<T>& m, T a) {
  return m.s0 + (m.sinf - m.s0) * (T(1) - exp(-m.delta * a)) + m.H * a;
}
template <typename T>
__device__ __forceinline__ T hardening_slope(const MatP<T>& m, T a) {
  return (m.sinf - m.s0) * m.delta * exp(-m.delta * a) + m.H;
}

// First Piola-Kirchhoff stress of one particle; returns SPH_STATUS_NEWTON on a
// failed return mapping.  App. A.2-A.4 and B.2 of the paper; LE is the
// small-strain reading.  pl: Cbar_p^-1 (xx,yy,zz,xy,yz,xz) and alpha.
template <typename T>
__device__ int constitutive(const MatP<T>& m, const T* F, T* pl, T p, T* P) {
  T J = det3(F);
  T Fi[9];
  inv3(F, J, Fi);
  int st = 0;
  T tau[9];
  if (m.model == SPH_MODEL_LE) {
    T e0 = F[0] - T(1), e4 = F[4] - T(1), e8 = F[8] - T(1);
    T tr = e0 + e4 + e8;
    T tm = T(2) * m.mu;
    P[0] = tm * e0 + m.lam * tr;
    P[4] = tm * e4 + m.lam * tr;
    P[8] = tm * e8 + m.lam * tr;
    P[1] = P[3] = m.mu * (F[1] + F[3]);
    P[2] = P[6] = m.mu * (F[2] + F[6]);
    P[5] = P[7] = m.mu * (F[5] + F[7]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) P[i * 3 + j] -= J * p * Fi[j * 3 + i];
    return 0;
  }
  T cb = cbrt(J);
  T vol = T(0.5) * m.K * (J * J - T(1));
  if (m.model == SPH_MODEL_NH) {
    T b[9];
    mul3_bt(F, F, b);
    T s23 = T(1) / (cb * cb);
    T trb = (b[0] + b[4] + b[8]) * s23 * (T(1) / T(3));
#pragma unroll
    for (int i = 0; i < 9; ++i) tau[i] = m.mu * b[i] * s23;
    tau[0] += vol - m.mu * trb;
    tau[4] += vol - m.mu * trb;
    tau[8] += vol - m.mu * trb;
  } else {
    // Algorithm 1
    T s13 = T(1) / cb;
    T Fb[9], Xb[9], tmp[9], bp[9], s[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Fb[i] = s13 * F[i];
    Xb[0] = pl[0]; Xb[4] = pl[1]; Xb[8] = pl[2];
    Xb[1] = Xb[3] = pl[3];
    Xb[5] = Xb[7] = pl[4];
    Xb[2] = Xb[6] = pl[5];
    T alpha = pl[6];
    mul3(Fb, Xb, tmp);
    mul3_bt(tmp, Fb, bp);
    T trb3 = (bp[0] + bp[4] + bp[8]) * (T(1) / T(3));
    T n2 = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      s[i] = m.mu * bp[i];
      if (i == 0 || i == 4 || i == 8) s[i] -= m.mu * trb3;
      n2 += s[i] * s[i];
    }
    T sn = sqrt(n2);
    const T r23 = T(0.816496580927726);  // sqrt(2/3)
    T f = sn - r23 * hardening(m, alpha);
    if (f > T(0)) {
      T mub = m.mu * trb3;
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
    // internal variable: bbar_e = s/mu + tr(bbar_pre)/3 I; Cbar_p^-1 = Fbar^-1 bbar_e Fbar^-T
    T be[9], Fbi[9], t2[9], Xn[9];
    T imu = T(1) / m.mu;
#pragma unroll
    for (int i = 0; i < 9; ++i) be[i] = s[i] * imu;
    be[0] += trb3;
    be[4] += trb3;
    be[8] += trb3;
    inv3(Fb, det3(Fb), Fbi);
    mul3(Fbi, be, t2);
    mul3_bt(t2, Fbi, Xn);
    pl[0] = Xn[0]; pl[1] = Xn[4]; pl[2] = Xn[8];
    pl[3] = Xn[1]; pl[4] = Xn[5]; pl[5] = Xn[2];
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
// stress stage: F from u (corrected gradient), constitutive, PB = P B0
template <typename T, int D>
__global__ __launch_bounds__(256) void k_stress(Geo<T> g, MatP<T> m, const double* __restrict__ u,
                                                T* __restrict__ PB, T* __restrict__ plastic,
                                                const T* __restrict__ p, Ctrl* ctrl, bool gated) {
  if (gated && ctrl->done) return;
  const int64_t n = g.n;
  int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  double xa[D], ua[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    xa[k] = g.X[k * n + a];
    ua[k] = u[k * n + a];
  }
  T G[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) G[i][k] = T(0);
  const int64_t j1 = g.off[a + 1];
  for (int64_t j = g.off[a]; j < j1; ++j) {
    const uint32_t b = g.idx[j];
    T d[D], du[D];
    T r2 = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      d[k] = (T)(xa[k] - g.X[k * n + b]);
      du[k] = (T)(u[k * n + b] - ua[k]);
      r2 += d[k] * d[k];
    }
    const T w = dw_over_r(r2, g.inv_h, g.c5) * g.V[b];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const T wd = w * du[i];
#pragma unroll
      for (int k = 0; k < D; ++k) G[i][k] += wd * d[k];
    }
  }
  T F[9] = {T(1), T(0), T(0), T(0), T(1), T(0), T(0), T(0), T(1)};
  T B[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) B[i][k] = g.B0[(i * D + k) * n + a];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < D; ++l) acc += G[i][l] * B[l][k];
      F[i * 3 + k] += acc;
    }
  T pl[7];
  if (m.model == SPH_MODEL_J2) {
#pragma unroll
    for (int i = 0; i < 7; ++i) pl[i] = plastic[i * n + a];
  }
  T P[9];
  int st = constitutive(m, F, pl, p ? p[a] : T(0), P);
  if (st) atomicOr(&ctrl->status, st);
  if (m.model == SPH_MODEL_J2) {
#pragma unroll
    for (int i = 0; i < 7; ++i) plastic[i * n + a] = pl[i];
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < D; ++l) acc += P[i * 3 + l] * B[l][k];
      PB[(i * D + k) * n + a] = acc;
    }
}

// momentum: a = (1/rho0) sum_b V_b (PB_a + PB_b) grad_a W_ab; kick v += dt a
template <typename T, int D>
__global__ __launch_bounds__(256) void k_momentum(Geo<T> g, const T* __restrict__ PB,
                                                  T* __restrict__ v, T* __restrict__ acc_out,
                                                  const uint8_t* __restrict__ flags, T inv_rho0,
                                                  T dt, Ctrl* ctrl, bool gated) {
  if (gated && ctrl->done) return;
  const int64_t n = g.n;
  int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  double xa[D];
  T Pa[D * D];
#pragma unroll
  for (int k = 0; k < D; ++k) xa[k] = g.X[k * n + a];
#pragma unroll
  for (int k = 0; k < D * D; ++k) Pa[k] = PB[k * n + a];
  T f[D];
#pragma unroll
  for (int k = 0; k < D; ++k) f[k] = T(0);
  const int64_t j1 = g.off[a + 1];
  for (int64_t j = g.off[a]; j < j1; ++j) {
    const uint32_t b = g.idx[j];
    T d[D];
    T r2 = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      d[k] = (T)(xa[k] - g.X[k * n + b]);
      r2 += d[k] * d[k];
    }
    const T w = dw_over_r(r2, g.inv_h, g.c5) * g.V[b];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      T s = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) s += (Pa[i * D + k] + PB[(i * D + k) * n + b]) * d[k];
      f[i] += w * s;
    }
  }
  const bool fixed = flags && (flags[a] & SPH_FLAG_FIXED);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T ai = f[i] * inv_rho0;
    if (acc_out) acc_out[i * n + a] = ai;
    if (!fixed) v[i * n + a] += dt * ai;
  }
}

// damping: one wavefront per anchor of one colour; levels in order, the pairs
// of a level in parallel (they share no particle)
template <typename T, int D>
__global__ __launch_bounds__(64) void k_damp(Geo<T> g, const uint32_t* __restrict__ sa,
                                             const uint32_t* __restrict__ sb,
                                             const uint32_t* __restrict__ slev,
                                             const int64_t* __restrict__ aoff, int64_t a_begin,
                                             T* v, const uint8_t* __restrict__ flags, T rho0,
                                             T beta0, Ctrl* ctrl, bool gated) {
  if (gated && ctrl->done) return;
  const int64_t n = g.n;
  const int64_t ai = a_begin + blockIdx.x;
  const int64_t lo = aoff[ai], hi = aoff[ai + 1];
  const int lane = threadIdx.x;
  int64_t pos = lo;
  while (pos < hi) {
    const uint32_t L = slev[pos];
    const int64_t i = pos + lane;
    const bool act = (i < hi) && (slev[i] == L);
    if (act) {
      const uint32_t a = sa[i], b = sb[i];
      const bool fa = flags && (flags[a] & SPH_FLAG_FIXED);
      const bool fb = flags && (flags[b] & SPH_FLAG_FIXED);
      if (!(fa && fb)) {
        T r2 = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) {
          T d = (T)(g.X[k * n + a] - g.X[k * n + b]);
          r2 += d * d;
        }
        const T Va = g.V[a], Vb = g.V[b];
        const T beta = beta0 * Va * Vb * dw_over_r(r2, g.inv_h, g.c5);
        const T ma = rho0 * Va, mb = rho0 * Vb;
        if (!fa && !fb) {
          const T den = T(1) / (ma * mb - beta * (ma + mb));
#pragma unroll
          for (int k = 0; k < D; ++k) {
            T va = v[k * n + a], vb = v[k * n + b];
            T delta = beta * (va - vb) * den;
            v[k * n + a] = va + mb * delta;
            v[k * n + b] = vb - ma * delta;
          }
        } else if (fb) {
          const T den = T(1) / (ma - beta);
#pragma unroll
          for (int k = 0; k < D; ++k) {
            T va = v[k * n + a], vb = v[k * n + b];
            v[k * n + a] = va + beta * (va - vb) * den;
          }
        } else {
          const T den = T(1) / (mb - beta);
#pragma unroll
          for (int k = 0; k < D; ++k) {
            T va = v[k * n + a], vb = v[k * n + b];
            v[k * n + b] = vb + beta * (vb - va) * den;
          }
        }
      }
    }
    pos += __popcll(__ballot(act));
    __syncthreads();
  }
}

// drift + kinetic energy with a fixed-order two-stage reduction; the last
// block to finish reduces the partials, records E_k and updates the stop state
template <typename T, int D>
__global__ __launch_bounds__(kKeThreads) void k_drift_ke(
    int64_t n, double* __restrict__ u, const T* __restrict__ v, const uint8_t* __restrict__ flags,
    const double* __restrict__ V, double rho0, double dt, Ctrl* ctrl, double* partial,
    double* ke_out, bool gated) {
  if (gated && ctrl->done) return;
  __shared__ double red[kKeThreads];
  __shared__ bool last;
  double acc = 0.0;
  for (int64_t a = blockIdx.x * (int64_t)kKeThreads + threadIdx.x; a < n;
       a += (int64_t)gridDim.x * kKeThreads) {
    const bool fixed = flags && (flags[a] & SPH_FLAG_FIXED);
    double v2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double vk = (double)v[k * n + a];
      if (!fixed) u[k * n + a] += dt * vk;
      v2 += vk * vk;
    }
    acc += 0.5 * rho0 * V[a] * v2;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kKeThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = red[0];
    __threadfence();
    unsigned t = atomicAdd(&ctrl->ticket, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double s = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += kKeThreads)
    s += __builtin_nontemporal_load(&partial[b]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kKeThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double ke = red[0];
    ctrl->ticket = 0u;
    if (ke_out) *ke_out = ke;
    if (gated) {
      ctrl->ke = ke;
      const int64_t k = ctrl->k + 1;
      ctrl->k = k;
      if (!isfinite(ke)) {
        ctrl->status |= SPH_STATUS_NONFINITE;
        ctrl->done = 1;
      } else if (ke <= ctrl->ke_tol) {
        ctrl->stopped_by_ke = 1;
        ctrl->done = 1;
      } else if (k >= ctrl->k_limit) {
        ctrl->done = 1;
      }
    } else if (!isfinite(ke)) {
      ctrl->status |= SPH_STATUS_NONFINITE;
    }
  }
}

__global__ void k_reset_ctrl(Ctrl* c, int64_t k_limit, double ke_tol) {
  c->done = 0;
  c->k = 0;
  c->k_limit = k_limit;
  c->ke = 0.0;
  c->ke_tol = ke_tol;
  c->ticket = 0u;
  c->stopped_by_ke = 0;
}

template <typename T, int D>
__global__ void k_load(int64_t n, double* u, const T* vgrip, const uint8_t* flags, double dt) {
  int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n || !(flags[a] & SPH_FLAG_GRIP)) return;
#pragma unroll
  for (int k = 0; k < D; ++k) u[k * n + a] += dt * (double)vgrip[k * n + a];
}

// diffusion: flux q = -D B0 sum_b V_b (c_b - c_a) grad W
template <typename T, int D>
__global__ __launch_bounds__(256) void k_diff_grad(Geo<T> g, const T* __restrict__ c,
                                                   T* __restrict__ q, T Dc) {
  const int64_t n = g.n;
  int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  double xa[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xa[k] = g.X[k * n + a];
  const T ca = c[a];
  T s[D];
#pragma unroll
  for (int k = 0; k < D; ++k) s[k] = T(0);
  for (int64_t j = g.off[a]; j < g.off[a + 1]; ++j) {
    const uint32_t b = g.idx[j];
    T d[D];
    T r2 = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      d[k] = (T)(xa[k] - g.X[k * n + b]);
      r2 += d[k] * d[k];
    }
    const T w = dw_over_r(r2, g.inv_h, g.c5) * g.V[b] * (c[b] - ca);
#pragma unroll
    for (int k = 0; k < D; ++k) s[k] += w * d[k];
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) acc += g.B0[(i * D + k) * n + a] * s[k];
    q[i * n + a] = -Dc * acc;
  }
}

// c += dt (-sum_b V_b (B0_a q_a + B0_b q_b) . grad W); Dirichlet; p = C (c - c0)
template <typename T, int D>
__global__ __launch_bounds__(256) void k_diff_div(Geo<T> g, T* __restrict__ c,
                                                  const T* __restrict__ q, T* __restrict__ p,
                                                  const uint8_t* __restrict__ flags, T dt,
                                                  T c_bc, T Cs, T c0) {
  const int64_t n = g.n;
  int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  double xa[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xa[k] = g.X[k * n + a];
  T ga[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) acc += g.B0[(i * D + k) * n + a] * q[k * n + a];
    ga[i] = acc;
  }
  T div = T(0);
  for (int64_t j = g.off[a]; j < g.off[a + 1]; ++j) {
    const uint32_t b = g.idx[j];
    T d[D];
    T r2 = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      d[k] = (T)(xa[k] - g.X[k * n + b]);
      r2 += d[k] * d[k];
    }
    const T w = dw_over_r(r2, g.inv_h, g.c5) * g.V[b];
    T s = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      T gb = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) gb += g.B0[(i * D + k) * n + b] * q[k * n + b];
      s += (ga[i] + gb) * d[i];
    }
    div += w * s;
  }
  T cn = c[a] - dt * div;
  if (flags && (flags[a] & SPH_FLAG_CDIR)) cn = c_bc;
  c[a] = cn;
  if (p) p[a] = Cs * (cn - c0);
}

// ---------------------------------------------------------------------------
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
  return r;
}

int check_state(const sph_nbr* nb, const sph_state* st, bool need_v) {
  if (!nb || !st) {
    set_error("null handle or state");
    return SPH_E_ARG;
  }
  if (st->prec != SPH_F32 && st->prec != SPH_F64) {
    set_error("prec must be SPH_F32 or SPH_F64");
    return SPH_E_UNSUPPORTED;
  }
  if (!st->u || (need_v && !st->v)) {
    set_error("state arrays u/v missing");
    return SPH_E_ARG;
  }
  return SPH_OK;
}

template <typename T, int D>
static int solid_stage_t(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
                         hipStream_t s, bool gated) {
  Geo<T> g = geo<T>(nb);
  MatP<T> mp = matp<T>(m);
  k_stress<T, D><<<nblk(nb->n, 256), 256, 0, s>>>(g, mp, st->u, (T*)st->PB, (T*)st->plastic,
                                                  (const T*)st->p, nb->ctrl, gated);
  SPH_LAUNCH_CHECK();
  k_momentum<T, D><<<nblk(nb->n, 256), 256, 0, s>>>(g, (const T*)st->PB, (T*)st->v, (T*)st->acc,
                                                    st->flags, (T)(1.0 / m->rho0), (T)dt,
                                                    nb->ctrl, gated);
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

int solid_stage(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
                hipStream_t s, bool gated) {
  if (m->model == SPH_MODEL_J2 && !st->plastic) {
    set_error("J2 needs the plastic state array");
    return SPH_E_ARG;
  }
  if (!st->PB) {
    set_error("PB scratch missing");
    return SPH_E_ARG;
  }
  if (st->prec == SPH_F64)
    return nb->dim == 2 ? solid_stage_t<double, 2>(nb, m, st, dt, s, gated)
                        : solid_stage_t<double, 3>(nb, m, st, dt, s, gated);
  return nb->dim == 2 ? solid_stage_t<float, 2>(nb, m, st, dt, s, gated)
                      : solid_stage_t<float, 3>(nb, m, st, dt, s, gated);
}

template <typename T, int D>
static int damping_t(const sph_nbr* nb, const sph_material* m, const sph_state* st, double eta,
                     double dt, hipStream_t s, bool gated) {
  Geo<T> g = geo<T>(nb);
  const int ncol = 1 << D;
  for (int col = 0; col < ncol; ++col) {
    int64_t a0 = nb->color_off[col], a1 = nb->color_off[col + 1];
    if (a1 <= a0) continue;
    k_damp<T, D><<<(unsigned)(a1 - a0), 64, 0, s>>>(g, nb->sa, nb->sb, nb->slev, nb->aoff, a0,
                                                     (T*)st->v, st->flags, (T)m->rho0,
                                                     (T)(2.0 * eta * dt), nb->ctrl, gated);
    SPH_LAUNCH_CHECK();
  }
  return SPH_OK;
}

int damping_sweep(const sph_nbr* nb, const sph_material* m, const sph_state* st, double eta,
                  double dt, hipStream_t s, bool gated) {
  if (st->prec == SPH_F64)
    return nb->dim == 2 ? damping_t<double, 2>(nb, m, st, eta, dt, s, gated)
                        : damping_t<double, 3>(nb, m, st, eta, dt, s, gated);
  return nb->dim == 2 ? damping_t<float, 2>(nb, m, st, eta, dt, s, gated)
                      : damping_t<float, 3>(nb, m, st, eta, dt, s, gated);
}

template <typename T, int D>
static int drift_t(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
                   double* ke_out, hipStream_t s, bool gated) {
  int64_t nb_ = std::min<int64_t>(kKeMaxBlocks, std::max<int64_t>(1, (nb->n + kKeThreads - 1) / kKeThreads));
  k_drift_ke<T, D><<<(unsigned)nb_, kKeThreads, 0, s>>>(nb->n, st->u, (const T*)st->v, st->flags,
                                                       nb->V, m->rho0, dt, nb->ctrl,
                                                       nb->ke_partial, ke_out, gated);
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

int drift_ke(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
             double* ke_out, hipStream_t s, bool gated) {
  if (st->prec == SPH_F64)
    return nb->dim == 2 ? drift_t<double, 2>(nb, m, st, dt, ke_out, s, gated)
                        : drift_t<double, 3>(nb, m, st, dt, ke_out, s, gated);
  return nb->dim == 2 ? drift_t<float, 2>(nb, m, st, dt, ke_out, s, gated)
                      : drift_t<float, 3>(nb, m, st, dt, ke_out, s, gated);
}

int reset_ctrl(const sph_nbr* nb, int64_t k_limit, double ke_tol, hipStream_t s) {
  k_reset_ctrl<<<1, 1, 0, s>>>(nb->ctrl, k_limit, ke_tol);
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

int load_step(const sph_nbr* nb, const sph_state* st, double dt_l, hipStream_t s) {
  if (!st->vgrip || !st->flags) return SPH_OK;
  if (st->prec == SPH_F64) {
    if (nb->dim == 2) k_load<double, 2><<<nblk(nb->n, 256), 256, 0, s>>>(nb->n, st->u, (const double*)st->vgrip, st->flags, dt_l);
    else k_load<double, 3><<<nblk(nb->n, 256), 256, 0, s>>>(nb->n, st->u, (const double*)st->vgrip, st->flags, dt_l);
  } else {
    if (nb->dim == 2) k_load<float, 2><<<nblk(nb->n, 256), 256, 0, s>>>(nb->n, st->u, (const float*)st->vgrip, st->flags, dt_l);
    else k_load<float, 3><<<nblk(nb->n, 256), 256, 0, s>>>(nb->n, st->u, (const float*)st->vgrip, st->flags, dt_l);
  }
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

template <typename T, int D>
static int diffusion_t(const sph_nbr* nb, const sph_material* m, const sph_state* st, double Dc,
                       double dt, double c_bc, hipStream_t s) {
  Geo<T> g = geo<T>(nb);
  k_diff_grad<T, D><<<nblk(nb->n, 256), 256, 0, s>>>(g, (const T*)st->c, (T*)st->q, (T)Dc);
  SPH_LAUNCH_CHECK();
  k_diff_div<T, D><<<nblk(nb->n, 256), 256, 0, s>>>(g, (T*)st->c, (const T*)st->q, (T*)st->p,
                                                    st->flags, (T)dt, (T)c_bc, (T)m->C_swell,
                                                    (T)m->c0);
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

int diffusion_step(const sph_nbr* nb, const sph_material* m, const sph_state* st, double Dc,
                   double dt, double c_bc, hipStream_t s) {
  if (!st->c || !st->q) {
    set_error("diffusion needs c and q");
    return SPH_E_ARG;
  }
  if (st->prec == SPH_F64)
    return nb->dim == 2 ? diffusion_t<double, 2>(nb, m, st, Dc, dt, c_bc, s)
                        : diffusion_t<double, 3>(nb, m, st, Dc, dt, c_bc, s);
  return nb->dim == 2 ? diffusion_t<float, 2>(nb, m, st, Dc, dt, c_bc, s)
                      : diffusion_t<float, 3>(nb, m, st, Dc, dt, c_bc, s);
}

}  // namespace sph
