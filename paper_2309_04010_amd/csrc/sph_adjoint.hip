// sph_adjoint.hip -- reverse mode of the TL-SPH multi-time-step path on gfx950.
//
// Every map of the inner step is either linear in the state (displacement
// gradient sum, momentum sum, kick, damping sweep, drift) or local to one
// particle (the constitutive update), so its transpose is written directly:
//   drift^T      w += dt u_bar                      (free particles)
//   sweep^T      pair maps transposed, colours and levels in reverse
//   kick^T       a_bar = dt w                       (free particles)
//   momentum^T   PB_bar_a = (1/rho0) sum_b (V_b a_bar_a - V_a a_bar_b) (x) grad_a W_ab
//   stress^T     P_bar = PB_bar B0^T, exact derivative of P(H, state, p; theta)
//   grad^T       G_bar = H_bar B0^T,
//                u_bar_a -= sum_b (V_a G_bar_b + V_b G_bar_a) grad_a W_ab
// The stress transpose and the momentum transpose share one pass over the
// neighbours (both gather in the same LDS window), the displacement-gradient
// transpose is a second pass shaped like the momentum kernel.  Parameter
// gradients are summed per workgroup in FP64 into fixed slots and reduced in
// a fixed order, so the reverse pass is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "sph_device.h"

namespace sph {

constexpr int kNTheta = 5;  // E, sigma0, sigma_inf, delta, H (the stress-stage parameters)

template <typename T>
__device__ __forceinline__ T dot9(const T* A, const T* B) {
  T s = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) s += A[i] * B[i];
  return s;
}
// C = A^T B
template <typename T>
__device__ __forceinline__ void mul3_tn(const T* A, const T* B, T* C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[i * 3 + j] = A[i] * B[j] + A[3 + i] * B[3 + j] + A[6 + i] * B[6 + j];
}
// D += (S + S^T) A
template <typename T>
__device__ __forceinline__ void add_symx(const T* S, const T* A, T* D) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T s = T(0);
#pragma unroll
      for (int k = 0; k < 3; ++k) s += (S[i * 3 + k] + S[k * 3 + i]) * A[k * 3 + j];
      D[i * 3 + j] += s;
    }
}

// Reverse of constitutive(): given P_bar (adjoint of P) and plb (adjoint of
// the updated J2 state, 7 entries; replaced by the adjoint of the state
// before the update), returns H_bar, p_bar and th = adjoints of (E, sigma0,
// sigma_inf, delta, H).  pl is the state BEFORE the update.  The forward
// quantities are recomputed as constitutive() computes them; the return
// mapping's increment dgamma is differentiated through its scalar residual
//   f(dg) = |s_pre| - sqrt(2/3) k(alpha + sqrt(2/3) dg) - 2 mubar dg = 0
// (implicit-function theorem: d dg = -(df/dx dx) / (df/d dg)).
template <typename T, int MODEL = -1>
__device__ int constitutive_vjp(const MatP<T>& m, const T* H, const T* pl, T p, const T* Pb,
                                T* plb, T* Hbar, T& pbar, T* th) {
  const T trH = H[0] + H[4] + H[8];
  const T trH2 =
      H[0] * H[0] + H[4] * H[4] + H[8] * H[8] + T(2) * (H[1] * H[3] + H[2] * H[6] + H[5] * H[7]);
  const T jm1 = trH + T(0.5) * (trH * trH - trH2) + det3(H);
  const T J = T(1) + jm1;
  T F[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) F[i] = H[i];
  F[0] += T(1);
  F[4] += T(1);
  F[8] += T(1);
  T Fi[9];
  inv3(F, J, Fi);
#pragma unroll
  for (int i = 0; i < kNTheta; ++i) th[i] = T(0);
  T mub = T(0), Kb = T(0), Jb = T(0);
  int st = 0;
  if (model_is<MODEL>(m, SPH_MODEL_LE)) {
    // P = 2 mu sym(H) + lam tr(H) I - p J F^-T, lam = K - 2 mu / 3
    const T trPb = Pb[0] + Pb[4] + Pb[8];
    T sHP = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        Hbar[i * 3 + j] = m.mu * (Pb[i * 3 + j] + Pb[j * 3 + i]);
        sHP += Pb[i * 3 + j] * T(0.5) * (H[i * 3 + j] + H[j * 3 + i]);
      }
    Hbar[0] += m.lam * trPb;
    Hbar[4] += m.lam * trPb;
    Hbar[8] += m.lam * trPb;
    mub = T(2) * sHP - T(2.0 / 3.0) * trH * trPb;
    Kb = trH * trPb;
    // d(J F^-T)[dF] = J tr(F^-1 dF) F^-T - J F^-T dF^T F^-T
    T cd = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) cd += Pb[i * 3 + j] * Fi[j * 3 + i];
    pbar = -J * cd;
    T t[9], N[9];
    mul3(Fi, Pb, t);
    mul3(t, Fi, N);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Hbar[i * 3 + j] -= p * J * (cd * Fi[j * 3 + i] - N[j * 3 + i]);
    th[0] = mub * m.dmu_dE + Kb * m.dK_dE;
    return 0;
  }
  const T vol = T(0.5) * m.K * jm1 * (T(2) + jm1);
  T Fbar[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Fbar[i] = T(0);
  // ---- forward values -------------------------------------------------------
  T s[9];  // deviatoric Kirchhoff stress
  // NH
  T dB[9], s23 = T(0);
  // J2
  T c = T(0), Fb[9], Y[9], FFm[9], E[9], spre[9], Dm[9], G[9];
  T trE3 = T(0), sn = T(0), mubr = T(0), dg = T(0), fac = T(1), alpha = T(0);
  bool plastic = false;
  const T r23 = T(0.816496580927726);  // sqrt(2/3)
  if (model_is<MODEL>(m, SPH_MODEL_NH)) {
    T Bm[9];
    sym_sum(H, Bm);
    const T cb = cbrt(J);
    s23 = T(1) / (cb * cb);
    const T tr3 = (Bm[0] + Bm[4] + Bm[8]) * (T(1) / T(3));
#pragma unroll
    for (int i = 0; i < 9; ++i) dB[i] = Bm[i];
    dB[0] -= tr3;
    dB[4] -= tr3;
    dB[8] -= tr3;
#pragma unroll
    for (int i = 0; i < 9; ++i) s[i] = m.mu * s23 * dB[i];
  } else {
    c = T(1) / cbrt(J);
    const T cm1 = expm1(log1p(jm1) * T(-1.0 / 3.0));
    T Hb[9];
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
    Y[0] = pl[0];
    Y[4] = pl[1];
    Y[8] = pl[2];
    Y[1] = Y[3] = pl[3];
    Y[5] = Y[7] = pl[4];
    Y[2] = Y[6] = pl[5];
    alpha = pl[6];
    sym_sum(Hb, FFm);
    T tmp[9];
    mul3(Fb, Y, tmp);
    mul3_bt(tmp, Fb, E);
#pragma unroll
    for (int i = 0; i < 9; ++i) E[i] += FFm[i];
    trE3 = (E[0] + E[4] + E[8]) * (T(1) / T(3));
    T n2 = T(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      spre[i] = m.mu * E[i];
      if (i == 0 || i == 4 || i == 8) spre[i] -= m.mu * trE3;
      n2 += spre[i] * spre[i];
    }
    sn = sqrt(n2);
    const T f = sn - r23 * hardening(m, alpha);
    if (f > T(0)) {
      plastic = true;
      mubr = m.mu * (T(1) + trE3);
      const T tol = m.newton_tol * (sn > T(1) ? sn : T(1));
      bool ok = false;
      for (int it = 0; it < 50; ++it) {
        const T a1 = alpha + r23 * dg;
        const T fh = sn - r23 * hardening(m, a1) - T(2) * mubr * dg;
        if (fabs(fh) <= tol) {
          ok = true;
          break;
        }
        const T dfh = -(T(2) / T(3)) * hardening_slope(m, a1) - T(2) * mubr;
        dg -= fh / dfh;
      }
      if (!ok) st = SPH_STATUS_NEWTON;
      fac = T(1) - T(2) * mubr * dg / sn;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) s[i] = fac * spre[i];
    const T imu = T(1) / m.mu;
#pragma unroll
    for (int i = 0; i < 9; ++i) Dm[i] = s[i] * imu - FFm[i];
    Dm[0] += trE3;
    Dm[4] += trE3;
    Dm[8] += trE3;
    inv3(Fb, det3(Fb), G);
  }
  // ---- P = (s + (vol - J p) I) F^-T ------------------------------------------
  T tauT[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) tauT[i] = s[i];
  tauT[0] += vol - J * p;
  tauT[4] += vol - J * p;
  tauT[8] += vol - J * p;
  T sb[9], Fib[9];
  mul3(Pb, Fi, sb);       // tau_bar = P_bar F^-1
  mul3_tn(Pb, tauT, Fib);  // (F^-1)_bar = P_bar^T tau
  const T trtb = sb[0] + sb[4] + sb[8];
  pbar = -J * trtb;
  Jb += (m.K * J - p) * trtb;
  Kb += T(0.5) * jm1 * (T(2) + jm1) * trtb;
  if (model_is<MODEL>(m, SPH_MODEL_NH)) {
    // s = mu J^(-2/3) dev(F F^T - I)
    const T dBd = dot9(sb, dB);
    mub += s23 * dBd;
    const T s23b = m.mu * dBd;
    T Bmb[9];
    const T trs3 = (sb[0] + sb[4] + sb[8]) * (T(1) / T(3));
#pragma unroll
    for (int i = 0; i < 9; ++i) Bmb[i] = m.mu * s23 * sb[i];
    Bmb[0] -= m.mu * s23 * trs3;
    Bmb[4] -= m.mu * s23 * trs3;
    Bmb[8] -= m.mu * s23 * trs3;
    Jb += s23b * T(-2.0 / 3.0) * s23 / J;
    add_symx(Bmb, F, Fbar);
  } else {
    // state update Y' = G Dm G^T, G = Fbar^-1, Dm = s/mu + trE3 I - (Fb Fb^T - I)
    T Yb[9];
    Yb[0] = plb[0];
    Yb[4] = plb[1];
    Yb[8] = plb[2];
    Yb[1] = Yb[3] = T(0.5) * plb[3];
    Yb[5] = Yb[7] = T(0.5) * plb[4];
    Yb[2] = Yb[6] = T(0.5) * plb[5];
    const T ab = plb[6];
    T t[9], t2[9], Dmb[9], Gb[9], Fbb[9];
    mul3_tn(G, Yb, t);
    mul3(t, G, Dmb);  // Dm_bar = G^T Y'_bar G
    mul3(Yb, G, t);
    mul3(t, Dm, Gb);  // G_bar = 2 Y'_bar G Dm  (Y'_bar, Dm symmetric)
#pragma unroll
    for (int i = 0; i < 9; ++i) Gb[i] *= T(2);
    mul3_tn(G, Gb, t);
    mul3_bt(t, G, t2);  // Fb_bar = -G^T G_bar G^T
#pragma unroll
    for (int i = 0; i < 9; ++i) Fbb[i] = -t2[i];
    const T imu = T(1) / m.mu;
#pragma unroll
    for (int i = 0; i < 9; ++i) sb[i] += Dmb[i] * imu;
    mub -= dot9(Dmb, s) * imu * imu;
    T trE3b = Dmb[0] + Dmb[4] + Dmb[8];
    T FFmb[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) FFmb[i] = -Dmb[i];
    // return mapping: s = fac s_pre, alpha' = alpha + sqrt(2/3) dg
    T spb[9];
    T snb = T(0);
    T alphab = ab;
    if (plastic) {
      const T facb = dot9(sb, spre);
#pragma unroll
      for (int i = 0; i < 9; ++i) spb[i] = fac * sb[i];
      T mubrb = -T(2) * dg / sn * facb;
      const T dgb = -T(2) * mubr / sn * facb + r23 * ab;
      snb = T(2) * mubr * dg / (sn * sn) * facb;
      const T a1 = alpha + r23 * dg;
      const T kp = hardening_slope(m, a1);
      const T Rg = -(T(2) / T(3)) * kp - T(2) * mubr;
      const T lam = -dgb / Rg;
      snb += lam;
      alphab -= lam * r23 * kp;
      mubrb -= T(2) * dg * lam;
      const T e = exp(-m.delta * a1);
      th[1] -= lam * r23 * e;
      th[2] -= lam * r23 * (T(1) - e);
      th[3] -= lam * r23 * (m.sinf - m.s0) * a1 * e;
      th[4] -= lam * r23 * a1;
      mub += mubrb * (T(1) + trE3);
      trE3b += mubrb * m.mu;
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) spb[i] = sb[i];
    }
    if (sn > T(0)) {
      const T r = snb / sn;
#pragma unroll
      for (int i = 0; i < 9; ++i) spb[i] += r * spre[i];
    }
    // s_pre = mu dev(E), trE3 = tr(E)/3
    mub += dot9(spb, spre) * imu;
    T Eb[9];
    const T trsp3 = (spb[0] + spb[4] + spb[8]) * (T(1) / T(3));
#pragma unroll
    for (int i = 0; i < 9; ++i) Eb[i] = m.mu * spb[i];
    const T dd = -m.mu * trsp3 + trE3b * (T(1) / T(3));
    Eb[0] += dd;
    Eb[4] += dd;
    Eb[8] += dd;
    // E = Fb Y Fb^T + (Fb Fb^T - I)
    T Yf[9];
    mul3_tn(Fb, Eb, t);
    mul3(t, Fb, Yf);  // Y_bar = Fb^T E_bar Fb
    mul3(Fb, Y, t);
    add_symx(Eb, t, Fbb);  // += (E_bar + E_bar^T) Fb Y
#pragma unroll
    for (int i = 0; i < 9; ++i) FFmb[i] += Eb[i];
    add_symx(FFmb, Fb, Fbb);  // += (FFm_bar + FFm_bar^T) Fb
    // Fb = c F, c = J^(-1/3)
    const T cbar = dot9(Fbb, F);
#pragma unroll
    for (int i = 0; i < 9; ++i) Fbar[i] += c * Fbb[i];
    Jb += cbar * T(-1.0 / 3.0) * c / J;
    plb[0] = Yf[0];
    plb[1] = Yf[4];
    plb[2] = Yf[8];
    plb[3] = Yf[1] + Yf[3];
    plb[4] = Yf[5] + Yf[7];
    plb[5] = Yf[2] + Yf[6];
    plb[6] = alphab;
  }
  // F^-1 and J = det F
  {
    T t[9], t2[9];
    mul3_tn(Fi, Fib, t);
    mul3_bt(t, Fi, t2);  // F_bar -= F^-T (F^-1)_bar F^-T
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Fbar[i * 3 + j] += Jb * J * Fi[j * 3 + i] - t2[i * 3 + j];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) Hbar[i] = Fbar[i];
  th[0] = mub * m.dmu_dE + Kb * m.dK_dE;
  return st;
}

// ---------------------------------------------------------------------------
// point evaluation (n independent particles)
template <typename T>
__global__ void k_constitutive(MatP<T> m, int64_t n, const T* __restrict__ H, T* plastic,
                               const T* __restrict__ p, T* __restrict__ P, Ctrl* ctrl) {
  const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  T Hm[9], pl[7] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0)}, Pm[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Hm[i] = H[i * n + a];
  if (plastic)
#pragma unroll
    for (int i = 0; i < 7; ++i) pl[i] = plastic[i * n + a];
  const int st = constitutive(m, Hm, pl, p ? p[a] : T(0), Pm);
  if (st) atomicOr(&ctrl->status, st);
#pragma unroll
  for (int i = 0; i < 9; ++i) P[i * n + a] = Pm[i];
  if (plastic)
#pragma unroll
    for (int i = 0; i < 7; ++i) plastic[i * n + a] = pl[i];
}

template <typename T>
__global__ void k_constitutive_vjp(MatP<T> m, int64_t n, const T* __restrict__ H,
                                   const T* __restrict__ plastic, const T* __restrict__ p,
                                   const T* __restrict__ Pbar, T* plb, T* __restrict__ Hbar,
                                   T* __restrict__ pbar, T* __restrict__ thb, Ctrl* ctrl) {
  const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  T Hm[9], pl[7] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0)}, Pb[9], pv[7], Hb[9], th[kNTheta];
  T pb = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    Hm[i] = H[i * n + a];
    Pb[i] = Pbar[i * n + a];
  }
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    pl[i] = plastic ? plastic[i * n + a] : T(0);
    pv[i] = plb ? plb[i * n + a] : T(0);
  }
  const int st = constitutive_vjp(m, Hm, pl, p ? p[a] : T(0), Pb, pv, Hb, pb, th);
  if (st) atomicOr(&ctrl->status, st);
#pragma unroll
  for (int i = 0; i < 9; ++i) Hbar[i * n + a] = Hb[i];
  if (plb)
#pragma unroll
    for (int i = 0; i < 7; ++i) plb[i * n + a] = pv[i];
  if (pbar) pbar[a] = pb;
  if (thb)
#pragma unroll
    for (int i = 0; i < kNTheta; ++i) thb[i * n + a] = th[i];
}

// ---------------------------------------------------------------------------
// block sum of a few doubles (all threads call it); thread 0 adds the totals
// into this workgroup's gradient slots
template <int NV>
__device__ __forceinline__ void block_grad_add(double (&v)[NV], const int (&slot)[NV],
                                               double* gpart) {
  __shared__ double wsum[NV][16];
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    double x = v[j];
#pragma unroll
    for (int mk = 1; mk < 64; mk <<= 1) x += __shfl_xor(x, mk, 64);
    v[j] = x;
  }
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) wsum[j][w] = v[j];
  __syncthreads();
  if (threadIdx.x == 0) {
    double* g = gpart + (int64_t)blockIdx.x * SPH_NGRAD;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      double s = 0.0;
      for (int k = 0; k < nw; ++k) s += wsum[j][k];
      g[slot[j]] += s;
    }
  }
}

// reverse of the stress stage + momentum sum + kick, one tile per workgroup:
// gathers a_bar = dt w (free particles) from the LDS window; takes the step's
// H = F - I from the forward run's record (Hin), writes G_bar = H_bar B0^T
// (Gb may be Hin: a particle's H is read before its G_bar is written, by the
// same thread), updates the J2 state adjoint, accumulates p_bar and the
// parameter partials.  The momentum transpose keeps its per-pair difference
// V_b a_a - V_a a_b: taking the own particle's term out of the loop makes the
// terms cancel across the pairs, which costs FP32 gradients an order of
// magnitude on smooth fields.  The window holds the relative position, V_b
// and a_b: seven values and a pad in 3D (two 16-byte LDS reads per pair),
// five and a pad in 2D.
template <typename T, int D, int LPP, int MODEL>
__global__ __launch_bounds__(256 * LPP) void k_adj_stress(
    TileGeo<T> g, MatP<T> m, const T* Hin, const T* __restrict__ w,
    const uint8_t* __restrict__ flags, T dt, T inv_rho0, const T* __restrict__ plastic,
    T* __restrict__ plb, const T* __restrict__ p, double* __restrict__ pbar, T* Gb,
    double* __restrict__ gpart, Ctrl* ctrl, Bat bt) {
  const int64_t tile = xcd_tile(g.n_tiles);
  if (tile >= g.n_tiles) return;
  constexpr int OV = D, OA = D + 1;             // offsets of V and a
  using PK = Pk<T, D == 3 ? 8 : 6>;              // (position, V, a[, 0])
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileDesc& td = g.tiles[tile];
  const uint32_t window = td.window;
  const int64_t n = g.n;
  const int64_t p0 = td.p0;
  double xo[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < D; ++k) xo[k] = g.X[k * n + p0];
  const WinMap wm = win_map(td);
  for (uint32_t l = threadIdx.x; l < window; l += blockDim.x) {
    const int64_t gi = wm(l);
    const bool fixed = flags && (flags[gi] & SPH_FLAG_FIXED);
    const T kf = fixed ? T(0) : (bt.spec ? bt.get<T>(BT_DT, bt.spec[gi]) : dt);
    T vv[D == 3 ? 8 : 6];
    vv[OV] = g.V[gi];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      vv[k] = (T)(g.X[k * n + gi] - xo[k]);
      vv[OA + k] = kf * w[k * n + gi];
    }
    vv[2 * D + 1] = T(0);
    PK::store(smem_raw, window, l, vv);
  }
  __syncthreads();
  const int t = threadIdx.x / LPP, h = threadIdx.x % LPP;
  const bool active = (uint32_t)t < td.count;
  uint32_t la, nb4;
  const int64_t a_own = tile_own(g.tslot, g.tmax, tile, td, active ? (uint32_t)t : 0u, la, nb4);
  T va[D == 3 ? 8 : 6];
  PK::load(smem_raw, window, la, va);
  T Qs[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) Qs[i][k] = T(0);
  if (active)
    ell_walk<LPP>(g.ell, td.ell_off, g.tmax, t, h, nb4, [&](uint32_t l) {
      T vb[D == 3 ? 8 : 6];
      PK::load(smem_raw, window, l, vb);
      T d[3] = {T(0), T(0), T(0)};
#pragma unroll
      for (int k = 0; k < D; ++k) d[k] = va[k] - vb[k];
      T r2 = d[0] * d[0] + d[1] * d[1];
      if (D == 3) r2 += d[2] * d[2];
      const T w0 = dw_over_r(r2, g.inv_h, g.c5);
      T e[3];
#pragma unroll
      for (int k = 0; k < D; ++k) e[k] = w0 * d[k];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const T qa = vb[OV] * va[OA + i] - va[OV] * vb[OA + i];
#pragma unroll
        for (int k = 0; k < D; ++k) Qs[i][k] += qa * e[k];
      }
    });
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) Qs[i][k] = lane_sum<LPP>(Qs[i][k]);
  double thd[kNTheta] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (active && h == 0) {
    const int64_t a = a_own;
    T B[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int k = 0; k < D; ++k) B[i][k] = g.B0[(i * D + k) * n + a];
    T Hm[9], Pb[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Hm[i] = Pb[i] = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int k = 0; k < D; ++k) {
        T ps = T(0);
#pragma unroll
        for (int l = 0; l < D; ++l) ps += Qs[i][l] * B[k][l];
        Hm[i * 3 + k] = Hin[(i * D + k) * n + a];
        Pb[i * 3 + k] = ps * inv_rho0;
      }
    T pl[7] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0)}, pv[7] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    if (model_is<MODEL>(m, SPH_MODEL_J2)) {
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        pl[i] = plastic[i * n + a];
        pv[i] = plb[i * n + a];
      }
    }
    T Hb[9], th[kNTheta], pb = T(0);
    MatP<T> mm = m;
    if (bt.spec) {
      const int sp = bt.spec[a];
      mm.mu = bt.get<T>(BT_MU, sp);
      mm.K = bt.get<T>(BT_K, sp);
      mm.lam = bt.get<T>(BT_LAM, sp);
    }
    const int st = constitutive_vjp<T, MODEL>(mm, Hm, pl, p ? p[a] : T(0), Pb, pv, Hb, pb, th);
    if (st) atomicOr(&ctrl->status, st);
    if (model_is<MODEL>(m, SPH_MODEL_J2)) {
#pragma unroll
      for (int i = 0; i < 7; ++i) plb[i * n + a] = pv[i];
    }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int k = 0; k < D; ++k) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < D; ++l) acc += Hb[i * 3 + l] * B[k][l];
        Gb[(i * D + k) * n + a] = acc;
      }
    if (pbar) pbar[a] += (double)pb;
#pragma unroll
    for (int i = 0; i < kNTheta; ++i) thd[i] = (double)th[i];
  }
  if constexpr (MODEL == SPH_MODEL_LE || MODEL == SPH_MODEL_NH) {
    // the hardening parameters' partials are zero for these models: reduce E's only
    double the[1] = {thd[0]};
    const int slot1[1] = {SPH_GRAD_E};
    block_grad_add<1>(the, slot1, gpart);
  } else {
    const int slots[kNTheta] = {SPH_GRAD_E, SPH_GRAD_S0, SPH_GRAD_SINF, SPH_GRAD_DELTA, SPH_GRAD_H};
    block_grad_add<kNTheta>(thd, slots, gpart);
  }
}

// reverse of the displacement-gradient sum:
//   u_bar_a -= sum_b (V_a G_bar_b + V_b G_bar_a) grad_a W_ab
//            = V_a sum_b G_bar_b grad_a W_ab + G_bar_a g_a,
// g_a = sum_b V_b grad_a W_ab from the build (the window holds the relative
// position and G_bar_b, twelve values in 3D); then (drift_dt != 0) the drift
// transpose of the previous inner step for free particles: w_a += drift_dt
// u_bar_a, or, with drift_incr, only this gather's increment,
// w_a -= drift_dt (...) (for a term added after that drift's transpose has
// already taken the rest of u_bar)
template <typename T, int D, int LPP>
__global__ __launch_bounds__(256 * LPP) void k_adj_gather(
    TileGeo<T> g, const T* __restrict__ Gb, double* __restrict__ ub, T* __restrict__ w,
    const uint8_t* __restrict__ flags, double drift_dt, Bat bt, int drift_incr = 0) {
  const int64_t tile = xcd_tile(g.n_tiles);
  if (tile >= g.n_tiles) return;
  using PK = Pk<T, D + D * D>;  // (relative position, G_bar_b)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileDesc& td = g.tiles[tile];
  const uint32_t window = td.window;
  const int64_t n = g.n;
  const int64_t p0 = td.p0;
  double xo[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < D; ++k) xo[k] = g.X[k * n + p0];
  const WinMap wm = win_map(td);
  for (uint32_t l = threadIdx.x; l < window; l += blockDim.x) {
    const int64_t gi = wm(l);
    T vv[D + D * D];
#pragma unroll
    for (int k = 0; k < D; ++k) vv[k] = (T)(g.X[k * n + gi] - xo[k]);
#pragma unroll
    for (int c = 0; c < D * D; ++c) vv[D + c] = Gb[c * n + gi];
    PK::store(smem_raw, window, l, vv);
  }
  __syncthreads();
  const int t = threadIdx.x / LPP, h = threadIdx.x % LPP;
  if ((uint32_t)t >= td.count) return;
  uint32_t la, nb4;
  const int64_t a = tile_own(g.tslot, g.tmax, tile, td, (uint32_t)t, la, nb4);
  T xa[D + D * D];
  PK::load(smem_raw, window, la, xa);
  const T* Ga = xa + D;
  T f[3] = {T(0), T(0), T(0)};
  ell_walk<LPP>(g.ell, td.ell_off, g.tmax, t, h, nb4, [&](uint32_t l) {
    T xb[D + D * D];
    PK::load(smem_raw, window, l, xb);
    const T* Gbb = xb + D;
    T d[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int k = 0; k < D; ++k) d[k] = xa[k] - xb[k];
    T r2 = d[0] * d[0] + d[1] * d[1];
    if (D == 3) r2 += d[2] * d[2];
    const T w0 = dw_over_r(r2, g.inv_h, g.c5);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      T s = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) s += Gbb[i * D + k] * d[k];
      f[i] += w0 * s;
    }
  });
#pragma unroll
  for (int i = 0; i < D; ++i) f[i] = lane_sum<LPP>(f[i]);
  if (h != 0) return;
  {
    const T Va = g.V[a];
    T ga[D];
#pragma unroll
    for (int k = 0; k < D; ++k) ga[k] = g.gsum[k * n + a];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      T x = Va * f[i];
#pragma unroll
      for (int k = 0; k < D; ++k) x += Ga[i * D + k] * ga[k];
      f[i] = x;
    }
  }
  const bool fixed = flags && (flags[a] & SPH_FLAG_FIXED);
  const double ddt = (drift_dt != 0.0 && bt.spec) ? bt.get<double>(BT_DT, bt.spec[a]) : drift_dt;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double un = ub[i * n + a] - (double)f[i];
    ub[i * n + a] = un;
    if (ddt != 0.0 && !fixed) w[i * n + a] += (T)(ddt * (drift_incr ? -(double)f[i] : un));
  }
}

template <typename T, int D>
__global__ void k_adj_drift(int64_t n, const double* __restrict__ ub, T* __restrict__ w,
                            const uint8_t* __restrict__ flags, double dt, Bat bt) {
  const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  if (flags && (flags[a] & SPH_FLAG_FIXED)) return;
  const double dta = bt.spec ? bt.get<double>(BT_DT, bt.spec[a]) : dt;
#pragma unroll
  for (int k = 0; k < D; ++k) w[k * n + a] += (T)(dta * ub[k * n + a]);
}

// reverse of the diffusion step, first pass (per particle a, gather over b):
//   cdot_bar_b = dt (c_bar_b + C p_bar_b) (0 on Dirichlet particles)
//   r_bar_a = -sum_b (V_b cdot_bar_a - V_a cdot_bar_b) grad_a W_ab,  q_bar = B0^T r_bar
//   D_bar += q_bar . (-B0 s_a),  s_a = sum_b V_b (c_b - c_a) grad_a W_ab (c before the step)
//   s_bar_a = -D B0^T q_bar,     C_bar += p_bar_a (c'_a - c0)
template <typename T, int D>
__global__ __launch_bounds__(kDiffBlock) void k_adiff_a(Geo<T> g, const T* __restrict__ cold,
                                                        const T* __restrict__ cnew,
                                                        const T* __restrict__ cb,
                                                        const double* __restrict__ pbar,
                                                        const uint8_t* __restrict__ flags, T dt,
                                                        T Dc, T Cs, T c0, T* __restrict__ sbar,
                                                        double* __restrict__ gpart, Bat bt,
                                                        double* __restrict__ gdiff) {
  constexpr int L = kDiffLanes;  // lanes per particle, each a strided share of its list
  const int64_t n = g.n;
  const int64_t a = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / L;
  const int h = threadIdx.x % L;
  const bool live = a < n;  // uniform over a lane group
  double gd[2] = {0.0, 0.0};
  auto cdb = [&](int64_t i) -> T {
    if (flags && (flags[i] & SPH_FLAG_CDIR)) return T(0);
    const T dti = bt.spec ? bt.get<T>(BT_DTD, bt.spec[i]) : dt;
    return dti * (cb[i] + (pbar ? Cs * (T)pbar[i] : T(0)));
  };
  T r[D], s[D];
#pragma unroll
  for (int k = 0; k < D; ++k) r[k] = s[k] = T(0);
  if (live) {
    double xa[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xa[k] = g.X[k * n + a];
    const T ca = cold[a], Va = g.V[a], cda = cdb(a);
    for (int64_t j = g.off[a] + h; j < g.off[a + 1]; j += L) {
      const uint32_t b = g.idx[j];
      T d[D];
      T r2 = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        d[k] = (T)(xa[k] - g.X[k * n + b]);
        r2 += d[k] * d[k];
      }
      const T w0 = dw_over_r(r2, g.inv_h, g.c5);
      const T Vb = g.V[b];
      const T cr = -w0 * (Vb * cda - Va * cdb(b));
      const T cs = w0 * Vb * (cold[b] - ca);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        r[k] += cr * d[k];
        s[k] += cs * d[k];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
    r[k] = lane_sum<L>(r[k]);
    s[k] = lane_sum<L>(s[k]);
  }
  if (live && h == 0) {
    const T Da = bt.spec ? bt.get<T>(BT_D, bt.spec[a]) : Dc;
    T qb[D], Bs[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T x = T(0), y = T(0);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        x += g.B0[(i * D + k) * n + a] * r[i];
        y += g.B0[(k * D + i) * n + a] * s[i];
      }
      qb[k] = x;
      Bs[k] = y;
    }
    double dsum = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      dsum -= (double)qb[k] * (double)Bs[k];
      T x = T(0);
#pragma unroll
      for (int i = 0; i < D; ++i) x += g.B0[(i * D + k) * n + a] * qb[i];
      sbar[k * n + a] = -Da * x;
    }
    gd[0] = dsum;
    gd[1] = pbar ? pbar[a] * ((double)cnew[a] - (double)c0) : 0.0;
  }
  if (bt.spec) {  // batched: per-particle partials, reduced per specimen later
    if (live && h == 0) {
      gdiff[a] += gd[0];
      gdiff[n + a] += gd[1];
    }
    return;
  }
  const int slots[2] = {SPH_GRAD_D, SPH_GRAD_C};
  block_grad_add<2>(gd, slots, gpart);
}

// second pass: c_bar_a <- (0 on Dirichlet particles, else c_bar_a + C p_bar_a)
//   - sum_b (V_a s_bar_b + V_b s_bar_a) . grad_a W_ab;  p_bar_a <- 0
template <typename T, int D>
__global__ __launch_bounds__(kDiffBlock) void k_adiff_b(Geo<T> g, const T* __restrict__ sbar,
                                                        T* __restrict__ cb, double* __restrict__ pbar,
                                                        const uint8_t* __restrict__ flags, T Cs) {
  constexpr int L = kDiffLanes;
  const int64_t n = g.n;
  const int64_t a = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / L;
  const int h = threadIdx.x % L;
  if (a >= n) return;  // the whole lane group
  double xa[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xa[k] = g.X[k * n + a];
  const T Va = g.V[a];
  T sa[D];
#pragma unroll
  for (int k = 0; k < D; ++k) sa[k] = sbar[k * n + a];
  T acc = T(0);
  for (int64_t j = g.off[a] + h; j < g.off[a + 1]; j += L) {
    const uint32_t b = g.idx[j];
    T d[D];
    T r2 = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      d[k] = (T)(xa[k] - g.X[k * n + b]);
      r2 += d[k] * d[k];
    }
    const T w0 = dw_over_r(r2, g.inv_h, g.c5);
    const T Vb = g.V[b];
    T x = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) x += (Va * sbar[k * n + b] + Vb * sa[k]) * d[k];
    acc += w0 * x;
  }
  acc = lane_sum<L>(acc);
  if (h != 0) return;
  const bool dir = flags && (flags[a] & SPH_FLAG_CDIR);
  const T direct = dir ? T(0) : cb[a] + (pbar ? Cs * (T)pbar[a] : T(0));
  cb[a] = direct - acc;
  if (pbar) pbar[a] = 0.0;
}

// ---------------------------------------------------------------------------
// reverse of the two-way coupled diffusion step.  Forward, per particle a,
// with F from u (F^-1 = Fi, J = det F), a = c / J the saturation:
//   s = sum_b V_b (a_b - a_a) grad0 W,  gr = B0 s,  gc = Fi^T gr,
//   qc = -D w gc (w = a or 1),  Q = J Fi qc,  y = B0 Q,
//   c' = c - dt sum_b V_b (y_a + y_b) . grad0 W   (Dirichlet: c' = c_bc J),
//   p = C (c' / J - c0).
// Three passes after the recomputation of Fi and a (the forward deformation
// pass): the pressure and Dirichlet terms per particle; a gather over a and
// div_bar = -dt c'_bar giving s_bar, Fi_bar and the J_bar, D and own-saturation
// terms; a gather over s_bar giving the rest of a_bar, then
// F_bar = -Fi^T Fi_bar Fi^T + J_bar J Fi^T and G_bar = F_bar B0^T, which the
// displacement-gradient transpose turns into u_bar.

template <typename T, int D>
__device__ __forceinline__ T adet(const T* A) {
  if constexpr (D == 2) return A[0] * A[3] - A[1] * A[2];
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// pass 1 (per particle): p_bar -> C gradient, c'_bar, J_bar; Dirichlet rows;
// div_bar = -dt c'_bar; the direct part of c_bar; p_bar is consumed
template <typename T, int D>
__global__ __launch_bounds__(256) void k_acd_pre(int64_t n, const T* __restrict__ Fi,
                                                 const T* __restrict__ cnew, T* __restrict__ cb,
                                                 double* __restrict__ pbar,
                                                 const uint8_t* __restrict__ flags, T dt, T c_bc,
                                                 T Cs, T c0, T* __restrict__ divb,
                                                 T* __restrict__ Jb, double* __restrict__ gpart) {
  const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double gC = 0.0;
  if (a < n) {
    T Fa[D * D];
#pragma unroll
    for (int i = 0; i < D * D; ++i) Fa[i] = Fi[i * n + a];
    const T J = T(1) / adet<T, D>(Fa);
    const T cp = cnew[a];
    const double pb = pbar ? pbar[a] : 0.0;
    gC = pb * ((double)cp / (double)J - (double)c0);
    const T cbp = cb[a] + Cs * (T)pb / J;
    T Jbar = -(Cs * (T)pb) * cp / (J * J);
    T dv = T(0), direct = T(0);
    if (flags && (flags[a] & SPH_FLAG_CDIR)) {
      Jbar += c_bc * cbp;
    } else {
      dv = -dt * cbp;
      direct = cbp;
    }
    divb[a] = dv;
    Jb[a] = Jbar;
    cb[a] = direct;
    if (pbar) pbar[a] = 0.0;
  }
  double v[1] = {gC};
  const int slot[1] = {SPH_GRAD_C};
  block_grad_add<1>(v, slot, gpart);
}

// pass 2 (tiled gather over the saturation and div_bar)
template <typename T, int D, int LPP>
__global__ __launch_bounds__(256 * LPP) void k_acd_a(
    TileGeo<T> g, const T* __restrict__ sat, const T* __restrict__ divb, const T* __restrict__ Fi,
    T* __restrict__ Jb, T* __restrict__ sbar, T* __restrict__ Fib, T* __restrict__ cb,
    const T* __restrict__ cold, T Dc, int nonlinear, double* __restrict__ gpart) {
  const int64_t tile = xcd_tile(g.n_tiles);
  if (tile >= g.n_tiles) return;  // the whole block
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileDesc& td = g.tiles[tile];
  const uint32_t window = td.window;
  vec4<T>* sx = reinterpret_cast<vec4<T>*>(smem_raw);
  vec4<T>* sf = sx + window;  // (saturation, div_bar, -, -)
  const int64_t n = g.n;
  const int64_t p0 = td.p0;
  double xo[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < D; ++k) xo[k] = g.X[k * n + p0];
  const WinMap wm = win_map(td);
  for (uint32_t l = threadIdx.x; l < window; l += blockDim.x) {
    const int64_t gi = wm(l);
    vec4<T> xv, fv;
    xv.x = (T)(g.X[gi] - xo[0]);
    xv.y = (T)(g.X[n + gi] - xo[1]);
    xv.z = D == 3 ? (T)(g.X[2 * n + gi] - xo[2]) : T(0);
    xv.w = g.V[gi];
    fv.x = sat[gi];
    fv.y = divb[gi];
    fv.z = T(0);
    fv.w = T(0);
    sx[l] = xv;
    sf[l] = fv;
  }
  __syncthreads();
  const int t = threadIdx.x / LPP, h = threadIdx.x % LPP;
  const bool active = (uint32_t)t < td.count;
  uint32_t la, nb4;
  const int64_t a = tile_own(g.tslot, g.tmax, tile, td, active ? (uint32_t)t : 0u, la, nb4);
  const vec4<T> xa = sx[la], fa = sf[la];
  T sv[3] = {T(0), T(0), T(0)}, m[3] = {T(0), T(0), T(0)}, e[3] = {T(0), T(0), T(0)};
  if (active)
    ell_walk<LPP>(g.ell, td.ell_off, g.tmax, t, h, nb4, [&](uint32_t l) {
      const vec4<T> xb = sx[l], fb = sf[l];
      T d[3] = {xa.x - xb.x, xa.y - xb.y, xa.z - xb.z};
      T r2 = d[0] * d[0] + d[1] * d[1];
      if (D == 3) r2 += d[2] * d[2];
      const T w0 = dw_over_r(r2, g.inv_h, g.c5);
      const T wb = w0 * xb.w;
      const T ws = wb * (fb.x - fa.x), we = w0 * fb.y;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        sv[k] += ws * d[k];
        m[k] += wb * d[k];
        e[k] += we * d[k];
      }
    });
#pragma unroll
  for (int k = 0; k < D; ++k) {
    sv[k] = lane_sum<LPP>(sv[k]);
    m[k] = lane_sum<LPP>(m[k]);
    e[k] = lane_sum<LPP>(e[k]);
  }
  double gD = 0.0;
  if (active && h == 0) {
    T B[D][D], Fa[D * D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int k = 0; k < D; ++k) B[i][k] = g.B0[(i * D + k) * n + a];
#pragma unroll
    for (int i = 0; i < D * D; ++i) Fa[i] = Fi[i * n + a];
    const T J = T(1) / adet<T, D>(Fa);
    // y_bar = div_bar_a sum_b V_b grad W - V_a sum_b div_bar_b grad W
    T yb[D], gr[D], gc[D], qc[D], Qb[D], qcb[D], gcb[D], grb[D];
#pragma unroll
    for (int k = 0; k < D; ++k) yb[k] = fa.y * m[k] - xa.w * e[k];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      T x = T(0), y = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        x += B[i][k] * sv[k];   // gr = B0 s
        y += B[k][i] * yb[k];   // Q_bar = B0^T y_bar
      }
      gr[i] = x;
      Qb[i] = y;
    }
#pragma unroll
    for (int mm = 0; mm < D; ++mm) {
      T x = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) x += Fa[k * D + mm] * gr[k];  // Fi^T gr
      gc[mm] = x;
    }
    const T wa = nonlinear ? fa.x : T(1);
#pragma unroll
    for (int mm = 0; mm < D; ++mm) qc[mm] = -Dc * wa * gc[mm];
    // Q = J Fi qc
    T Jbar = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T x = T(0);
#pragma unroll
      for (int mm = 0; mm < D; ++mm) x += Fa[mm * D + k] * Qb[mm];
      qcb[k] = J * x;  // J Fi^T Q_bar
    }
#pragma unroll
    for (int mm = 0; mm < D; ++mm) {
      T x = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) x += Fa[mm * D + k] * qc[k];
      Jbar += Qb[mm] * x;  // Q_bar . (Fi qc)
    }
    // qc = -D w gc
    T gq = T(0);
#pragma unroll
    for (int mm = 0; mm < D; ++mm) {
      gcb[mm] = -Dc * wa * qcb[mm];
      gq += gc[mm] * qcb[mm];
    }
    gD = -(double)wa * (double)gq;
    const T a_own = nonlinear ? -Dc * gq : T(0);  // w_bar, w = a
    // gc = Fi^T gr
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T x = T(0);
#pragma unroll
      for (int mm = 0; mm < D; ++mm) x += Fa[k * D + mm] * gcb[mm];
      grb[k] = x;  // Fi gc_bar
    }
    // Fi_bar = J Q_bar (x) qc + gr (x) gc_bar
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int k = 0; k < D; ++k) Fib[(i * D + k) * n + a] = J * Qb[i] * qc[k] + gr[i] * gcb[k];
    // s_bar = B0^T gr_bar
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T x = T(0);
#pragma unroll
      for (int i = 0; i < D; ++i) x += B[i][k] * grb[i];
      sbar[k * n + a] = x;
    }
    // a = c / J: the own saturation term of the nonlinear flux
    const T ca = cold[a];
    cb[a] += a_own / J;
    Jb[a] += Jbar - a_own * ca / (J * J);
  }
  double v[1] = {gD};
  const int slot[1] = {SPH_GRAD_D};
  block_grad_add<1>(v, slot, gpart);
}

// pass 3 (tiled gather over s_bar): a_bar_a = -sum_b (V_a s_bar_b + V_b s_bar_a) . grad0 W;
// c_bar += a_bar / J, J_bar -= a_bar c / J^2; F_bar and G_bar = F_bar B0^T (into Fib)
template <typename T, int D, int LPP>
__global__ __launch_bounds__(256 * LPP) void k_acd_b(TileGeo<T> g, const T* __restrict__ sbar,
                                                     const T* __restrict__ Fi, T* __restrict__ Fib,
                                                     const T* __restrict__ Jb, T* __restrict__ cb,
                                                     const T* __restrict__ cold) {
  const int64_t tile = xcd_tile(g.n_tiles);
  if (tile >= g.n_tiles) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileDesc& td = g.tiles[tile];
  const uint32_t window = td.window;
  vec4<T>* sx = reinterpret_cast<vec4<T>*>(smem_raw);
  vec4<T>* ss = sx + window;
  const int64_t n = g.n;
  const int64_t p0 = td.p0;
  double xo[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < D; ++k) xo[k] = g.X[k * n + p0];
  const WinMap wm = win_map(td);
  for (uint32_t l = threadIdx.x; l < window; l += blockDim.x) {
    const int64_t gi = wm(l);
    vec4<T> xv, sv;
    xv.x = (T)(g.X[gi] - xo[0]);
    xv.y = (T)(g.X[n + gi] - xo[1]);
    xv.z = D == 3 ? (T)(g.X[2 * n + gi] - xo[2]) : T(0);
    xv.w = g.V[gi];
    sv.x = sbar[gi];
    sv.y = sbar[n + gi];
    sv.z = D == 3 ? sbar[2 * n + gi] : T(0);
    sv.w = T(0);
    sx[l] = xv;
    ss[l] = sv;
  }
  __syncthreads();
  const int t = threadIdx.x / LPP, h = threadIdx.x % LPP;
  if ((uint32_t)t >= td.count) return;
  uint32_t la, nb4;
  const int64_t a = tile_own(g.tslot, g.tmax, tile, td, (uint32_t)t, la, nb4);
  const vec4<T> xa = sx[la], sa = ss[la];
  T t1 = T(0), m[3] = {T(0), T(0), T(0)};
  ell_walk<LPP>(g.ell, td.ell_off, g.tmax, t, h, nb4, [&](uint32_t l) {
    const vec4<T> xb = sx[l], sb = ss[l];
    T d[3] = {xa.x - xb.x, xa.y - xb.y, xa.z - xb.z};
    T r2 = d[0] * d[0] + d[1] * d[1];
    if (D == 3) r2 += d[2] * d[2];
    const T w0 = dw_over_r(r2, g.inv_h, g.c5);
    T sd = sb.x * d[0] + sb.y * d[1];
    if (D == 3) sd += sb.z * d[2];
    t1 += w0 * sd;
    const T wb = w0 * xb.w;
#pragma unroll
    for (int k = 0; k < D; ++k) m[k] += wb * d[k];
  });
  T tot = xa.w * t1 + sa.x * m[0] + sa.y * m[1];
  if (D == 3) tot += sa.z * m[2];
  tot = lane_sum<LPP>(tot);
  if (h != 0) return;
  const T abar = -tot;
  T Fa[D * D], M[D * D];
#pragma unroll
  for (int i = 0; i < D * D; ++i) {
    Fa[i] = Fi[i * n + a];
    M[i] = Fib[i * n + a];
  }
  const T J = T(1) / adet<T, D>(Fa);
  const T ca = cold[a];
  cb[a] += abar / J;
  const T Jbar = Jb[a] - abar * ca / (J * J);
  // F_bar = -Fi^T Fi_bar Fi^T + J_bar J Fi^T
  T P[D * D], Fb[D * D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T x = T(0);
#pragma unroll
      for (int l = 0; l < D; ++l) x += M[i * D + l] * Fa[k * D + l];  // Fi_bar Fi^T
      P[i * D + k] = x;
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T x = T(0);
#pragma unroll
      for (int l = 0; l < D; ++l) x += Fa[l * D + i] * P[l * D + k];  // Fi^T (...)
      Fb[i * D + k] = -x + Jbar * J * Fa[k * D + i];
    }
  // G_bar = F_bar B0^T
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T x = T(0);
#pragma unroll
      for (int l = 0; l < D; ++l) x += Fb[i * D + l] * g.B0[(k * D + l) * n + a];
      Fib[(i * D + k) * n + a] = x;
    }
}

// fixed-order reduction of the gradient partials into grad (+=); clears them
__global__ __launch_bounds__(256) void k_grad_reduce(double* __restrict__ gpart, int64_t slots,
                                                     double* __restrict__ grad) {
  __shared__ double red[256];
  for (int gi = 0; gi < SPH_NGRAD; ++gi) {
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < slots; j += 256) {
      s += gpart[j * SPH_NGRAD + gi];
      gpart[j * SPH_NGRAD + gi] = 0.0;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) grad[gi] += red[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// host side
static inline unsigned nblk256(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

int grad_reduce(const sph_nbr* nb, double* grad, hipStream_t s) {
  k_grad_reduce<<<1, 256, 0, s>>>(nb->gpart, nb->gpart_slots, grad);
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

template <typename T, int D, int LS, int LG, int MODEL>
static int adj_solid_l(const sph_nbr* nb, const sph_material* m, const void* H,
                       const void* plastic, const sph_state* st, const sph_adjoint* adj,
                       double dt, double drift_dt, hipStream_t s) {
  const int prec = sizeof(T) == 8 ? SPH_F64 : SPH_F32;
  TileGeo<T> g = tile_geo<T>(nb, prec);
  if (g.n_tiles == 0) return SPH_OK;
  MatP<T> mp = matp<T>(m);
  const unsigned grid = (unsigned)(8 * ((g.n_tiles + 7) / 8));
  if ((int64_t)grid > nb->gpart_slots) {
    set_error("gradient partial slots too few");
    return SPH_E_CAPACITY;
  }
  const size_t wm = (size_t)nb->tiling[prec].window_max;
  const size_t lds_s = wm * Pk<T, D == 3 ? 8 : 6>::bytes + 16;
  const size_t lds_g = wm * Pk<T, D + D * D>::bytes + 16;
  int rc = SPH_OK;
  if constexpr (LS > 0) {
    if ((rc = lds_attr(k_adj_stress<T, D, LS, MODEL>, lds_s))) return rc;
    hipEvent_t pe_ = prof_begin(nb, SPH_KERNEL_ADJ_STRESS, s);
    k_adj_stress<T, D, LS, MODEL><<<grid, (unsigned)(g.tmax * LS), lds_s, s>>>(
        g, mp, (const T*)H, (const T*)adj->v, st->flags, (T)dt, (T)(1.0 / m->rho0), (const T*)plastic,
        (T*)adj->plastic, (const T*)st->p, adj->p, (T*)adj->work, nb->gpart, nb->ctrl,
        bat_view(nb));
    prof_end(nb, SPH_KERNEL_ADJ_STRESS, pe_, s);
    SPH_LAUNCH_CHECK();
  }
  if constexpr (LG > 0) {
    if ((rc = lds_attr(k_adj_gather<T, D, LG>, lds_g))) return rc;
    hipEvent_t pe_ = prof_begin(nb, SPH_KERNEL_ADJ_GATHER, s);
    k_adj_gather<T, D, LG><<<grid, (unsigned)(g.tmax * LG), lds_g, s>>>(
        g, (const T*)adj->work, adj->u, (T*)adj->v, st->flags, drift_dt, bat_view(nb));
    prof_end(nb, SPH_KERNEL_ADJ_GATHER, pe_, s);
    SPH_LAUNCH_CHECK();
  }
  return SPH_OK;
}

template <typename T, int D>
static int adj_solid_t(const sph_nbr* nb, const sph_material* m, const void* u,
                       const void* plastic, const sph_state* st, const sph_adjoint* adj,
                       double dt, double drift_dt, hipStream_t s) {
  const int prec = sizeof(T) == 8 ? SPH_F64 : SPH_F32;
  int rc;
  const int ls = nb->tune.lpp[TUNE_ADJ_STRESS][prec];
  auto stress = [&](auto model_c) -> int {
    constexpr int M = decltype(model_c)::value;
    switch (ls) {
      case 1: return adj_solid_l<T, D, 1, 0, M>(nb, m, u, plastic, st, adj, dt, drift_dt, s);
      case 4: return adj_solid_l<T, D, 4, 0, M>(nb, m, u, plastic, st, adj, dt, drift_dt, s);
      default: return adj_solid_l<T, D, 2, 0, M>(nb, m, u, plastic, st, adj, dt, drift_dt, s);
    }
  };
  switch (m->model) {
    case SPH_MODEL_LE: rc = stress(std::integral_constant<int, SPH_MODEL_LE>{}); break;
    case SPH_MODEL_NH: rc = stress(std::integral_constant<int, SPH_MODEL_NH>{}); break;
    default: rc = stress(std::integral_constant<int, SPH_MODEL_J2>{}); break;
  }
  if (rc) return rc;
  switch (nb->tune.lpp[TUNE_ADJ_GATHER][prec]) {
    case 2: return adj_solid_l<T, D, 0, 2, -1>(nb, m, u, plastic, st, adj, dt, drift_dt, s);
    case 1: return adj_solid_l<T, D, 0, 1, -1>(nb, m, u, plastic, st, adj, dt, drift_dt, s);
    default: return adj_solid_l<T, D, 0, 4, -1>(nb, m, u, plastic, st, adj, dt, drift_dt, s);
  }
}

static int check_adj(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                     const sph_adjoint* adj) {
  int rc = check_state(nb, st, false);
  if (rc) return rc;
  if (!m || !adj) {
    set_error("material or adjoint is NULL");
    return SPH_E_ARG;
  }
  if (adj->prec != st->prec) {
    set_error("adjoint and state precisions differ");
    return SPH_E_ARG;
  }
  if (m->rho_l0 != 0.0) {
    set_error("the reverse steps cover the dry solid only (rho_l0 = 0)");
    return SPH_E_UNSUPPORTED;
  }
  if (!adj->u || !adj->v || !adj->work || !adj->grad) {
    set_error("adjoint arrays u, v, work and grad are required");
    return SPH_E_ARG;
  }
  if (m->model == SPH_MODEL_J2 && (!st->plastic || !adj->plastic)) {
    set_error("J2 needs the plastic state and its adjoint");
    return SPH_E_ARG;
  }
  return SPH_OK;
}

int adj_solid(const sph_nbr* nb, const sph_material* m, const void* u, const void* plastic,
              const sph_state* st, const sph_adjoint* adj, double dt, double drift_dt,
              hipStream_t s) {
  if (st->prec == SPH_F64)
    return nb->dim == 2 ? adj_solid_t<double, 2>(nb, m, u, plastic, st, adj, dt, drift_dt, s)
                        : adj_solid_t<double, 3>(nb, m, u, plastic, st, adj, dt, drift_dt, s);
  return nb->dim == 2 ? adj_solid_t<float, 2>(nb, m, u, plastic, st, adj, dt, drift_dt, s)
                      : adj_solid_t<float, 3>(nb, m, u, plastic, st, adj, dt, drift_dt, s);
}

int adj_damping(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                const sph_adjoint* adj, double eta, double dt, hipStream_t s) {
  sph_state w = *st;
  w.prec = adj->prec;
  w.v = adj->v;
  return damping_sweep_rev(nb, m, &w, eta, dt, s);
}

int adj_drift(const sph_nbr* nb, const sph_state* st, const sph_adjoint* adj, double dt,
              hipStream_t s) {
  const unsigned gr = nblk256(nb->n);
  if (adj->prec == SPH_F64) {
    if (nb->dim == 2) k_adj_drift<double, 2><<<gr, 256, 0, s>>>(nb->n, adj->u, (double*)adj->v, st->flags, dt, bat_view(nb));
    else k_adj_drift<double, 3><<<gr, 256, 0, s>>>(nb->n, adj->u, (double*)adj->v, st->flags, dt, bat_view(nb));
  } else {
    if (nb->dim == 2) k_adj_drift<float, 2><<<gr, 256, 0, s>>>(nb->n, adj->u, (float*)adj->v, st->flags, dt, bat_view(nb));
    else k_adj_drift<float, 3><<<gr, 256, 0, s>>>(nb->n, adj->u, (float*)adj->v, st->flags, dt, bat_view(nb));
  }
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

template <typename T, int D>
static int adj_diffusion_t(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                           const void* c_before, const sph_adjoint* adj, double Dc, double dt,
                           hipStream_t s) {
  Geo<T> g = geo<T>(nb);
  const unsigned gr = nblk(nb->n, kDiffPerBlock);
  if ((int64_t)gr > nb->gpart_slots) {
    set_error("gradient partial slots too few");
    return SPH_E_CAPACITY;
  }
  k_adiff_a<T, D><<<gr, kDiffBlock, 0, s>>>(g, (const T*)c_before, (const T*)st->c, (const T*)adj->c,
                                     adj->p, st->flags, (T)dt, (T)Dc, (T)m->C_swell, (T)m->c0,
                                     (T*)adj->work, nb->gpart, bat_view(nb), nb->gdiff);
  SPH_LAUNCH_CHECK();
  k_adiff_b<T, D><<<gr, kDiffBlock, 0, s>>>(g, (const T*)adj->work, (T*)adj->c, adj->p, st->flags,
                                     (T)m->C_swell);
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

template <typename T, int D>
static int adj_diffusion_coupled_t(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                                   const double* u_before, const void* c_before,
                                   const sph_adjoint* adj, double Dc, double dt, double c_bc,
                                   int nonlinear, double drift_dt, hipStream_t s) {
  const int prec = sizeof(T) == 8 ? SPH_F64 : SPH_F32;
  const int64_t n = nb->n;
  TileGeo<T> g = tile_geo<T>(nb, prec);
  if (g.n_tiles == 0) return SPH_OK;
  const unsigned grid = (unsigned)(8 * ((g.n_tiles + 7) / 8));
  const unsigned gr0 = nblk(n, 256);
  if ((int64_t)grid > nb->gpart_slots || (int64_t)gr0 > nb->gpart_slots) {
    set_error("gradient partial slots too few");
    return SPH_E_CAPACITY;
  }
  constexpr int L = 2;
  const size_t wm = (size_t)nb->tiling[prec].window_max;
  const size_t lds2 = wm * 2 * sizeof(vec4<T>);
  const size_t lds_g = wm * Pk<T, D + D * D>::bytes + 16;
  int rc;
  if ((rc = lds_attr(k_acd_a<T, D, L>, lds2)) || (rc = lds_attr(k_acd_b<T, D, L>, lds2)) ||
      (rc = lds_attr(k_adj_gather<T, D, L>, lds_g)))
    return rc;
  // scratch: the state arrays the reverse pass re-runs over anyway
  T* Fi = (T*)st->PB;              // F^-1 of the step's u
  T* sat = (T*)st->p;              // c / J
  T* sbar = (T*)st->q;             // [D][n]
  T* divb = (T*)st->v;             // first component of v
  T* Jb = (T*)st->v + n;           // second component of v
  T* Fib = (T*)adj->work;          // Fi_bar, then G_bar
  if ((rc = diffusion_F(nb, prec, u_before, c_before, Fi, sat, s))) return rc;
  k_acd_pre<T, D><<<gr0, 256, 0, s>>>(n, Fi, (const T*)st->c, (T*)adj->c, adj->p, st->flags, (T)dt,
                                      (T)c_bc, (T)m->C_swell, (T)m->c0, divb, Jb, nb->gpart);
  SPH_LAUNCH_CHECK();
  k_acd_a<T, D, L><<<grid, (unsigned)(g.tmax * L), lds2, s>>>(g, sat, divb, Fi, Jb, sbar, Fib,
                                                               (T*)adj->c, (const T*)c_before,
                                                               (T)Dc, nonlinear, nb->gpart);
  SPH_LAUNCH_CHECK();
  k_acd_b<T, D, L><<<grid, (unsigned)(g.tmax * L), lds2, s>>>(g, sbar, Fi, Fib, Jb, (T*)adj->c,
                                                               (const T*)c_before);
  SPH_LAUNCH_CHECK();
  k_adj_gather<T, D, L><<<grid, (unsigned)(g.tmax * L), lds_g, s>>>(g, Fib, adj->u, (T*)adj->v,
                                                                     st->flags, drift_dt,
                                                                     bat_view(nb), 1);
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

int adj_diffusion_coupled(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                          const double* u_before, const void* c_before, const sph_adjoint* adj,
                          double Dc, double dt, double c_bc, int nonlinear, double drift_dt,
                          hipStream_t s) {
  if (!st->c || !st->q || !st->p || !st->PB || !st->v || !c_before || !u_before || !adj->c ||
      !adj->work) {
    set_error("the coupled diffusion reverse needs c, q, p, PB, v, the step's u and c and the "
              "adjoint c and work arrays");
    return SPH_E_ARG;
  }
  if (st->prec == SPH_F64)
    return nb->dim == 2
               ? adj_diffusion_coupled_t<double, 2>(nb, m, st, u_before, c_before, adj, Dc, dt, c_bc, nonlinear, drift_dt, s)
               : adj_diffusion_coupled_t<double, 3>(nb, m, st, u_before, c_before, adj, Dc, dt, c_bc, nonlinear, drift_dt, s);
  return nb->dim == 2
             ? adj_diffusion_coupled_t<float, 2>(nb, m, st, u_before, c_before, adj, Dc, dt, c_bc, nonlinear, drift_dt, s)
             : adj_diffusion_coupled_t<float, 3>(nb, m, st, u_before, c_before, adj, Dc, dt, c_bc, nonlinear, drift_dt, s);
}

int adj_diffusion(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                  const void* c_before, const sph_adjoint* adj, double Dc, double dt,
                  hipStream_t s) {
  if (!st->c || !c_before || !adj->c || !adj->work) {
    set_error("the diffusion reverse needs c, c_before and the adjoint c and work arrays");
    return SPH_E_ARG;
  }
  if (st->prec == SPH_F64)
    return nb->dim == 2 ? adj_diffusion_t<double, 2>(nb, m, st, c_before, adj, Dc, dt, s)
                        : adj_diffusion_t<double, 3>(nb, m, st, c_before, adj, Dc, dt, s);
  return nb->dim == 2 ? adj_diffusion_t<float, 2>(nb, m, st, c_before, adj, Dc, dt, s)
                      : adj_diffusion_t<float, 3>(nb, m, st, c_before, adj, Dc, dt, s);
}

}  // namespace sph

using namespace sph;

extern "C" int sph_solid_relax_step_vjp(const sph_nbr* nb, const sph_material* mat,
                                        const sph_state* st, const sph_adjoint* adj, double dt_s,
                                        void* stream) {
  clear_error();
  int rc = check_adj(nb, mat, st, adj);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  // the step's H from u, into adj->work, where the reverse replaces it by G_bar
  if ((rc = displacement_gradient(nb, st, adj->work, s))) return rc;
  rc = adj_solid(nb, mat, adj->work, st->plastic, st, adj, dt_s, 0.0, s);
  if (rc) return rc;
  return grad_reduce(nb, adj->grad, s);
}

extern "C" int sph_damping_sweep_vjp(const sph_nbr* nb, const sph_material* mat,
                                     const sph_state* st, const sph_adjoint* adj, double eta,
                                     double dt_s, void* stream) {
  clear_error();
  int rc = check_state(nb, st, false);
  if (rc) return rc;
  if (!mat || !adj || !adj->v || adj->prec != st->prec) {
    set_error("material and the adjoint v (in the state's precision) are required");
    return SPH_E_ARG;
  }
  return adj_damping(nb, mat, st, adj, eta, dt_s, (hipStream_t)stream);
}

extern "C" int sph_drift_vjp(const sph_nbr* nb, const sph_state* st, const sph_adjoint* adj,
                             double dt_s, void* stream) {
  clear_error();
  int rc = check_state(nb, st, false);
  if (rc) return rc;
  if (!adj || !adj->u || !adj->v || adj->prec != st->prec) {
    set_error("adjoint u and v required, in the state's precision");
    return SPH_E_ARG;
  }
  return adj_drift(nb, st, adj, dt_s, (hipStream_t)stream);
}

extern "C" int sph_diffusion_step_vjp(const sph_nbr* nb, const sph_material* mat,
                                      const sph_state* st, const void* c_before,
                                      const sph_adjoint* adj, double D, double dt_d, double c_bc,
                                      void* stream) {
  clear_error();
  (void)c_bc;  // the Dirichlet value is a constant: it has no derivative
  int rc = check_adj(nb, mat, st, adj);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  rc = adj_diffusion(nb, mat, st, c_before, adj, D, dt_d, s);
  if (rc) return rc;
  return grad_reduce(nb, adj->grad, s);
}

extern "C" int sph_diffusion_step_coupled_vjp(const sph_nbr* nb, const sph_material* mat,
                                              const sph_state* st, const void* c_before,
                                              const sph_adjoint* adj, double D, double dt_d,
                                              double c_bc, int32_t nonlinear, void* stream) {
  clear_error();
  int rc = check_adj(nb, mat, st, adj);
  if (rc) return rc;
  if (nb->spec) {
    set_error("the coupled diffusion reverse takes one specimen (D is a scalar here)");
    return SPH_E_UNSUPPORTED;
  }
  if (!st->v) {
    set_error("the coupled diffusion reverse needs st->v as working storage");
    return SPH_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  // no inner step precedes a lone step: nothing to fold into a drift
  rc = adj_diffusion_coupled(nb, mat, st, st->u, c_before, adj, D, dt_d, c_bc, nonlinear, 0.0, s);
  if (rc) return rc;
  return grad_reduce(nb, adj->grad, s);
}

namespace {
Ctrl* g_point_ctrl = nullptr;  // status word of the point evaluations (per process)

int point_ctrl(Ctrl** out) {
  if (!g_point_ctrl) {
    SPH_HIP(hipMalloc(&g_point_ctrl, sizeof(Ctrl)));
    SPH_HIP(hipMemset(g_point_ctrl, 0, sizeof(Ctrl)));
  }
  *out = g_point_ctrl;
  return SPH_OK;
}

int point_status(hipStream_t s) {
  Ctrl h;
  SPH_HIP(hipMemcpyAsync(&h, g_point_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  if (h.status) {
    SPH_HIP(hipMemset(g_point_ctrl, 0, sizeof(Ctrl)));
    set_error("device status bits 0x%x", h.status);
    return SPH_E_NUMERIC;
  }
  return SPH_OK;
}
}  // namespace

extern "C" int sph_constitutive(const sph_material* mat, int prec, int64_t n, const void* H,
                                void* plastic, const void* p, void* P, void* stream) {
  clear_error();
  if (!mat || n < 0 || (n > 0 && (!H || !P)) || (mat->model == SPH_MODEL_J2 && n > 0 && !plastic)) {
    set_error("bad arguments");
    return SPH_E_ARG;
  }
  if (prec != SPH_F32 && prec != SPH_F64) {
    set_error("prec must be SPH_F32 or SPH_F64");
    return SPH_E_UNSUPPORTED;
  }
  if (n == 0) return SPH_OK;
  Ctrl* c = nullptr;
  int rc = point_ctrl(&c);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  void* pl = mat->model == SPH_MODEL_J2 ? plastic : nullptr;
  if (prec == SPH_F64)
    k_constitutive<double><<<nblk256(n), 256, 0, s>>>(matp<double>(mat), n, (const double*)H,
                                                      (double*)pl, (const double*)p, (double*)P, c);
  else
    k_constitutive<float><<<nblk256(n), 256, 0, s>>>(matp<float>(mat), n, (const float*)H,
                                                     (float*)pl, (const float*)p, (float*)P, c);
  SPH_LAUNCH_CHECK();
  return point_status(s);
}

extern "C" int sph_constitutive_vjp(const sph_material* mat, int prec, int64_t n, const void* H,
                                    const void* plastic, const void* p, const void* Pbar,
                                    void* plastic_bar, void* Hbar, void* pbar, void* theta_bar,
                                    void* stream) {
  clear_error();
  if (!mat || n < 0 || (n > 0 && (!H || !Pbar || !Hbar)) ||
      (mat->model == SPH_MODEL_J2 && n > 0 && (!plastic || !plastic_bar))) {
    set_error("bad arguments");
    return SPH_E_ARG;
  }
  if (prec != SPH_F32 && prec != SPH_F64) {
    set_error("prec must be SPH_F32 or SPH_F64");
    return SPH_E_UNSUPPORTED;
  }
  if (n == 0) return SPH_OK;
  Ctrl* c = nullptr;
  int rc = point_ctrl(&c);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const bool j2 = mat->model == SPH_MODEL_J2;
  if (prec == SPH_F64)
    k_constitutive_vjp<double><<<nblk256(n), 256, 0, s>>>(
        matp<double>(mat), n, (const double*)H, j2 ? (const double*)plastic : nullptr,
        (const double*)p, (const double*)Pbar, j2 ? (double*)plastic_bar : nullptr, (double*)Hbar,
        (double*)pbar, (double*)theta_bar, c);
  else
    k_constitutive_vjp<float><<<nblk256(n), 256, 0, s>>>(
        matp<float>(mat), n, (const float*)H, j2 ? (const float*)plastic : nullptr,
        (const float*)p, (const float*)Pbar, j2 ? (float*)plastic_bar : nullptr, (float*)Hbar,
        (float*)pbar, (float*)theta_bar, c);
  SPH_LAUNCH_CHECK();
  return point_status(s);
}
