// sph_step.hip -- inner-step and slow-step kernels of the TL-SPH path on gfx950.
//
// Layout: structure-of-arrays [component][n] in cell-sorted order, so that a
// wavefront of 64 consecutive particles reads 64 consecutive words of every
// component, and the neighbours it gathers sit in the same few cells.
// Reference geometry (X) and displacement (u) are FP64.  A tile stages its
// window's positions and displacements relative to the tile's first particle,
// differenced in FP64 and then rounded to the working type T; the per-pair
// differences are then taken in T.  In FP32 each staged value carries a
// rounding error of at most 2^-24 of its offset from that particle, so a pair
// difference is off by at most ~2^-23 times the tile's extent (a few support
// radii), not by the rounding of the absolute coordinates.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "sph_device.h"

namespace sph {

// Mixture terms of an inner step (a solid saturated by a fluid, Sec. 2.2.1):
// the momentum the fluid carries, beside the stress, and the fluid's mass in
// the inertia.  Dry (c == nullptr) unless the material has a fluid density
// and the state holds the content c and the reference flux q of the last
// slow step.
template <typename T>
struct Mix {
  const T* v;  // [d][n] solid velocity
  const T* c;  // [n] fluid content per reference volume; nullptr: dry
  const T* q;  // [d][n] reference flux of fluid content
  T rho0, rho_l0;
};

template <typename T>
static Mix<T> mix_view(const sph_material* m, const sph_state* st) {
  const bool on = m->rho_l0 > 0.0 && st->c && st->q;
  return Mix<T>{(const T*)st->v, on ? (const T*)st->c : nullptr, (const T*)st->q, (T)m->rho0,
                (T)m->rho_l0};
}

// stress stage: H = (sum_b V_b (u_b - u_a) (x) grad_a W_ab) B0_a; P(H); PB = P B0.
// A recorded run (rec_H) keeps the H of every inner step, [k][D*D][n], for
// the reverse pass; HONLY writes H to rec_H (no step index) and stops there.
template <typename T, int D, int LPP, int MODEL, bool HONLY = false>
__global__ __launch_bounds__(256 * LPP) void k_stress(TileGeo<T> g, MatP<T> m,
                                                             const double* __restrict__ u,
                                                             T* __restrict__ PB,
                                                             T* __restrict__ plastic,
                                                             const T* __restrict__ p, Ctrl* ctrl,
                                                             bool gated, T* __restrict__ rec_pl,
                                                             T* __restrict__ rec_H,
                                                             Bat bt, Mix<T> mx) {
  if (gated && ctrl->done) return;
  const int64_t tile = xcd_tile(g.n_tiles);
  if (tile >= g.n_tiles) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileDesc& td = g.tiles[tile];
  const uint32_t window = td.window;
  vec4<T>* sx = reinterpret_cast<vec4<T>*>(smem_raw);
  vec4<T>* su = sx + window;
  const int64_t n = g.n;
  const int64_t p0 = td.p0;
  double xo[3] = {0, 0, 0}, uo[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < D; ++k) {
    xo[k] = g.X[k * n + p0];
    uo[k] = u[k * n + p0];
  }
  const WinMap wm = win_map(td);
  // stage the window, two particles per thread in flight
  for (uint32_t l0 = threadIdx.x; l0 < window; l0 += 2 * blockDim.x) {
    vec4<T> xv[2], uv[2];
    uint32_t ls[2] = {l0, l0 + blockDim.x};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (ls[e] < window) {
        const int64_t gi = wm(ls[e]);
        xv[e].x = (T)(g.X[gi] - xo[0]);
        xv[e].y = (T)(g.X[n + gi] - xo[1]);
        xv[e].z = D == 3 ? (T)(g.X[2 * n + gi] - xo[2]) : T(0);
        xv[e].w = g.V[gi];
        uv[e].x = (T)(u[gi] - uo[0]);
        uv[e].y = (T)(u[n + gi] - uo[1]);
        uv[e].z = D == 3 ? (T)(u[2 * n + gi] - uo[2]) : T(0);
        uv[e].w = T(0);
      }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (ls[e] < window) {
        sx[ls[e]] = xv[e];
        su[ls[e]] = uv[e];
      }
  }
  __syncthreads();
  const int t = threadIdx.x / LPP, h = threadIdx.x % LPP;
  if ((uint32_t)t >= td.count) return;
  uint32_t la, nb4;
  const int64_t a = tile_own(g.tslot, g.tmax, tile, td, (uint32_t)t, la, nb4);
  const vec4<T> xa = sx[la], ua = su[la];
  T G[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) G[i][k] = T(0);
  ell_walk<LPP>(g.ell, td.ell_off, g.tmax, t, h, nb4, [&](uint32_t l) {
    const vec4<T> xb = sx[l], ub = su[l];
    T d[3] = {xa.x - xb.x, xa.y - xb.y, xa.z - xb.z};
    T du[3] = {ub.x - ua.x, ub.y - ua.y, ub.z - ua.z};
    T r2 = d[0] * d[0] + d[1] * d[1];
    if (D == 3) r2 += d[2] * d[2];
    const T w = dw_over_r(r2, g.inv_h, g.c5) * xb.w;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const T wd = w * du[i];
#pragma unroll
      for (int k = 0; k < D; ++k) G[i][k] += wd * d[k];
    }
  });
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) G[i][k] = lane_sum<LPP>(G[i][k]);
  if (h != 0) return;
  T Hm[9] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
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
      Hm[i * 3 + k] = acc;
    }
  if (rec_H) {
    T* r = HONLY ? rec_H : rec_H + ctrl->k * D * D * n;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int k = 0; k < D; ++k) r[(i * D + k) * n + a] = Hm[i * 3 + k];
  }
  if constexpr (HONLY) return;
  T pl[7];
  if (model_is<MODEL>(m, SPH_MODEL_J2)) {
#pragma unroll
    for (int i = 0; i < 7; ++i) pl[i] = plastic[i * n + a];
    if (rec_pl) {
      T* r = rec_pl + ctrl->k * 7 * n;
#pragma unroll
      for (int i = 0; i < 7; ++i) r[i * n + a] = pl[i];
    }
  }
  T P[9];
  MatP<T> mm = m;
  if (bt.spec) {
    const int sp = bt.spec[a];
    mm.mu = bt.get<T>(BT_MU, sp);
    mm.K = bt.get<T>(BT_K, sp);
    mm.lam = bt.get<T>(BT_LAM, sp);
  }
  int st = constitutive<T, MODEL>(mm, Hm, pl, p ? p[a] : T(0), P);
  if (st) atomicOr(&ctrl->status, st);
  if (model_is<MODEL>(m, SPH_MODEL_J2)) {
#pragma unroll
    for (int i = 0; i < 7; ++i) plastic[i * n + a] = pl[i];
  }
  T Pb[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < D; ++l) acc += P[i * 3 + l] * B[l][k];
      Pb[i][k] = acc;
    }
  if (mx.c) {
    // the fluid's momentum flux as a Piola tensor: PB -= rho_l0 v^l (x) (B^T Q),
    // with the fluid velocity v^l = v + F Q / c (no relative part where c <= 0)
    const T ca = mx.c[a];
    T Q[D], vl[D], BQ[D];
#pragma unroll
    for (int i = 0; i < D; ++i) Q[i] = mx.q[i * n + a];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      vl[i] = mx.v[i * n + a];
      if (ca > T(0)) {
        T fq = Q[i];
#pragma unroll
        for (int k = 0; k < D; ++k) fq += Hm[i * 3 + k] * Q[k];
        vl[i] += fq / ca;
      }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < D; ++l) acc += Q[l] * B[l][k];
      BQ[k] = acc;
    }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int k = 0; k < D; ++k) Pb[i][k] -= mx.rho_l0 * vl[i] * BQ[k];
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) PB[(i * D + k) * n + a] = Pb[i][k];
}

// momentum: a = (1/rho0) sum_b V_b (PB_a + PB_b) grad_a W_ab; kick v += dt a.
// Summed as PB_a g_a + sum_b (V_b PB_b) grad_a W_ab, with the kernel-gradient
// sum g_a = sum_b V_b grad_a W_ab of the reference configuration taken from
// the build: the window holds the relative position and V_b PB_b, twelve
// values in 3D, and the pair loop needs no neighbour volume.
template <typename T, int D, int LPP>
__global__ __launch_bounds__(256 * LPP) void k_momentum(TileGeo<T> g,
                                                                 const T* __restrict__ PB,
                                                                 T* __restrict__ v,
                                                                 T* __restrict__ acc_out,
                                                                 const uint8_t* __restrict__ flags,
                                                                 T inv_rho0, T dt, Ctrl* ctrl,
                                                                 bool gated, Bat bt, Mix<T> mx) {
  if (gated && ctrl->done) return;
  const int64_t tile = xcd_tile(g.n_tiles);
  if (tile >= g.n_tiles) return;
  using PK = Pk<T, D + D * D>;  // (relative position, V_b PB_b)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileDesc& td = g.tiles[tile];
  const uint32_t window = td.window;
  const int64_t n = g.n;
  const int64_t p0 = td.p0;
  double xo[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < D; ++k) xo[k] = g.X[k * n + p0];
  const WinMap wm = win_map(td);
  for (uint32_t l0 = threadIdx.x; l0 < window; l0 += 2 * blockDim.x) {
    T vv[2][D + D * D];
    uint32_t ls[2] = {l0, l0 + blockDim.x};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (ls[e] < window) {
        const int64_t gi = wm(ls[e]);
#pragma unroll
        for (int k = 0; k < D; ++k) vv[e][k] = (T)(g.X[k * n + gi] - xo[k]);
        const T Vb = g.V[gi];
#pragma unroll
        for (int c = 0; c < D * D; ++c) vv[e][D + c] = Vb * PB[c * n + gi];
      }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (ls[e] < window) PK::store(smem_raw, window, ls[e], vv[e]);
  }
  __syncthreads();
  const int t = threadIdx.x / LPP, h = threadIdx.x % LPP;
  if ((uint32_t)t >= td.count) return;
  uint32_t la, nb4;
  const int64_t a = tile_own(g.tslot, g.tmax, tile, td, (uint32_t)t, la, nb4);
  T xa[D + D * D];
  PK::load(smem_raw, window, la, xa);
  T f[3] = {T(0), T(0), T(0)};
  ell_walk<LPP>(g.ell, td.ell_off, g.tmax, t, h, nb4, [&](uint32_t l) {
    T xb[D + D * D];
    PK::load(smem_raw, window, l, xb);
    const T* Pb = xb + D;
    T d[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int k = 0; k < D; ++k) d[k] = xa[k] - xb[k];
    T r2 = d[0] * d[0] + d[1] * d[1];
    if (D == 3) r2 += d[2] * d[2];
    const T w = dw_over_r(r2, g.inv_h, g.c5);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      T s = T(0);
#pragma unroll
      for (int k = 0; k < D; ++k) s += Pb[i * D + k] * d[k];
      f[i] += w * s;
    }
  });
#pragma unroll
  for (int i = 0; i < D; ++i) f[i] = lane_sum<LPP>(f[i]);
  if (h != 0) return;
  // the own term PB_a g_a
  T ga[D];
#pragma unroll
  for (int k = 0; k < D; ++k) ga[k] = g.gsum[k * n + a];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) f[i] += PB[(i * D + k) * n + a] * ga[k];
  const bool fixed = flags && (flags[a] & SPH_FLAG_FIXED);
  const T dta = bt.spec ? bt.get<T>(BT_DT, bt.spec[a]) : dt;
  // the inertia of the mixture: rho0 + rho_l0 c per reference volume
  const T rho_a = mx.c ? mx.rho0 + mx.rho_l0 * mx.c[a] : T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T ai = mx.c ? f[i] / rho_a : f[i] * inv_rho0;
    if (acc_out) acc_out[i * n + a] = ai;
    if (!fixed) v[i * n + a] += dta * ai;
  }
}

// damping: anchors of one colour, 64 / G anchors per wavefront (one
// workgroup), G lanes per anchor while staging.  The implicit update of one
// pair, with inverse masses i_a, i_b (zero for a fixed particle, which then
// acts as infinite mass) and beta = eta dt g_ab <= 0, g_ab = 2 V_a V_b (dW/dr)/r:
//   v_ab' = v_ab / (1 - beta (i_a + i_b)),  v_a += beta i_a v_ab',  v_b -= beta i_b v_ab',
// i.e. v_a += i_a q (v_a - v_b), v_b -= i_b q (v_a - v_b) with
// q = beta / (1 - beta (i_a + i_b)), precomputed per run with i_a, i_b.
//
// Each anchor's 2^d-cell block lives in LDS as one 4-vector per particle
// (velocity, inverse mass), and a spare zero slot after it.  The wavefront
// runs the joint rows of its anchors (build_joint_rows): a row holds up to 64
// pairs, from one level of each anchor at most, one pair per lane; its pairs
// share no particle, the rows run in order.  A lane without a pair in a row
// updates the first group's spare slot with q = 0 (no change), so the row
// body has no branch, and only the velocity is written back.  Row words and
// (pair word, q) records stream from memory through two register rings (the
// row word 2K steps ahead, the record K steps ahead), so the serial row loop
// has one LDS round trip per row and the LDS holds only the blocks: many
// wavefronts share a CU.  Each wavefront's row list is framed by empty rows,
// so the ring reads need no bounds tests; a record is addressed by a 32-bit
// offset from the colour's first pair, and a pair word holds the two
// particles' LDS byte offsets in the wavefront's blocks.  One wavefront: its
// LDS accesses complete in issue order, so a row reads what the previous row
// wrote without a barrier.  The blocks are written back at the end; anchors
// of one colour touch disjoint blocks.
//
// SKIP: lanes without a pair skip the row's LDS work instead (a branch, but
// no LDS traffic for them); which is faster depends on how many wavefronts
// share the CUs.
//
// REV: the transposed sweep used by the reverse pass: rows in reverse order
// and the transposed pair map  s = q (i_a w_a - i_b w_b),  w_a += s,  w_b -= s.
constexpr uint32_t kNoPair = 0xFFFFFFFFu;  // the record after the last pair holds (kNoPair, 0)

template <typename T, int D, int G, bool REV, bool SKIP>
__global__ __launch_bounds__(64) void k_damp(const PairQ<T>* __restrict__ dwq_c, uint32_t sent,
                                             const T* __restrict__ imass,
                                             const uint32_t* __restrict__ rows,
                                             const int64_t* __restrict__ rbase,
                                             const uint32_t* __restrict__ wave_blk,
                                             const uint32_t* __restrict__ wave_rec, int64_t w0,
                                             int bmax, int64_t n, T* v, Ctrl* ctrl, bool gated) {
  if (gated && ctrl->done) return;
  constexpr int APW = 64 / G;
  constexpr int K = 8;  // steps of records in flight (deeper rings measured slower)
  // the last pass of the step loop runs up to K - 1 steps past the list and
  // reads row words 2K steps ahead: every row read stays within the frames
  static_assert(3 * K <= kDampRowPad, "row frames too short for the ring");
  constexpr int SB = 8;  // block particles per lane in flight while staging
  constexpr uint32_t S4 = sizeof(vec4<T>);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int grp = threadIdx.x / G, lg = threadIdx.x % G;
  const uint32_t lane = threadIdx.x;
  // group g's block at byte g * per; slot bmax of group 0 serves the idle lanes
  const size_t per = ((size_t)bmax + 1) * S4;
  const uint32_t idle_w = ((uint32_t)bmax * S4) | (((uint32_t)bmax * S4) << 16);
  vec4<T>* sv = reinterpret_cast<vec4<T>*>(smem_raw + grp * per);
  const int64_t wv = w0 + blockIdx.x;
  const uint32_t lo_rel = wave_rec[wv];
  const int64_t rb = rbase[wv];
  const int nrw = (int)(rbase[wv + 1] - rb) - 2 * kDampRowPad;  // the same for all lanes
  const uint32_t* rp = rows + rb + kDampRowPad + (REV ? nrw - 1 : 0);
  // this group's anchor block: four runs (begin, count) of sorted particles
  // (all counts zero when the wavefront has no anchor for the group)
  const uint32_t* bl = wave_blk + (wv * APW + grp) * 8;
  const uint32_t b0 = bl[0], b2 = bl[2], b4 = bl[4], b6 = bl[6];
  const uint32_t e0 = bl[1], e1 = e0 + bl[3], e2 = e1 + bl[5], nblk = e2 + bl[7];
  auto row = [&](const uint32_t* p, int k) -> uint32_t { return REV ? p[-k] : p[k]; };
  // this lane's record in a row (the sentinel when the lane has no pair there)
  const unsigned char* dwqb = reinterpret_cast<const unsigned char*>(dwq_c);
  auto rec = [&](uint32_t rw) -> PairQ<T> {
    const uint32_t i = (rw & 0xFFFFu) + lane;
    const uint32_t idx = i < (rw >> 16) ? lo_rel + i : sent;
    return *reinterpret_cast<const PairQ<T>*>(dwqb + (size_t)(idx * (uint32_t)sizeof(PairQ<T>)));
  };
  uint32_t rwr[K];
  PairQ<T> ring[K];
  {
    uint32_t rw0[K];
#pragma unroll
    for (int k = 0; k < K; ++k) rw0[k] = row(rp, k);
#pragma unroll
    for (int k = 0; k < K; ++k) rwr[k] = row(rp, K + k);
#pragma unroll
    for (int k = 0; k < K; ++k) ring[k] = rec(rw0[k]);
  }
  auto gidx = [&](uint32_t l) -> int64_t {
    return l < e0 ? (int64_t)b0 + l
                  : (l < e1 ? (int64_t)b2 + (l - e0)
                            : (l < e2 ? (int64_t)b4 + (l - e1) : (int64_t)b6 + (l - e2)));
  };
  // stage the block (loads clamped to valid entries)
  for (uint32_t l0 = lg; l0 < nblk; l0 += SB * G) {
    vec4<T> x[SB];
#pragma unroll
    for (int e = 0; e < SB; ++e) {
      const uint32_t l = l0 + e * G;
      const int64_t gi = gidx(l < nblk ? l : l0);
      x[e].x = v[gi];
      x[e].y = v[n + gi];
      x[e].z = D == 3 ? v[2 * n + gi] : T(0);
      x[e].w = imass[gi];
    }
#pragma unroll
    for (int e = 0; e < SB; ++e)
      if (l0 + e * G < nblk) sv[l0 + e * G] = x[e];
  }
  if (lg == 0) sv[bmax] = vec4<T>{T(0), T(0), T(0), T(0)};
  __syncthreads();
  for (int t0 = 0; t0 < nrw; t0 += K) {
    const uint32_t* pi = REV ? rp - t0 : rp + t0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const PairQ<T> pq = ring[k];
      const uint32_t w = SKIP ? pq.w : (pq.w == kNoPair ? idle_w : pq.w);
      if (!SKIP || w != kNoPair) {
        vec4<T>* pa = reinterpret_cast<vec4<T>*>(smem_raw + (w & 0xFFFFu));
        vec4<T>* pb = reinterpret_cast<vec4<T>*>(smem_raw + (w >> 16));
        vec4<T> va = *pa, vb = *pb;
        const T ka = va.w * pq.q, kb = vb.w * pq.q;
        if constexpr (!REV) {
          const T dx = va.x - vb.x, dy = va.y - vb.y, dz = va.z - vb.z;
          va.x += ka * dx;
          va.y += ka * dy;
          va.z += ka * dz;
          vb.x -= kb * dx;
          vb.y -= kb * dy;
          vb.z -= kb * dz;
        } else {
          const T sx = ka * va.x - kb * vb.x, sy = ka * va.y - kb * vb.y,
                  sz = ka * va.z - kb * vb.z;
          va.x += sx;
          va.y += sy;
          va.z += sz;
          vb.x -= sx;
          vb.y -= sy;
          vb.z -= sz;
        }
        // the inverse mass (w) stays as staged
        struct V3 { T x, y, z; };
        *reinterpret_cast<V3*>(pa) = V3{va.x, va.y, va.z};
        *reinterpret_cast<V3*>(pb) = V3{vb.x, vb.y, vb.z};
      }
      // refill after the record's last use, into the same registers (a
      // copy would have to wait for the load); rwr[k] holds the row word of
      // step t0 + k + K
      ring[k] = rec(rwr[k]);
      rwr[k] = row(pi, k + 2 * K);
    }
  }
  __syncthreads();
  for (uint32_t l = lg; l < nblk; l += G) {
    const int64_t gi = gidx(l);
    const vec4<T> x = sv[l];
    v[gi] = x.x;
    v[n + gi] = x.y;
    if (D == 3) v[2 * n + gi] = x.z;
  }
}

// Per-run damping records: the pair word (the two particles' LDS byte
// offsets in their wavefront's blocks) and q, at the pair's position in the
// joint rows of its colour's lane-group width.  q and the inverse masses
// depend only on eta dt, rho0, the volumes and the flags, which a
// multi-time-step run holds fixed, so they are computed once per run (or per
// call of a lone sweep).
struct DampLayout {
  int64_t pair_off[9];                // first pair of each colour
  int32_t per[8];                     // LDS slots of one anchor: its colour's bmax + 1
  const uint32_t* jinfo[8];           // the colour's width's record position | group << 28
};

template <typename T>
__global__ void k_damp_prep(int64_t n_upairs, int64_t n, const uint32_t* __restrict__ sa,
                            const uint32_t* __restrict__ sb, const uint32_t* __restrict__ dpair,
                            const T* __restrict__ dgeo, const T* __restrict__ V,
                            const uint8_t* __restrict__ flags, T inv_rho0, T eta_dt, Bat bt,
                            DampLayout lay, PairQ<T>* __restrict__ dwq, T* __restrict__ imass,
                            Mix<T> mx) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  auto im = [&](int64_t a) -> T {
    const bool fixed = flags && (flags[a] & SPH_FLAG_FIXED);
    if (fixed) return T(0);
    return mx.c ? T(1) / ((mx.rho0 + mx.rho_l0 * mx.c[a]) * V[a]) : inv_rho0 / V[a];
  };
  if (i < n) imass[i] = im(i);
  if (i == n_upairs) {
    PairQ<T> none{};
    none.w = 0xFFFFFFFFu;
    dwq[i] = none;
  }
  if (i >= n_upairs) return;
  int c = 0;
  while (c < 7 && i >= lay.pair_off[c + 1]) ++c;
  const uint32_t inf = lay.jinfo[c][i];
  const uint32_t base = (inf >> 28) * (uint32_t)lay.per[c];
  const uint32_t a = sa[i], b = sb[i];
  const T edt = bt.spec ? bt.get<T>(BT_ETADT, bt.spec[a]) : eta_dt;
  const T beta = edt * dgeo[i];
  constexpr uint32_t S = sizeof(vec4<T>);
  const uint32_t w = dpair[i];
  PairQ<T> pq{};
  pq.w = ((base + (w & 0xFFFFu)) * S) | (((base + (w >> 16)) * S) << 16);
  pq.q = beta / (T(1) - beta * (im(a) + im(b)));
  dwq[inf & 0x0FFFFFFFu] = pq;
}

// The stop state after an inner step's kinetic energy ke: the step count, the
// early exit, the cap and the non-finite status (one thread).
__device__ __forceinline__ void ke_finish(Ctrl* ctrl, double ke, double* ke_out, bool gated) {
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

// drift + kinetic energy: every block writes its partial E_k (fixed-order
// tree), then the partials are reduced in a fixed order, E_k recorded and the
// stop state updated (deterministic: no floating-point atomics).  On a large
// grid a second kernel (k_ke_reduce) reduces them.  On a grid of at most
// kKeFinishBlocks blocks (FIN) the last block to finish, elected with a
// ticket, reduces them itself and saves that launch; its sum takes the same
// order as k_ke_reduce's, so E_k is the same bit for bit.  (On large grids
// the device-scope release fence every block then needs, an L2 write-back
// per block, costs more than the launch.)
template <typename T, int D, bool FIN>
__global__ __launch_bounds__(kKeThreads) void k_drift_ke(
    int64_t n, double* __restrict__ u, const T* __restrict__ v, const uint8_t* __restrict__ flags,
    const double* __restrict__ V, double rho0, double dt, Ctrl* ctrl, double* partial,
    bool gated, Bat bt, const T* __restrict__ cmix, double rho_l0, double* ke_out) {
  // a FIN grid: every block reads done before it takes its ticket, and the
  // last block, which may set it, takes the last ticket
  if (gated && ctrl->done) return;
  __shared__ double red[kKeThreads];
  const int64_t a0 = blockIdx.x * (int64_t)(kKeThreads * kKeItems) + threadIdx.x;
  // every load of the thread's particles first, then the updates
  double uo[kKeItems][D], Va[kKeItems], dta[kKeItems], ra[kKeItems];
  T vv[kKeItems][D];
  uint8_t fl[kKeItems];
#pragma unroll
  for (int it = 0; it < kKeItems; ++it) {
    const int64_t a = a0 + it * kKeThreads;
    fl[it] = SPH_FLAG_FIXED;
    Va[it] = 0.0;
    ra[it] = rho0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      vv[it][k] = T(0);
      uo[it][k] = 0.0;
    }
    if (a < n) {
      fl[it] = flags ? flags[a] : (uint8_t)0;
      Va[it] = V[a];
      if (cmix) ra[it] = rho0 + rho_l0 * (double)cmix[a];  // mixture mass
#pragma unroll
      for (int k = 0; k < D; ++k) {
        vv[it][k] = v[k * n + a];
        uo[it][k] = u[k * n + a];
      }
    }
  }
  if (bt.spec) {  // batched: each particle's own time step
#pragma unroll
    for (int it = 0; it < kKeItems; ++it) {
      const int64_t a = a0 + it * kKeThreads;
      dta[it] = a < n ? bt.get<double>(BT_DT, bt.spec[a]) : 0.0;
    }
  } else {
#pragma unroll
    for (int it = 0; it < kKeItems; ++it) dta[it] = dt;
  }
  double acc = 0.0;
#pragma unroll
  for (int it = 0; it < kKeItems; ++it) {
    const int64_t a = a0 + it * kKeThreads;
    if (a < n) {
      const bool fixed = fl[it] & SPH_FLAG_FIXED;
      double v2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double vk = (double)vv[it][k];
        if (!fixed) u[k * n + a] = uo[it][k] + dta[it] * vk;
        v2 += vk * vk;
      }
      acc += 0.5 * ra[it] * Va[it] * v2;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kKeThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if constexpr (!FIN) {
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
  } else {
    static_assert(kKeFinishBlocks <= kKeThreads, "one partial per thread of the last block");
    __shared__ bool last;
    if (threadIdx.x == 0) {
      __hip_atomic_store(&partial[blockIdx.x], red[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t t = __hip_atomic_fetch_add(&ctrl->ticket, 1u, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT);
      last = t == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    // the partials in k_ke_reduce's order: its 1024-slot tree over at most
    // kKeFinishBlocks values adds zeros until the slots below 64 remain
    const int nblk = (int)gridDim.x;
    red[threadIdx.x] = (int)threadIdx.x < nblk
                           ? __hip_atomic_load(&partial[threadIdx.x], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)
                           : 0.0;
    __syncthreads();
    for (int w = kKeThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      ctrl->ticket = 0u;
      ke_finish(ctrl, red[0], ke_out, gated);
    }
  }
}

__global__ __launch_bounds__(1024) void k_ke_reduce(const double* __restrict__ partial,
                                                    int nblk, Ctrl* ctrl, double* ke_out,
                                                    bool gated) {
  if (gated && ctrl->done) return;
  __shared__ double red[1024];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 1024) s += partial[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) ke_finish(ctrl, red[0], ke_out, gated);
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
__global__ void k_load(int64_t n, double* u, const T* vgrip, const uint8_t* flags, double dt, Bat bt) {
  int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n || !(flags[a] & SPH_FLAG_GRIP)) return;
  const double dta = bt.spec ? bt.get<double>(BT_DTD, bt.spec[a]) : dt;
#pragma unroll
  for (int k = 0; k < D; ++k) u[k * n + a] += dta * (double)vgrip[k * n + a];
}

template <typename T, int D>
__device__ __forceinline__ T det_d(const T* A) {
  if constexpr (D == 2) return A[0] * A[3] - A[1] * A[2];
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}
template <typename T, int D>
__device__ __forceinline__ void inv_d(const T* A, T det, T* Ai) {
  if constexpr (D == 2) {
    Ai[0] = A[3] / det;
    Ai[1] = -A[1] / det;
    Ai[2] = -A[2] / det;
    Ai[3] = A[0] / det;
  } else {
    Ai[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    Ai[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    Ai[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    Ai[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    Ai[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    Ai[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    Ai[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    Ai[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    Ai[8] = (A[0] * A[4] - A[1] * A[3]) / det;
  }
}

// The diffusion kernels work on the LDS tiles of the inner-step kernels: a
// tile stages its window (positions relative to the tile origin and volumes,
// plus one per-particle field), then LPP lanes per own particle walk its
// ELL list in LDS.  Padding entries of a list point at the particle itself
// (d = 0) and add nothing.

// Flux of one slow step.  Reference configuration (Fi == nullptr):
//   q = -D B0 sum_b V_b (f_b - f_a) grad0 W      (f = c, the saturation).
// Two-way coupled (Fi = F^-1, f = the saturation a = c / J): the gradient is
// taken in the current configuration, g = F^-T B0 sum_b V_b (a_b - a_a)
// grad0 W, the flux is q = -D w g with w = a (nonlinear) or 1, and what is
// stored is the reference (Piola) flux J F^-1 q.
template <typename T, int D, int LPP>
__global__ __launch_bounds__(256 * LPP) void k_diff_grad(TileGeo<T> g, const T* __restrict__ f,
                                                         const T* __restrict__ Fi,
                                                         T* __restrict__ q, T Dc, int nonlinear,
                                                         Bat bt) {
  const int64_t tile = xcd_tile(g.n_tiles);
  if (tile >= g.n_tiles) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileDesc& td = g.tiles[tile];
  const uint32_t window = td.window;
  vec4<T>* sx = reinterpret_cast<vec4<T>*>(smem_raw);
  T* sf = reinterpret_cast<T*>(sx + window);
  const int64_t n = g.n;
  const int64_t p0 = td.p0;
  double xo[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < D; ++k) xo[k] = g.X[k * n + p0];
  const WinMap wm = win_map(td);
  for (uint32_t l0 = threadIdx.x; l0 < window; l0 += 2 * blockDim.x) {
    vec4<T> xv[2];
    T fv[2];
    uint32_t ls[2] = {l0, l0 + blockDim.x};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (ls[e] < window) {
        const int64_t gi = wm(ls[e]);
        xv[e].x = (T)(g.X[gi] - xo[0]);
        xv[e].y = (T)(g.X[n + gi] - xo[1]);
        xv[e].z = D == 3 ? (T)(g.X[2 * n + gi] - xo[2]) : T(0);
        xv[e].w = g.V[gi];
        fv[e] = f[gi];
      }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (ls[e] < window) {
        sx[ls[e]] = xv[e];
        sf[ls[e]] = fv[e];
      }
  }
  __syncthreads();
  const int t = threadIdx.x / LPP, h = threadIdx.x % LPP;
  if ((uint32_t)t >= td.count) return;
  uint32_t la, nb4;
  const int64_t a = tile_own(g.tslot, g.tmax, tile, td, (uint32_t)t, la, nb4);
  const vec4<T> xa = sx[la];
  const T fa = sf[la];
  T s[D];
#pragma unroll
  for (int k = 0; k < D; ++k) s[k] = T(0);
  ell_walk<LPP>(g.ell, td.ell_off, g.tmax, t, h, nb4, [&](uint32_t l) {
    const vec4<T> xb = sx[l];
    T d[3] = {xa.x - xb.x, xa.y - xb.y, xa.z - xb.z};
    T r2 = d[0] * d[0] + d[1] * d[1];
    if (D == 3) r2 += d[2] * d[2];
    const T w = dw_over_r(r2, g.inv_h, g.c5) * xb.w * (sf[l] - fa);
#pragma unroll
    for (int k = 0; k < D; ++k) s[k] += w * d[k];
  });
#pragma unroll
  for (int k = 0; k < D; ++k) s[k] = lane_sum<LPP>(s[k]);
  if (h != 0) return;
  const T Da = bt.spec ? bt.get<T>(BT_D, bt.spec[a]) : Dc;
  T gr[D];
#pragma unroll
  for (int m = 0; m < D; ++m) {
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) acc += g.B0[(m * D + k) * n + a] * s[k];
    gr[m] = acc;
  }
  if (!Fi) {
#pragma unroll
    for (int m = 0; m < D; ++m) q[m * n + a] = -Da * gr[m];
    return;
  }
  T Fa[D * D];
#pragma unroll
  for (int i = 0; i < D * D; ++i) Fa[i] = Fi[i * n + a];
  const T J = T(1) / det_d<T, D>(Fa);
  T gc[D], qc[D];
#pragma unroll
  for (int m = 0; m < D; ++m) {
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) acc += Fa[k * D + m] * gr[k];  // F^-T
    gc[m] = acc;
  }
  const T wa = nonlinear ? fa : T(1);
#pragma unroll
  for (int m = 0; m < D; ++m) qc[m] = -Da * wa * gc[m];
#pragma unroll
  for (int m = 0; m < D; ++m) {
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) acc += Fa[m * D + k] * qc[k];  // F^-1
    q[m * n + a] = J * acc;
  }
}

// coupled diffusion, first pass: the deformation gradient F = I + H with
// H = (sum_b V_b (u_b - u_a) (x) grad0 W_ab) B0_a (eq. deformationtensor-
// displacement), kept as F^-1 in Fi [D*D][n], and the saturation c / det F
// in sat [n]
template <typename T, int D, int LPP>
__global__ __launch_bounds__(256 * LPP) void k_diff_F(TileGeo<T> g, const double* __restrict__ u,
                                                      const T* __restrict__ c, T* __restrict__ Fi,
                                                      T* __restrict__ sat) {
  const int64_t tile = xcd_tile(g.n_tiles);
  if (tile >= g.n_tiles) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileDesc& td = g.tiles[tile];
  const uint32_t window = td.window;
  vec4<T>* sx = reinterpret_cast<vec4<T>*>(smem_raw);
  vec4<T>* su = sx + window;
  const int64_t n = g.n;
  const int64_t p0 = td.p0;
  double xo[3] = {0, 0, 0}, uo[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < D; ++k) {
    xo[k] = g.X[k * n + p0];
    uo[k] = u[k * n + p0];
  }
  const WinMap wm = win_map(td);
  for (uint32_t l0 = threadIdx.x; l0 < window; l0 += 2 * blockDim.x) {
    vec4<T> xv[2], uv[2];
    uint32_t ls[2] = {l0, l0 + blockDim.x};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (ls[e] < window) {
        const int64_t gi = wm(ls[e]);
        xv[e].x = (T)(g.X[gi] - xo[0]);
        xv[e].y = (T)(g.X[n + gi] - xo[1]);
        xv[e].z = D == 3 ? (T)(g.X[2 * n + gi] - xo[2]) : T(0);
        xv[e].w = g.V[gi];
        uv[e].x = (T)(u[gi] - uo[0]);
        uv[e].y = (T)(u[n + gi] - uo[1]);
        uv[e].z = D == 3 ? (T)(u[2 * n + gi] - uo[2]) : T(0);
        uv[e].w = T(0);
      }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (ls[e] < window) {
        sx[ls[e]] = xv[e];
        su[ls[e]] = uv[e];
      }
  }
  __syncthreads();
  const int t = threadIdx.x / LPP, h = threadIdx.x % LPP;
  if ((uint32_t)t >= td.count) return;
  uint32_t la, nb4;
  const int64_t a = tile_own(g.tslot, g.tmax, tile, td, (uint32_t)t, la, nb4);
  const vec4<T> xa = sx[la], ua = su[la];
  T G[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) G[i][k] = T(0);
  ell_walk<LPP>(g.ell, td.ell_off, g.tmax, t, h, nb4, [&](uint32_t l) {
    const vec4<T> xb = sx[l], ub = su[l];
    T d[3] = {xa.x - xb.x, xa.y - xb.y, xa.z - xb.z};
    T du[3] = {ub.x - ua.x, ub.y - ua.y, ub.z - ua.z};
    T r2 = d[0] * d[0] + d[1] * d[1];
    if (D == 3) r2 += d[2] * d[2];
    const T w = dw_over_r(r2, g.inv_h, g.c5) * xb.w;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const T wd = w * du[i];
#pragma unroll
      for (int k = 0; k < D; ++k) G[i][k] += wd * d[k];
    }
  });
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) G[i][k] = lane_sum<LPP>(G[i][k]);
  if (h != 0) return;
  T F[D * D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < D; ++l) acc += G[i][l] * g.B0[(l * D + k) * n + a];
      F[i * D + k] = (i == k ? T(1) : T(0)) + acc;
    }
  const T J = det_d<T, D>(F);
  T Fin[D * D];
  inv_d<T, D>(F, J, Fin);
#pragma unroll
  for (int i = 0; i < D * D; ++i) Fi[i * n + a] = Fin[i];
  sat[a] = c[a] / J;
}

// c += dt (-sum_b V_b (B0_a q_a + B0_b q_b) . grad W); Dirichlet; p = C (c - c0).
// The window stages y_b = B0_b q_b; the own term is y_a . sum_b V_b grad W,
// once per lane.  With Fi (coupled), c is the content per reference volume:
// the Dirichlet value is c_bc J and p = C (c / J - c0).
template <typename T, int D, int LPP>
__global__ __launch_bounds__(256 * LPP) void k_diff_div(TileGeo<T> g, T* __restrict__ c,
                                                        const T* __restrict__ q, T* __restrict__ p,
                                                        const uint8_t* __restrict__ flags, T dt,
                                                        T c_bc, T Cs, T c0, Bat bt,
                                                        const T* __restrict__ Fi) {
  const int64_t tile = xcd_tile(g.n_tiles);
  if (tile >= g.n_tiles) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileDesc& td = g.tiles[tile];
  const uint32_t window = td.window;
  vec4<T>* sx = reinterpret_cast<vec4<T>*>(smem_raw);
  vec4<T>* sy = sx + window;
  const int64_t n = g.n;
  const int64_t p0 = td.p0;
  double xo[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < D; ++k) xo[k] = g.X[k * n + p0];
  const WinMap wm = win_map(td);
  for (uint32_t l0 = threadIdx.x; l0 < window; l0 += 2 * blockDim.x) {
    vec4<T> xv[2], yv[2];
    uint32_t ls[2] = {l0, l0 + blockDim.x};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (ls[e] < window) {
        const int64_t gi = wm(ls[e]);
        xv[e].x = (T)(g.X[gi] - xo[0]);
        xv[e].y = (T)(g.X[n + gi] - xo[1]);
        xv[e].z = D == 3 ? (T)(g.X[2 * n + gi] - xo[2]) : T(0);
        xv[e].w = g.V[gi];
        T qb[D], y[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int k = 0; k < D; ++k) qb[k] = q[k * n + gi];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          T acc = T(0);
#pragma unroll
          for (int k = 0; k < D; ++k) acc += g.B0[(i * D + k) * n + gi] * qb[k];
          y[i] = acc;
        }
        yv[e].x = y[0];
        yv[e].y = y[1];
        yv[e].z = y[2];
        yv[e].w = T(0);
      }
    }
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (ls[e] < window) {
        sx[ls[e]] = xv[e];
        sy[ls[e]] = yv[e];
      }
  }
  __syncthreads();
  const int t = threadIdx.x / LPP, h = threadIdx.x % LPP;
  if ((uint32_t)t >= td.count) return;
  uint32_t la, nb4;
  const int64_t a = tile_own(g.tslot, g.tmax, tile, td, (uint32_t)t, la, nb4);
  const vec4<T> xa = sx[la], ya = sy[la];
  T m[3] = {T(0), T(0), T(0)};
  T tb = T(0);
  ell_walk<LPP>(g.ell, td.ell_off, g.tmax, t, h, nb4, [&](uint32_t l) {
    const vec4<T> xb = sx[l], yb = sy[l];
    T d[3] = {xa.x - xb.x, xa.y - xb.y, xa.z - xb.z};
    T r2 = d[0] * d[0] + d[1] * d[1];
    if (D == 3) r2 += d[2] * d[2];
    const T w = dw_over_r(r2, g.inv_h, g.c5) * xb.w;
    T yd = yb.x * d[0] + yb.y * d[1];
    if (D == 3) yd += yb.z * d[2];
    tb += w * yd;
#pragma unroll
    for (int k = 0; k < D; ++k) m[k] += w * d[k];
  });
  T div = tb + ya.x * m[0] + ya.y * m[1];
  if (D == 3) div += ya.z * m[2];
  div = lane_sum<LPP>(div);
  if (h != 0) return;
  T cn = c[a] - (bt.spec ? bt.get<T>(BT_DTD, bt.spec[a]) : dt) * div;
  if (Fi) {
    T Fa[D * D];
#pragma unroll
    for (int i = 0; i < D * D; ++i) Fa[i] = Fi[i * n + a];
    const T J = T(1) / det_d<T, D>(Fa);
    if (flags && (flags[a] & SPH_FLAG_CDIR)) cn = c_bc * J;
    c[a] = cn;
    if (p) p[a] = Cs * (cn / J - c0);
    return;
  }
  if (flags && (flags[a] & SPH_FLAG_CDIR)) cn = c_bc;
  c[a] = cn;
  if (p) p[a] = Cs * (cn - c0);
}

// ---------------------------------------------------------------------------

int check_mixture(const sph_material* m, const sph_state* st) {
  if (!(m->rho_l0 >= 0.0)) {
    set_error("rho_l0 must be >= 0");
    return SPH_E_ARG;
  }
  if (m->rho_l0 > 0.0 && (!st->c || !st->q)) {
    set_error("a mixture (rho_l0 > 0) needs the state's content c and flux q");
    return SPH_E_ARG;
  }
  return SPH_OK;
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


template <typename T, int D, int LS, int LM, int MODEL>
static int solid_stage_l(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
                         hipStream_t s, bool gated) {
  const int prec = sizeof(T) == 8 ? SPH_F64 : SPH_F32;
  TileGeo<T> g = tile_geo<T>(nb, prec);
  if (g.n_tiles == 0) return SPH_OK;
  MatP<T> mp = matp<T>(m);
  const unsigned grid = (unsigned)(8 * ((g.n_tiles + 7) / 8));
  const size_t wm = (size_t)nb->tiling[prec].window_max;
  const size_t lds_s = wm * 2 * sizeof(vec4<T>);
  const size_t lds_m = wm * Pk<T, D + D * D>::bytes + 16;
  int rc = SPH_OK;
  if constexpr (LS > 0) {
    if ((rc = lds_attr(k_stress<T, D, LS, MODEL>, lds_s))) return rc;
    hipEvent_t pe_ = prof_begin(nb, SPH_KERNEL_STRESS, s);
    k_stress<T, D, LS, MODEL><<<grid, (unsigned)(g.tmax * LS), lds_s, s>>>(
        g, mp, st->u, (T*)st->PB, (T*)st->plastic, (const T*)st->p, nb->ctrl, gated,
        m->model == SPH_MODEL_J2 ? (T*)nb->rec_pl : nullptr, (T*)nb->rec_H, bat_view(nb),
        mix_view<T>(m, st));
    prof_end(nb, SPH_KERNEL_STRESS, pe_, s);
    SPH_LAUNCH_CHECK();
  }
  if constexpr (LM > 0) {
    if ((rc = lds_attr(k_momentum<T, D, LM>, lds_m))) return rc;
    hipEvent_t pe_ = prof_begin(nb, SPH_KERNEL_MOMENTUM, s);
    k_momentum<T, D, LM><<<grid, (unsigned)(g.tmax * LM), lds_m, s>>>(
        g, (const T*)st->PB, (T*)st->v, (T*)st->acc, st->flags, (T)(1.0 / m->rho0), (T)dt,
        nb->ctrl, gated, bat_view(nb), mix_view<T>(m, st));
    prof_end(nb, SPH_KERNEL_MOMENTUM, pe_, s);
    SPH_LAUNCH_CHECK();
  }
  return SPH_OK;
}

// lanes per particle of the two tiled kernels: the handle's tuned choice
// (sph_autotune), else the defaults
template <typename T, int D>
static int solid_stage_t(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
                         hipStream_t s, bool gated) {
  const int prec = sizeof(T) == 8 ? SPH_F64 : SPH_F32;
  const int ls = nb->tune.lpp[TUNE_STRESS][prec], lm = nb->tune.lpp[TUNE_MOMENTUM][prec];
  int rc;
  auto stress = [&](auto model_c) -> int {
    constexpr int M = decltype(model_c)::value;
    switch (ls) {
      case 1: return solid_stage_l<T, D, 1, 0, M>(nb, m, st, dt, s, gated);
      case 4: return solid_stage_l<T, D, 4, 0, M>(nb, m, st, dt, s, gated);
      default: return solid_stage_l<T, D, 2, 0, M>(nb, m, st, dt, s, gated);
    }
  };
  switch (m->model) {
    case SPH_MODEL_LE: rc = stress(std::integral_constant<int, SPH_MODEL_LE>{}); break;
    case SPH_MODEL_NH: rc = stress(std::integral_constant<int, SPH_MODEL_NH>{}); break;
    default: rc = stress(std::integral_constant<int, SPH_MODEL_J2>{}); break;
  }
  if (rc) return rc;
  switch (lm) {
    case 2: return solid_stage_l<T, D, 0, 2, -1>(nb, m, st, dt, s, gated);
    case 1: return solid_stage_l<T, D, 0, 1, -1>(nb, m, st, dt, s, gated);
    default: return solid_stage_l<T, D, 0, 4, -1>(nb, m, st, dt, s, gated);
  }
}

// H = F - I of st->u into H [D*D][n] (the stress stage's gather alone)
template <typename T, int D>
static int displacement_gradient_t(const sph_nbr* nb, const sph_state* st, void* H, hipStream_t s) {
  const int prec = sizeof(T) == 8 ? SPH_F64 : SPH_F32;
  TileGeo<T> g = tile_geo<T>(nb, prec);
  if (g.n_tiles == 0) return SPH_OK;
  const unsigned grid = (unsigned)(8 * ((g.n_tiles + 7) / 8));
  const size_t lds_s = (size_t)nb->tiling[prec].window_max * 2 * sizeof(vec4<T>);
  constexpr int L = 2;
  auto kern = k_stress<T, D, L, SPH_MODEL_LE, true>;
  int rc = lds_attr(kern, lds_s);
  if (rc) return rc;
  kern<<<grid, (unsigned)(g.tmax * L), lds_s, s>>>(g, MatP<T>{}, st->u, nullptr, nullptr, nullptr,
                                                   nb->ctrl, false, nullptr, (T*)H, bat_view(nb),
                                                   Mix<T>{});
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

int displacement_gradient(const sph_nbr* nb, const sph_state* st, void* H, hipStream_t s) {
  if (st->prec == SPH_F64)
    return nb->dim == 2 ? displacement_gradient_t<double, 2>(nb, st, H, s)
                        : displacement_gradient_t<double, 3>(nb, st, H, s);
  return nb->dim == 2 ? displacement_gradient_t<float, 2>(nb, st, H, s)
                      : displacement_gradient_t<float, 3>(nb, st, H, s);
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

template <int G>
constexpr int damp_width_index() {
  return G == 8 ? 0 : (G == 16 ? 1 : (G == 32 ? 2 : 3));
}

template <typename T>
static size_t damp_lds_per_anchor(const sph_nbr* nb, int col) {
  const size_t bmax = (size_t)std::max<int64_t>(nb->damp_bmax[col], 1);
  return (bmax + 1) * sizeof(vec4<T>);  // the block and its spare slot
}

// Lane-group width of a colour pass: the tuned width (sph_autotune), else 16;
// widened while the wavefront's blocks would exceed the LDS budget or the
// 16-bit byte offsets of the pair words, or its joint rows are unusable.
template <typename T>
static int damp_width(const sph_nbr* nb, int col) {
  const int prec = sizeof(T) == 8 ? SPH_F64 : SPH_F32;
  int G = nb->tune.damp_g[prec][col];
  if (G == 0) G = 16;
  const size_t per = damp_lds_per_anchor<T>(nb, col);
  auto fits = [&](int g) {
    const int gi = g == 8 ? 0 : (g == 16 ? 1 : (g == 32 ? 2 : 3));
    const size_t lds = (size_t)(64 / g) * per;
    return nb->dwidth_ok[gi] && lds <= (size_t)kDampLdsBudget && lds <= 65536;
  };
  while (G < 64 && !fits(G)) G *= 2;
  return G;
}

// automatic idle-lane mode: skip from this many wavefronts a pass up (the 1M
// plate's passes have 2304 at 16 lanes per anchor and run 5-8% faster
// skipping; the 40k-particle bar's 160 run 13% slower)
constexpr int64_t kDampSkipWaves = 512;

template <typename T, int D, int G, bool REV>
static int damp_launch(const sph_nbr* nb, const sph_state* st, hipStream_t s, bool gated,
                       int col) {
  constexpr int APW = 64 / G, gi = damp_width_index<G>();
  const int64_t w0 = nb->dwave_off[gi][col], w1 = nb->dwave_off[gi][col + 1];
  if (w1 <= w0) return SPH_OK;
  const int bmax = (int)std::max<int64_t>(nb->damp_bmax[col], 1);
  const size_t lds = APW * damp_lds_per_anchor<T>(nb, col);
  const int p = sizeof(T) == 8 ? SPH_F64 : SPH_F32;
  const int idle = nb->tune.damp_idle[p][col];
  const bool skip = idle == 2 || (idle == 0 && w1 - w0 >= kDampSkipWaves);
  auto kern = skip ? k_damp<T, D, G, REV, true> : k_damp<T, D, G, REV, false>;
  int rc = lds_attr(kern, lds);
  if (rc) return rc;
  const int64_t po = nb->damp_pair_off[col];
  kern<<<(unsigned)(w1 - w0), 64, lds, s>>>(
      (const PairQ<T>*)nb->dwq[p] + po, (uint32_t)(nb->n_upairs - po), (const T*)nb->imass[p],
      nb->drow[gi], nb->drow_base[gi], nb->dwave[gi], nb->dwrec[gi], w0, bmax, nb->n,
      (T*)st->v, nb->ctrl, gated);
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

template <typename T>
static int damp_prepare_t(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                          double eta, double dt, hipStream_t s) {
  // records hold 32-bit byte offsets from a colour's first pair
  if ((nb->n_upairs + 1) * (int64_t)sizeof(PairQ<T>) > (int64_t)0xFFFFFFFF) {
    set_error("damping sweep: %lld pairs exceed its addressing", (long long)nb->n_upairs);
    return SPH_E_CAPACITY;
  }
  const int p = sizeof(T) == 8 ? SPH_F64 : SPH_F32;
  DampLayout lay{};
  for (int c = 0; c < 9; ++c) lay.pair_off[c] = nb->damp_pair_off[c];
  for (int c = 0; c < 8; ++c) {
    const int G = damp_width<T>(nb, c);
    const int gi = G == 8 ? 0 : (G == 16 ? 1 : (G == 32 ? 2 : 3));
    if (64 / G * damp_lds_per_anchor<T>(nb, c) > 65536) {
      set_error("damping sweep: an anchor block of %lld particles exceeds its LDS addressing",
                (long long)nb->damp_bmax[c]);
      return SPH_E_CAPACITY;
    }
    lay.per[c] = (int32_t)std::max<int64_t>(nb->damp_bmax[c], 1) + 1;
    lay.jinfo[c] = nb->djinfo[gi];
    nb->damp_g_used[p][c] = G;
  }
  Geo<T> g = geo<T>(nb);
  const T* dgeo = reinterpret_cast<const T*>(sizeof(T) == 8 ? (const void*)nb->dgeo64
                                                           : (const void*)nb->dgeo32);
  const int64_t m_ = std::max<int64_t>(nb->n_upairs + 1, nb->n);
  k_damp_prep<T><<<nblk(std::max<int64_t>(m_, 1), 256), 256, 0, s>>>(
      nb->n_upairs, nb->n, nb->sa, nb->sb, nb->dpair, dgeo, g.V, st->flags, (T)(1.0 / m->rho0),
      (T)(eta * dt), bat_view(nb), lay, (PairQ<T>*)nb->dwq[p], (T*)nb->imass[p],
      mix_view<T>(m, st));
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

// One sweep, colour after colour, each pass with its colour's width.  The
// per-run records are laid out for the widths in force when they were made;
// outside a run, or when a width has changed since, they are made first.
template <typename T, int D, bool REV>
static int damping_t(const sph_nbr* nb, const sph_material* m, const sph_state* st, double eta,
                     double dt, hipStream_t s, bool gated) {
  int rc;
  const int ncol = 1 << D;
  const int prec = sizeof(T) == 8 ? SPH_F64 : SPH_F32;
  bool stale = !nb->damp_pre;
  for (int c = 0; c < ncol && !stale; ++c) stale = nb->damp_g_used[prec][c] != damp_width<T>(nb, c);
  if (stale && (rc = damp_prepare_t<T>(nb, m, st, eta, dt, s))) return rc;
  // timed per sweep: one event pair around its colour passes, which share
  // the sweep's time (an event pair per pass adds its queue time to each)
  const int kind = REV ? SPH_KERNEL_ADJ_DAMPING : SPH_KERNEL_DAMPING;
  hipEvent_t pe_ = prof_begin(nb, kind, s);
  int passes = 0;
  for (int c_ = 0; c_ < ncol; ++c_) {
    const int col = REV ? ncol - 1 - c_ : c_;
    if (nb->color_off[col + 1] <= nb->color_off[col]) continue;
    switch (nb->damp_g_used[prec][col]) {
      case 8: rc = damp_launch<T, D, 8, REV>(nb, st, s, gated, col); break;
      case 16: rc = damp_launch<T, D, 16, REV>(nb, st, s, gated, col); break;
      case 32: rc = damp_launch<T, D, 32, REV>(nb, st, s, gated, col); break;
      default: rc = damp_launch<T, D, 64, REV>(nb, st, s, gated, col); break;
    }
    if (rc) {
      prof_end(nb, kind, pe_, s, passes);
      return rc;
    }
    ++passes;
  }
  prof_end(nb, kind, pe_, s, passes);
  return SPH_OK;
}

template <typename T, int D>
static int damping_pass_t(const sph_nbr* nb, const sph_state* st, int col, hipStream_t s) {
  const int prec = sizeof(T) == 8 ? SPH_F64 : SPH_F32;
  switch (nb->damp_g_used[prec][col]) {
    case 8: return damp_launch<T, D, 8, false>(nb, st, s, false, col);
    case 16: return damp_launch<T, D, 16, false>(nb, st, s, false, col);
    case 32: return damp_launch<T, D, 32, false>(nb, st, s, false, col);
    default: return damp_launch<T, D, 64, false>(nb, st, s, false, col);
  }
}

int damping_pass(const sph_nbr* nb, const sph_state* st, int col, hipStream_t s) {
  if (st->prec == SPH_F64)
    return nb->dim == 2 ? damping_pass_t<double, 2>(nb, st, col, s)
                        : damping_pass_t<double, 3>(nb, st, col, s);
  return nb->dim == 2 ? damping_pass_t<float, 2>(nb, st, col, s)
                      : damping_pass_t<float, 3>(nb, st, col, s);
}

int damping_sweep(const sph_nbr* nb, const sph_material* m, const sph_state* st, double eta,
                  double dt, hipStream_t s, bool gated) {
  if (st->prec == SPH_F64)
    return nb->dim == 2 ? damping_t<double, 2, false>(nb, m, st, eta, dt, s, gated)
                        : damping_t<double, 3, false>(nb, m, st, eta, dt, s, gated);
  return nb->dim == 2 ? damping_t<float, 2, false>(nb, m, st, eta, dt, s, gated)
                      : damping_t<float, 3, false>(nb, m, st, eta, dt, s, gated);
}

int damp_prepare(const sph_nbr* nb, const sph_material* m, const sph_state* st, double eta,
                 double dt, hipStream_t s) {
  const int rc = st->prec == SPH_F64 ? damp_prepare_t<double>(nb, m, st, eta, dt, s)
                                     : damp_prepare_t<float>(nb, m, st, eta, dt, s);
  if (rc == SPH_OK) nb->damp_pre = true;
  return rc;
}

int damping_sweep_rev(const sph_nbr* nb, const sph_material* m, const sph_state* st, double eta,
                      double dt, hipStream_t s) {
  if (st->prec == SPH_F64)
    return nb->dim == 2 ? damping_t<double, 2, true>(nb, m, st, eta, dt, s, false)
                        : damping_t<double, 3, true>(nb, m, st, eta, dt, s, false);
  return nb->dim == 2 ? damping_t<float, 2, true>(nb, m, st, eta, dt, s, false)
                      : damping_t<float, 3, true>(nb, m, st, eta, dt, s, false);
}

template <typename T, int D>
static int drift_t(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
                   double* ke_out, hipStream_t s, bool gated, double* partial, int64_t max_blocks,
                   bool timed) {
  const int64_t per = (int64_t)kKeThreads * kKeItems;
  const int64_t nb_ = std::max<int64_t>(1, (nb->n + per - 1) / per);
  if (nb_ > max_blocks) {
    set_error("too many particles for the kinetic-energy partials (%lld > %lld)",
              (long long)nb->n, (long long)(max_blocks * per));
    return SPH_E_CAPACITY;
  }
  {
    hipEvent_t pe_ = timed ? prof_begin(nb, SPH_KERNEL_DRIFT_KE, s) : nullptr;
    if (nb_ <= kKeFinishBlocks) {
      k_drift_ke<T, D, true><<<(unsigned)nb_, kKeThreads, 0, s>>>(
          nb->n, st->u, (const T*)st->v, st->flags, nb->V, m->rho0, dt, nb->ctrl, partial, gated,
          bat_view(nb), mix_view<T>(m, st).c, m->rho_l0, ke_out);
    } else {
      k_drift_ke<T, D, false><<<(unsigned)nb_, kKeThreads, 0, s>>>(
          nb->n, st->u, (const T*)st->v, st->flags, nb->V, m->rho0, dt, nb->ctrl, partial, gated,
          bat_view(nb), mix_view<T>(m, st).c, m->rho_l0, nullptr);
      SPH_LAUNCH_CHECK();
      k_ke_reduce<<<1, 1024, 0, s>>>(partial, (int)nb_, nb->ctrl, ke_out, gated);
    }
    if (timed) prof_end(nb, SPH_KERNEL_DRIFT_KE, pe_, s);
  }
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

static int drift_dispatch(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
                          double* ke_out, hipStream_t s, bool gated, double* partial,
                          int64_t max_blocks, bool timed) {
  if (st->prec == SPH_F64)
    return nb->dim == 2
               ? drift_t<double, 2>(nb, m, st, dt, ke_out, s, gated, partial, max_blocks, timed)
               : drift_t<double, 3>(nb, m, st, dt, ke_out, s, gated, partial, max_blocks, timed);
  return nb->dim == 2
             ? drift_t<float, 2>(nb, m, st, dt, ke_out, s, gated, partial, max_blocks, timed)
             : drift_t<float, 3>(nb, m, st, dt, ke_out, s, gated, partial, max_blocks, timed);
}

int drift_ke(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
             double* ke_out, hipStream_t s, bool gated) {
  return drift_dispatch(nb, m, st, dt, ke_out, s, gated, nb->ke_partial, kKeMaxBlocks, true);
}

// ---- drift + kinetic energy with the partials in a static device array -------
// The block partials of the kinetic-energy reduction sit in `scratch`, one
// copy per GPU that loads the library (kept until the process ends).  In host
// code `scratch` names a host-side stand-in, not the device copy: its device
// address is taken once per device with hipGetSymbolAddress and only that
// address reaches the kernels.  Every block writes its own partial and the
// reducer reads exactly the blocks of the launch, so nothing needs clearing
// between calls; two calls that overlap in time on one GPU race on it.
static __device__ __align__(256) double scratch[kStaticKeBlocks];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device

int scratch_address(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device ordinal %d out of range", device);
    return SPH_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
      return SPH_E_DEVICE;
    }
    g_scratch_dev[device] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[device];
  return SPH_OK;
}
}  // namespace

int drift_ke_static(const sph_nbr* nb, const sph_material* m, const sph_state* st, double dt,
                    double* ke_out, hipStream_t s) {
  int device = -1;
  SPH_HIP(hipGetDevice(&device));
  if (device != nb->device) {
    set_error("the current device (%d) is not the neighbourhood's (%d)", device, nb->device);
    return SPH_E_ARG;
  }
  double* partial = nullptr;
  const int rc = scratch_address(device, &partial);
  if (rc) return rc;
  return drift_dispatch(nb, m, st, dt, ke_out, s, false, partial, kStaticKeBlocks, false);
}

int reset_ctrl(const sph_nbr* nb, int64_t k_limit, double ke_tol, hipStream_t s) {
  k_reset_ctrl<<<1, 1, 0, s>>>(nb->ctrl, k_limit, ke_tol);
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

int load_step(const sph_nbr* nb, const sph_state* st, double dt_l, hipStream_t s) {
  if (!st->vgrip || !st->flags) return SPH_OK;
  if (st->prec == SPH_F64) {
    if (nb->dim == 2) k_load<double, 2><<<nblk(nb->n, 256), 256, 0, s>>>(nb->n, st->u, (const double*)st->vgrip, st->flags, dt_l, bat_view(nb));
    else k_load<double, 3><<<nblk(nb->n, 256), 256, 0, s>>>(nb->n, st->u, (const double*)st->vgrip, st->flags, dt_l, bat_view(nb));
  } else {
    if (nb->dim == 2) k_load<float, 2><<<nblk(nb->n, 256), 256, 0, s>>>(nb->n, st->u, (const float*)st->vgrip, st->flags, dt_l, bat_view(nb));
    else k_load<float, 3><<<nblk(nb->n, 256), 256, 0, s>>>(nb->n, st->u, (const float*)st->vgrip, st->flags, dt_l, bat_view(nb));
  }
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

// lanes per particle of the tiled diffusion kernels
constexpr int kDiffLpp = 2;

template <typename T>
struct DiffLaunch {
  TileGeo<T> g;
  unsigned grid, block;
  size_t lds1, lds2;  // window of one vec4 + one scalar, of two vec4
};

template <typename T>
static DiffLaunch<T> diff_launch(const sph_nbr* nb) {
  const int prec = sizeof(T) == 8 ? SPH_F64 : SPH_F32;
  DiffLaunch<T> L;
  L.g = tile_geo<T>(nb, prec);
  L.grid = (unsigned)(8 * ((L.g.n_tiles + 7) / 8));
  L.block = (unsigned)(L.g.tmax * kDiffLpp);
  const size_t wm = (size_t)nb->tiling[prec].window_max;
  L.lds1 = wm * (sizeof(vec4<T>) + sizeof(T));
  L.lds2 = wm * 2 * sizeof(vec4<T>);
  return L;
}

template <typename T, int D>
static int diffusion_t(const sph_nbr* nb, const sph_material* m, const sph_state* st, double Dc,
                       double dt, double c_bc, hipStream_t s) {
  const DiffLaunch<T> L = diff_launch<T>(nb);
  if (L.g.n_tiles == 0) return SPH_OK;
  int rc;
  if ((rc = lds_attr(k_diff_grad<T, D, kDiffLpp>, L.lds1)) ||
      (rc = lds_attr(k_diff_div<T, D, kDiffLpp>, L.lds2)))
    return rc;
  {
    hipEvent_t pe_ = prof_begin(nb, SPH_KERNEL_DIFF_GRAD, s);
    k_diff_grad<T, D, kDiffLpp><<<L.grid, L.block, L.lds1, s>>>(
        L.g, (const T*)st->c, nullptr, (T*)st->q, (T)Dc, 0, bat_view(nb));
    prof_end(nb, SPH_KERNEL_DIFF_GRAD, pe_, s);
  }
  SPH_LAUNCH_CHECK();
  {
    hipEvent_t pe_ = prof_begin(nb, SPH_KERNEL_DIFF_DIV, s);
    k_diff_div<T, D, kDiffLpp><<<L.grid, L.block, L.lds2, s>>>(
        L.g, (T*)st->c, (const T*)st->q, (T*)st->p, st->flags, (T)dt, (T)c_bc, (T)m->C_swell,
        (T)m->c0, bat_view(nb), nullptr);
    prof_end(nb, SPH_KERNEL_DIFF_DIV, pe_, s);
  }
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

// two-way coupled form: deformation pass (F^-1 into the PB scratch, the
// saturation into p), flux, then the divergence with the J-aware epilogue
template <typename T, int D>
static int diffusion_coupled_t(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                               double Dc, double dt, double c_bc, int nonlinear, hipStream_t s) {
  const DiffLaunch<T> L = diff_launch<T>(nb);
  if (L.g.n_tiles == 0) return SPH_OK;
  int rc;
  if ((rc = lds_attr(k_diff_F<T, D, kDiffLpp>, L.lds2)) ||
      (rc = lds_attr(k_diff_grad<T, D, kDiffLpp>, L.lds1)) ||
      (rc = lds_attr(k_diff_div<T, D, kDiffLpp>, L.lds2)))
    return rc;
  T* Fi = (T*)st->PB;
  T* sat = (T*)st->p;
  {
    hipEvent_t pe_ = prof_begin(nb, SPH_KERNEL_DIFF_GRAD, s);
    k_diff_F<T, D, kDiffLpp><<<L.grid, L.block, L.lds2, s>>>(L.g, st->u, (const T*)st->c, Fi, sat);
    SPH_LAUNCH_CHECK();
    k_diff_grad<T, D, kDiffLpp><<<L.grid, L.block, L.lds1, s>>>(L.g, sat, Fi, (T*)st->q, (T)Dc,
                                                                nonlinear, bat_view(nb));
    prof_end(nb, SPH_KERNEL_DIFF_GRAD, pe_, s);
  }
  SPH_LAUNCH_CHECK();
  {
    hipEvent_t pe_ = prof_begin(nb, SPH_KERNEL_DIFF_DIV, s);
    k_diff_div<T, D, kDiffLpp><<<L.grid, L.block, L.lds2, s>>>(
        L.g, (T*)st->c, (const T*)st->q, (T*)st->p, st->flags, (T)dt, (T)c_bc, (T)m->C_swell,
        (T)m->c0, bat_view(nb), Fi);
    prof_end(nb, SPH_KERNEL_DIFF_DIV, pe_, s);
  }
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

// g_a = sum_b V_b grad_a W_ab of the reference configuration, computed once
// per precision with the tiled gathers' own arithmetic: positions relative to
// the tile's first particle rounded to T, the same kernel-gradient formula.
// The momentum sum and the reverse passes take their own-particle terms from
// it; computed this way it cancels against their pair sums as a per-pair
// evaluation would, where an exact g_a would leave a residual force of the
// positions' rounding on every particle (visible in FP32 on thin bodies).
template <typename T, int D, int LPP>
__global__ __launch_bounds__(256 * LPP) void k_gsum(TileGeo<T> g, T* __restrict__ gs) {
  const int64_t tile = xcd_tile(g.n_tiles);
  if (tile >= g.n_tiles) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileDesc& td = g.tiles[tile];
  const uint32_t window = td.window;
  vec4<T>* sx = reinterpret_cast<vec4<T>*>(smem_raw);
  const int64_t n = g.n;
  const int64_t p0 = td.p0;
  double xo[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < D; ++k) xo[k] = g.X[k * n + p0];
  const WinMap wm = win_map(td);
  for (uint32_t l = threadIdx.x; l < window; l += blockDim.x) {
    const int64_t gi = wm(l);
    vec4<T> xv;
    xv.x = (T)(g.X[gi] - xo[0]);
    xv.y = (T)(g.X[n + gi] - xo[1]);
    xv.z = D == 3 ? (T)(g.X[2 * n + gi] - xo[2]) : T(0);
    xv.w = g.V[gi];
    sx[l] = xv;
  }
  __syncthreads();
  const int t = threadIdx.x / LPP, h = threadIdx.x % LPP;
  if ((uint32_t)t >= td.count) return;
  uint32_t la, nb4;
  const int64_t a = tile_own(g.tslot, g.tmax, tile, td, (uint32_t)t, la, nb4);
  const vec4<T> xa = sx[la];
  T m[3] = {T(0), T(0), T(0)};
  ell_walk<LPP>(g.ell, td.ell_off, g.tmax, t, h, nb4, [&](uint32_t l) {
    const vec4<T> xb = sx[l];
    T d[3] = {xa.x - xb.x, xa.y - xb.y, xa.z - xb.z};
    T r2 = d[0] * d[0] + d[1] * d[1];
    if (D == 3) r2 += d[2] * d[2];
    const T w = dw_over_r(r2, g.inv_h, g.c5) * xb.w;
#pragma unroll
    for (int k = 0; k < D; ++k) m[k] += w * d[k];
  });
#pragma unroll
  for (int k = 0; k < D; ++k) m[k] = lane_sum<LPP>(m[k]);
  if (h != 0) return;
#pragma unroll
  for (int k = 0; k < D; ++k) gs[k * n + a] = m[k];
}

template <typename T, int D>
static int tile_gsum_t(const sph_nbr* nb, int prec, T* gs, hipStream_t s) {
  TileGeo<T> g = tile_geo<T>(nb, prec);
  if (g.n_tiles == 0) return SPH_OK;
  constexpr int L = 2;
  const size_t lds = (size_t)nb->tiling[prec].window_max * sizeof(vec4<T>);
  int rc = lds_attr(k_gsum<T, D, L>, lds);
  if (rc) return rc;
  const unsigned grid = (unsigned)(8 * ((g.n_tiles + 7) / 8));
  k_gsum<T, D, L><<<grid, (unsigned)(g.tmax * L), lds, s>>>(g, gs);
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

int tile_gsum(const sph_nbr* nb, hipStream_t s) {
  int rc = nb->dim == 2 ? tile_gsum_t<double, 2>(nb, SPH_F64, nb->gsum, s)
                        : tile_gsum_t<double, 3>(nb, SPH_F64, nb->gsum, s);
  if (rc) return rc;
  return nb->dim == 2 ? tile_gsum_t<float, 2>(nb, SPH_F32, nb->gsumf, s)
                      : tile_gsum_t<float, 3>(nb, SPH_F32, nb->gsumf, s);
}

// the deformation pass alone (F^-1 and the saturation c / J of a given u and
// c), for the reverse of the coupled step
template <typename T, int D>
static int diffusion_F_t(const sph_nbr* nb, const double* u, const void* c, void* Fi, void* sat,
                         hipStream_t s) {
  const DiffLaunch<T> L = diff_launch<T>(nb);
  if (L.g.n_tiles == 0) return SPH_OK;
  int rc;
  if ((rc = lds_attr(k_diff_F<T, D, kDiffLpp>, L.lds2))) return rc;
  k_diff_F<T, D, kDiffLpp><<<L.grid, L.block, L.lds2, s>>>(L.g, u, (const T*)c, (T*)Fi, (T*)sat);
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

int diffusion_F(const sph_nbr* nb, int prec, const double* u, const void* c, void* Fi, void* sat,
                hipStream_t s) {
  if (prec == SPH_F64)
    return nb->dim == 2 ? diffusion_F_t<double, 2>(nb, u, c, Fi, sat, s)
                        : diffusion_F_t<double, 3>(nb, u, c, Fi, sat, s);
  return nb->dim == 2 ? diffusion_F_t<float, 2>(nb, u, c, Fi, sat, s)
                      : diffusion_F_t<float, 3>(nb, u, c, Fi, sat, s);
}

int diffusion_step_coupled(const sph_nbr* nb, const sph_material* m, const sph_state* st,
                           double Dc, double dt, double c_bc, int nonlinear, hipStream_t s) {
  if (!st->c || !st->q || !st->p || !st->PB) {
    set_error("coupled diffusion needs c, q, p and the PB scratch");
    return SPH_E_ARG;
  }
  if (st->prec == SPH_F64)
    return nb->dim == 2 ? diffusion_coupled_t<double, 2>(nb, m, st, Dc, dt, c_bc, nonlinear, s)
                        : diffusion_coupled_t<double, 3>(nb, m, st, Dc, dt, c_bc, nonlinear, s);
  return nb->dim == 2 ? diffusion_coupled_t<float, 2>(nb, m, st, Dc, dt, c_bc, nonlinear, s)
                      : diffusion_coupled_t<float, 3>(nb, m, st, Dc, dt, c_bc, nonlinear, s);
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
