// sph_build.hip -- fixed total-Lagrangian neighbourhood on gfx950.
//
// Sec. 3.1 of the paper: in the TL form the neighbour set and the correction
// matrix B0 (eq. sph-correctmatrix) are built once, in the initial
// configuration.  Pipeline (all on the device, one host sync per size query):
//   bounds -> cell keys -> stable LSD radix sort (8-bit digits, bit-exact)
//   -> cell ranges -> neighbour count / scan / fill (FP64, no FMA in the
//   distance test) -> B0 -> damping schedule (anchors by cell parity, first-fit
//   levels inside each anchor).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstring>
#include <vector>

#include "sph_common.h"

namespace sph {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}
void clear_error() { g_err.clear(); }

// ---------------------------------------------------------------------------
// exclusive scan of int64 (setup only)
constexpr int kScanT = 256;
constexpr int kScanItems = 8;
constexpr int64_t kScanTile = kScanT * kScanItems;

__global__ __launch_bounds__(kScanT) void k_scan_local(const int64_t* in, int64_t* out,
                                                       int64_t* bsum, int64_t n) {
  __shared__ int64_t wsum[kScanT / 64];
  const int64_t base = blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    s += v[i];
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t incl = s;
  for (int off = 1; off < 64; off <<= 1) {
    int64_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int w = 0; w < kScanT / 64; ++w) {
      int64_t t = wsum[w];
      wsum[w] = run;
      run += t;
    }
  }
  __syncthreads();
  int64_t ex = incl - s + wsum[wid];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
  if (threadIdx.x == kScanT - 1) bsum[blockIdx.x] = ex;
}

__global__ void k_scan_add(int64_t* out, const int64_t* boff, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] += boff[i / kScanTile];
}

// out[i] = sum_{j<i} in[j]; *total (device, may be null) = sum of all
static int scan_exclusive(const int64_t* in, int64_t* out, int64_t n, int64_t* total,
                          hipStream_t s) {
  if (n <= 0) {
    if (total) SPH_HIP(hipMemsetAsync(total, 0, sizeof(int64_t), s));
    return SPH_OK;
  }
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  int64_t* bsum = nullptr;
  SPH_HIP(hipMalloc(&bsum, (nb + 1) * sizeof(int64_t)));
  k_scan_local<<<(unsigned)nb, kScanT, 0, s>>>(in, out, bsum, n);
  SPH_LAUNCH_CHECK();
  int rc = SPH_OK;
  if (nb > 1) {
    rc = scan_exclusive(bsum, bsum, nb, total, s);
    if (rc == SPH_OK) {
      k_scan_add<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(out, bsum, n);
      if (hipGetLastError() != hipSuccess) rc = SPH_E_DEVICE;
    }
  } else if (total) {
    if (hipMemcpyAsync(total, bsum, sizeof(int64_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
      rc = SPH_E_DEVICE;
  }
  hipStreamSynchronize(s);
  hipFree(bsum);
  return rc;
}

// ---------------------------------------------------------------------------
// bounds: componentwise min and max of X (one block, fixed-order tree)
__global__ __launch_bounds__(1024) void k_bounds(const double* X, int64_t n, int dim,
                                                 double* out /*[2*dim]*/) {
  __shared__ double slo[1024], shi[1024];
  for (int k = 0; k < dim; ++k) {
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      double x = X[k * n + i];
      lo = fmin(lo, x);
      hi = fmax(hi, x);
    }
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + w]);
        shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + w]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      out[2 * k] = slo[0];
      out[2 * k + 1] = shi[0];
    }
    __syncthreads();
  }
}

// The cell grid is a list of segments, one per specimen (one for an
// ordinary build): each has its own origin and cell counts, and its keys
// follow those of the previous segment, key = koff + x + nc0 (y + nc1 z).
// A specimen therefore gets exactly the cells, order and schedule it gets
// alone, and no cell or neighbour search crosses specimens.
struct Grid {
  int dim;
  int nseg;
  GridSeg g0;                 // the only segment when nseg == 1
  const GridSeg* seg;         // device [nseg]
  const uint16_t* cell_seg;   // device [n_cells]: segment of each cell (nseg > 1)
  double inv_rc;
};

__device__ __forceinline__ GridSeg seg_of_cell(const Grid& g, uint32_t key) {
  return g.nseg == 1 ? g.g0 : g.seg[g.cell_seg[key]];
}

__device__ __forceinline__ void key_coords_s(uint32_t key, const GridSeg& sg, int64_t c[3]) {
  int64_t k = (int64_t)key - sg.koff;
  c[0] = k % sg.nc0;
  k /= sg.nc0;
  c[1] = k % sg.nc1;
  c[2] = k / sg.nc1;
}

__device__ __forceinline__ void key_coords(uint32_t key, const Grid& g, int64_t c[3]) {
  key_coords_s(key, seg_of_cell(g, key), c);
}

__device__ __forceinline__ int64_t seg_key(const GridSeg& sg, int64_t x, int64_t y, int64_t z) {
  return sg.koff + x + sg.nc0 * (y + sg.nc1 * z);
}

__global__ void k_cellkey(const double* X, int64_t n, Grid g, const int32_t* __restrict__ spec_in,
                          uint32_t* key, uint32_t* val) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const GridSeg sg = g.nseg == 1 ? g.g0 : g.seg[spec_in[i]];
  int64_t c0 = (int64_t)floor((X[i] - sg.o0) * g.inv_rc);
  int64_t c1 = g.dim > 1 ? (int64_t)floor((X[n + i] - sg.o1) * g.inv_rc) : 0;
  int64_t c2 = g.dim > 2 ? (int64_t)floor((X[2 * n + i] - sg.o2) * g.inv_rc) : 0;
  c0 = c0 < 0 ? 0 : (c0 >= sg.nc0 ? sg.nc0 - 1 : c0);
  c1 = c1 < 0 ? 0 : (c1 >= sg.nc1 ? sg.nc1 - 1 : c1);
  c2 = c2 < 0 ? 0 : (c2 >= sg.nc2 ? sg.nc2 - 1 : c2);
  key[i] = (uint32_t)seg_key(sg, c0, c1, c2);
  val[i] = (uint32_t)i;
}

// segment of every cell (binary search over the segments' first keys)
__global__ void k_cell_seg(const GridSeg* __restrict__ seg, int nseg, int64_t ncells,
                           uint16_t* __restrict__ cell_seg) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (seg[mid].koff <= c) lo = mid;
    else hi = mid - 1;
  }
  cell_seg[c] = (uint16_t)lo;
}

// componentwise bounds of each specimen (one block per specimen)
__global__ __launch_bounds__(256) void k_bounds_seg(const double* X, int64_t n, int dim,
                                                    const int64_t* __restrict__ in_off,
                                                    double* out /*[nseg][6]*/) {
  __shared__ double slo[256], shi[256];
  const int64_t i0 = in_off[blockIdx.x], i1 = in_off[blockIdx.x + 1];
  for (int k = 0; k < dim; ++k) {
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
      const double x = X[k * n + i];
      lo = fmin(lo, x);
      hi = fmax(hi, x);
    }
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + w]);
        shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + w]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      out[blockIdx.x * 6 + 2 * k] = slo[0];
      out[blockIdx.x * 6 + 2 * k + 1] = shi[0];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (key, value), 8-bit digits
constexpr int kRsT = 256;
constexpr int kRsRounds = 4;
constexpr int64_t kRsTile = kRsT * kRsRounds;

__global__ __launch_bounds__(kRsT) void k_rs_hist(const uint32_t* keys, int64_t n, int shift,
                                                  int64_t* hist, int64_t nblk) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int r = 0; r < kRsRounds; ++r) {
    int64_t i = blockIdx.x * kRsTile + r * kRsT + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kRsT) void k_rs_scatter(const uint32_t* kin, const uint32_t* vin,
                                                     uint32_t* kout, uint32_t* vout, int64_t n,
                                                     int shift, const int64_t* offs,
                                                     int64_t nblk) {
  __shared__ uint32_t running[256];
  __shared__ uint32_t wcnt[kRsT / 64][256];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  running[threadIdx.x] = 0;
  for (int r = 0; r < kRsRounds; ++r) {
    int64_t i = blockIdx.x * kRsTile + r * kRsT + threadIdx.x;
    bool valid = i < n;
    uint32_t key = valid ? kin[i] : 0u;
    uint32_t d = (key >> shift) & 255u;
    for (int w = 0; w < kRsT / 64; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    uint64_t eq = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      int bit = (d >> b) & 1u;
      uint64_t bal = __ballot(bit);
      eq &= bit ? bal : ~bal;
    }
    uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    uint32_t rank = (uint32_t)__popcll(eq & lt);
    if (valid && rank == 0) wcnt[wid][d] = (uint32_t)__popcll(eq);
    __syncthreads();
    if (valid) {
      uint32_t pre = 0;
      for (int w = 0; w < wid; ++w) pre += wcnt[w][d];
      int64_t pos = offs[(int64_t)d * nblk + blockIdx.x] + running[d] + pre + rank;
      kout[pos] = key;
      vout[pos] = vin[i];
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kRsT / 64; ++w) add += wcnt[w][threadIdx.x];
    running[threadIdx.x] += add;
    __syncthreads();
  }
}

static int radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* kalt, uint32_t* valt, int64_t n,
                      uint32_t max_key, hipStream_t s) {
  int bits = 0;
  while (bits < 32 && (max_key >> bits) != 0u) ++bits;
  int passes = std::max(1, (bits + 7) / 8);
  int64_t nblk = (n + kRsTile - 1) / kRsTile;
  int64_t* hist = nullptr;
  SPH_HIP(hipMalloc(&hist, 256 * nblk * sizeof(int64_t)));
  uint32_t *ki = keys, *vi = vals, *ko = kalt, *vo = valt;
  int rc = SPH_OK;
  for (int p = 0; p < passes && rc == SPH_OK; ++p) {
    k_rs_hist<<<(unsigned)nblk, kRsT, 0, s>>>(ki, n, 8 * p, hist, nblk);
    if (hipGetLastError() != hipSuccess) { rc = SPH_E_DEVICE; break; }
    rc = scan_exclusive(hist, hist, 256 * nblk, nullptr, s);
    if (rc) break;
    k_rs_scatter<<<(unsigned)nblk, kRsT, 0, s>>>(ki, vi, ko, vo, n, 8 * p, hist, nblk);
    if (hipGetLastError() != hipSuccess) { rc = SPH_E_DEVICE; break; }
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  if (rc == SPH_OK && ki != keys) {
    if (hipMemcpyAsync(keys, ki, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(vals, vi, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
      rc = SPH_E_DEVICE;
  }
  hipStreamSynchronize(s);
  hipFree(hist);
  if (rc) set_error("radix sort failed");
  return rc;
}

// ---------------------------------------------------------------------------
__global__ void k_gather_sorted(const double* X, const double* V, const uint32_t* perm,
                                int64_t n, int dim, double* Xs, double* Vs, float* Vf) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  uint32_t id = perm[s];
  for (int k = 0; k < dim; ++k) Xs[k * n + s] = X[k * n + id];
  Vs[s] = V[id];
  Vf[s] = (float)V[id];
}

// cell_start[c] = first sorted position with key >= c, c in [0, ncells]
__global__ void k_cell_start(const uint32_t* key, int64_t n, int64_t ncells, uint32_t* cs) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c > ncells) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if ((int64_t)key[mid] < c) lo = mid + 1; else hi = mid;
  }
  cs[c] = (uint32_t)lo;
}

// neighbour test: r^2 in FP64 with no contraction, in a fixed operation order
template <bool FILL>
__global__ void k_nbr(const double* X, const uint32_t* key, const uint32_t* cs, int64_t n, Grid g,
                      double rc2, int64_t* deg, const int64_t* off, uint32_t* idx,
                      unsigned long long* maxdeg) {
#pragma clang fp contract(off)
  int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  int64_t c[3];
  const GridSeg sg = seg_of_cell(g, key[a]);
  key_coords_s(key[a], sg, c);
  double xa = X[a], ya = g.dim > 1 ? X[n + a] : 0.0, za = g.dim > 2 ? X[2 * n + a] : 0.0;
  int64_t cnt = 0;
  int64_t base = FILL ? off[a] : 0;
  int zlo = g.dim > 2 ? -1 : 0, zhi = g.dim > 2 ? 1 : 0;
  for (int dz = zlo; dz <= zhi; ++dz) {
    int64_t z = c[2] + dz;
    if (z < 0 || z >= sg.nc2) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      int64_t y = c[1] + dy;
      if (y < 0 || y >= sg.nc1) continue;
      int64_t x0 = c[0] > 0 ? c[0] - 1 : 0;
      int64_t x1 = c[0] + 1 < sg.nc0 ? c[0] + 1 : sg.nc0 - 1;
      int64_t k0 = seg_key(sg, x0, y, z);
      int64_t k1 = seg_key(sg, x1, y, z);
      for (int64_t b = cs[k0]; b < cs[k1 + 1]; ++b) {
        if (b == a) continue;
        double dx = X[b] - xa;
        double r2 = dx * dx;
        if (g.dim > 1) {
          double dy_ = X[n + b] - ya;
          r2 = r2 + dy_ * dy_;
        }
        if (g.dim > 2) {
          double dz_ = X[2 * n + b] - za;
          r2 = r2 + dz_ * dz_;
        }
        if (r2 < rc2) {
          if (FILL) idx[base + cnt] = (uint32_t)b;
          ++cnt;
        }
      }
    }
  }
  if (!FILL) {
    deg[a] = cnt;
    atomicMax(maxdeg, (unsigned long long)cnt);
  }
}

// B0_a = (sum_b V_b (X_b - X_a) (x) grad_a W_ab)^-1, eq. (sph-correctmatrix)
__global__ void k_B0(const double* X, const double* V, const int64_t* off, const uint32_t* idx,
                     int64_t n, int dim, double inv_h, double c5, double* B0, float* B0f,
                     int32_t* status) {
  int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  double M[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double xa[3] = {X[a], dim > 1 ? X[n + a] : 0.0, dim > 2 ? X[2 * n + a] : 0.0};
  for (int64_t j = off[a]; j < off[a + 1]; ++j) {
    int64_t b = idx[j];
    double d[3] = {0, 0, 0};
    double r2 = 0;
    for (int k = 0; k < dim; ++k) {
      d[k] = xa[k] - X[k * n + b];
      r2 += d[k] * d[k];
    }
    double w = dw_over_r(r2, inv_h, c5);
    for (int i = 0; i < dim; ++i)
      for (int k = 0; k < dim; ++k) M[i * 3 + k] += V[b] * (-d[i]) * (w * d[k]);
  }
  double Mi[9], det, fro = 0;
  for (int i = 0; i < dim; ++i)
    for (int k = 0; k < dim; ++k) fro += M[i * 3 + k] * M[i * 3 + k];
  fro = sqrt(fro);
  if (dim == 2) {
    det = M[0] * M[4] - M[1] * M[3];
    Mi[0] = M[4] / det;
    Mi[1] = -M[1] / det;
    Mi[3] = -M[3] / det;
    Mi[4] = M[0] / det;
  } else {
    double c00 = M[4] * M[8] - M[5] * M[7];
    double c01 = M[5] * M[6] - M[3] * M[8];
    double c02 = M[3] * M[7] - M[4] * M[6];
    det = M[0] * c00 + M[1] * c01 + M[2] * c02;
    Mi[0] = c00 / det;
    Mi[1] = (M[2] * M[7] - M[1] * M[8]) / det;
    Mi[2] = (M[1] * M[5] - M[2] * M[4]) / det;
    Mi[3] = c01 / det;
    Mi[4] = (M[0] * M[8] - M[2] * M[6]) / det;
    Mi[5] = (M[2] * M[3] - M[0] * M[5]) / det;
    Mi[6] = c02 / det;
    Mi[7] = (M[1] * M[6] - M[0] * M[7]) / det;
    Mi[8] = (M[0] * M[4] - M[1] * M[3]) / det;
  }
  double lim = 1e-12 * (dim == 2 ? fro * fro : fro * fro * fro);
  if (!(fabs(det) >= lim) || !isfinite(det)) atomicOr(status, SPH_STATUS_SINGULAR_B0);
  for (int i = 0; i < dim; ++i)
    for (int k = 0; k < dim; ++k) {
      B0[(i * dim + k) * n + a] = Mi[i * 3 + k];
      B0f[(i * dim + k) * n + a] = (float)Mi[i * 3 + k];
    }
}

// ---------------------------------------------------------------------------
// damping schedule
struct Block {
  int nr;
  int64_t beg[4], end[4];
};

__device__ __forceinline__ Block anchor_block(uint32_t akey, const Grid& g, const uint32_t* cs) {
  int64_t A[3];
  const GridSeg sg = seg_of_cell(g, akey);
  key_coords_s(akey, sg, A);
  Block blk;
  blk.nr = 0;
  int zmax = g.dim > 2 ? 1 : 0;
  for (int dz = 0; dz <= zmax; ++dz) {
    int64_t z = A[2] + dz;
    if (z >= sg.nc2) continue;
    for (int dy = 0; dy <= 1; ++dy) {
      int64_t y = A[1] + dy;
      if (y >= sg.nc1) continue;
      int64_t k0 = seg_key(sg, A[0], y, z);
      int64_t k1 = k0 + (A[0] + 1 < sg.nc0 ? 2 : 1);
      blk.beg[blk.nr] = cs[k0];
      blk.end[blk.nr] = cs[k1];
      ++blk.nr;
    }
  }
  return blk;
}

// a pair's anchor: a cell A whose block A .. A+1 holds both particles.
// Along an axis where the two cells differ it is the lower one; along an axis
// where both sit in cell c it is c - 1 when c >= 1 and bit k (the axis) of
// s + t is set, with s, t the pair's positions in its specimen's sorted
// range, else c (a particle's pairs spread over the colours instead of all
// landing on its own cell's anchor); along an axis of exactly two cells (of
// its specimen's grid segment) it is the first cell, so that the block spans
// the axis and one colour pass covers what the two parities along it would
// (same-colour blocks stay disjoint)
__device__ __forceinline__ bool anchored_at(int64_t s, int64_t t, uint32_t ks, uint32_t kt,
                                            const int64_t A[3], const Grid& g,
                                            const uint32_t* cs) {
  const GridSeg sg = seg_of_cell(g, ks);  // neighbours never cross specimens
  int64_t cs_[3], ct[3];
  key_coords_s(ks, sg, cs_);
  key_coords_s(kt, sg, ct);
  const int64_t nc[3] = {sg.nc0, sg.nc1, sg.nc2};
  const int64_t p0 = cs[sg.koff];  // the specimen's first sorted particle
  const int64_t sum = (s - p0) + (t - p0);
  for (int k = 0; k < 3; ++k) {
    int64_t m;
    if (nc[k] == 2)
      m = 0;
    else if (cs_[k] != ct[k])
      m = cs_[k] < ct[k] ? cs_[k] : ct[k];
    else
      m = (cs_[k] >= 1 && ((sum >> k) & 1)) ? cs_[k] - 1 : cs_[k];
    if (m != A[k]) return false;
  }
  return true;
}

// per cell: number of pairs anchored there, and the block's particle count
__global__ void k_sched_count(const uint32_t* key, const uint32_t* cs, const int64_t* off,
                              const uint32_t* idx, Grid g, int64_t ncells, int64_t* cnt,
                              unsigned long long* bmax) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  int64_t A[3];
  key_coords((uint32_t)c, g, A);
  Block blk = anchor_block((uint32_t)c, g, cs);
  int64_t m = 0, bc = 0;
  for (int r = 0; r < blk.nr; ++r) {
    bc += blk.end[r] - blk.beg[r];
    for (int64_t s = blk.beg[r]; s < blk.end[r]; ++s)
      for (int64_t j = off[s]; j < off[s + 1]; ++j) {
        uint32_t t = idx[j];
        if ((int64_t)t <= s) continue;
        if (anchored_at(s, t, key[s], key[t], A, g, cs)) ++m;
      }
  }
  cnt[c] = m;
  atomicMax(bmax, (unsigned long long)bc);
}

__global__ void k_color_flags(const int64_t* cnt, Grid g, int64_t ncells, int color,
                              int64_t* flag) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  int64_t A[3];
  key_coords((uint32_t)c, g, A);
  int col = (int)((A[0] & 1) | ((A[1] & 1) << 1) | ((A[2] & 1) << 2));
  flag[c] = (cnt[c] > 0 && col == color) ? 1 : 0;
}

__global__ void k_color_emit(const int64_t* cnt, const int64_t* flag, const int64_t* pos,
                             int64_t ncells, int64_t base, uint32_t* akey, int64_t* acnt) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncells || !flag[c]) return;
  akey[base + pos[c]] = (uint32_t)c;
  acnt[base + pos[c]] = cnt[c];
}

// one thread per anchor: enumerate its pairs in ascending (a, b), assign
// first-fit levels, write them level-major
__global__ void k_sched_fill(const uint32_t* key, const uint32_t* cs, const int64_t* off,
                             const uint32_t* idx, Grid g, const uint32_t* akey,
                             const int64_t* aoff, int64_t a0, int64_t a1, int words, int64_t bmax,
                             unsigned long long* scratch, uint32_t* ta, uint32_t* tb, uint32_t* tl,
                             uint32_t* pa, uint32_t* pb, uint32_t* pl, uint32_t* anlev,
                             unsigned long long* maxlev, int32_t* err) {
  int64_t ai = a0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (ai >= a1) return;
  unsigned long long* used = scratch + (ai - a0) * bmax * words;
  for (int64_t i = 0; i < bmax * words; ++i) used[i] = 0ull;
  uint32_t ak = akey[ai];
  int64_t A[3];
  key_coords(ak, g, A);
  Block blk = anchor_block(ak, g, cs);
  int64_t lbase[4];
  int64_t acc = 0;
  for (int r = 0; r < blk.nr; ++r) {
    lbase[r] = acc;
    acc += blk.end[r] - blk.beg[r];
  }
  int64_t o = aoff[ai];
  int64_t m = 0;
  uint32_t nl = 0;
  const int maxbits = words * 64;
  for (int r = 0; r < blk.nr; ++r)
    for (int64_t s = blk.beg[r]; s < blk.end[r]; ++s)
      for (int64_t j = off[s]; j < off[s + 1]; ++j) {
        uint32_t t = idx[j];
        if ((int64_t)t <= s) continue;
        if (!anchored_at(s, (int64_t)t, key[s], key[t], A, g, cs)) continue;
        int64_t ls = lbase[r] + (s - blk.beg[r]);
        int64_t lt = -1;
        for (int q = 0; q < blk.nr; ++q)
          if ((int64_t)t >= blk.beg[q] && (int64_t)t < blk.end[q]) lt = lbase[q] + ((int64_t)t - blk.beg[q]);
        if (lt < 0) {
          atomicOr(err, 1);
          return;
        }
        unsigned long long* Ua = used + ls * words;
        unsigned long long* Ub = used + lt * words;
        int lev = 0;
        while (lev < maxbits && (((Ua[lev >> 6] | Ub[lev >> 6]) >> (lev & 63)) & 1ull)) ++lev;
        if (lev >= maxbits) {
          atomicOr(err, 2);
          return;
        }
        Ua[lev >> 6] |= 1ull << (lev & 63);
        Ub[lev >> 6] |= 1ull << (lev & 63);
        ta[o + m] = (uint32_t)s;
        tb[o + m] = t;
        tl[o + m] = (uint32_t)lev;
        if ((uint32_t)lev + 1 > nl) nl = (uint32_t)lev + 1;
        ++m;
      }
  int64_t w = o;
  for (uint32_t lev = 0; lev < nl; ++lev)
    for (int64_t i = o; i < o + m; ++i)
      if (tl[i] == lev) {
        pa[w] = ta[i];
        pb[w] = tb[i];
        pl[w] = lev;
        ++w;
      }
  anlev[ai] = nl;
  atomicMax(maxlev, (unsigned long long)nl);
}

// ---------------------------------------------------------------------------
// tiles: ELL of window-local neighbour indices.  The order of a particle's
// neighbours is free (it only orders the terms of its sums), and is chosen
// for the LDS banks: a window particle's staged values sit at 16-byte slots,
// and a 128-bit LDS read serves sixteen lanes at a time, without a conflict
// when their slots are distinct mod 16.  Entry p of tile particle t takes, in
// ascending order within the class, a neighbour whose slot is
//   t + (p mod 4) + 8 ((p / 4) mod 2) + 4 (p / 8)   (mod 16)
// when one is left (else the next class that has one).  With one lane per
// particle, sixteen particles at one entry then read distinct classes; with
// two, eight particles at entries p and p + 4 (offsets 8 apart); with four,
// four particles at p, p + 4, p + 8, p + 12 (offsets 0, 8, 4, 12).  Along one
// particle's list every sixteen entries take every class once.
constexpr int kEllSpread = 256;  // longer lists keep ascending order

__global__ void k_tile_ell(const TileDesc* __restrict__ tiles, const uint32_t* __restrict__ tslot,
                           const int64_t* __restrict__ off, const uint32_t* __restrict__ idx,
                           int tmax, uint16_t* __restrict__ ell, int32_t* err) {
  const TileDesc& td = tiles[blockIdx.x];
  for (int t = threadIdx.x; t < tmax; t += blockDim.x) {
    uint32_t own = 0;
    int64_t j0 = 0, deg = 0;
    if ((uint32_t)t < td.count) {
      // thread slot t holds own particle s (slots by descending degree)
      const uint32_t sl = tslot[(int64_t)blockIdx.x * tmax + t] & 0xFFFFu;
      const int64_t a = sl < td.count0 ? (int64_t)td.p0 + sl : (int64_t)td.p1 + (sl - td.count0);
      own = sl < td.count0 ? td.own_base + sl : td.own_base1 + (sl - td.count0);
      j0 = off[a];
      deg = off[a + 1] - j0;
    } else {
      own = td.count0 > 0 ? td.own_base : td.own_base1;  // unused column: any valid index
    }
    auto at = [&](uint32_t j) -> uint16_t* {
      return ell + (int64_t)td.ell_off + (int64_t)(j >> 2) * 4 * tmax + 4 * t + (j & 3);
    };
    uint16_t L[kEllSpread];
    const bool spread = deg <= kEllSpread;
    for (uint32_t j = 0; j < td.width; ++j) {  // width: multiple of 4
      uint32_t loc = own;
      if ((int64_t)j < deg) {
        uint32_t b = idx[j0 + j];
        uint32_t base = 0;
        bool found = false;
        for (uint32_t r = 0; r < td.nruns; ++r) {
          uint32_t rel = b - td.run_start[r];
          if (rel < td.run_count[r]) {
            loc = base + rel;
            found = true;
            break;
          }
          base += td.run_count[r];
        }
        if (!found) atomicOr(err, 4);
        if (spread) L[j] = (uint16_t)loc;
      }
      *at(j) = (uint16_t)loc;
    }
    if (!spread) continue;
    int cur[16];  // next candidate of each class (ascending)
    for (int r = 0; r < 16; ++r) cur[r] = 0;
    for (int p = 0; p < (int)deg; ++p) {
      const int d = (t + (p & 3) + 8 * ((p >> 2) & 1) + 4 * (p >> 3)) & 15;
      int pick = -1;
      for (int k = 0; k < 16 && pick < 0; ++k) {
        const int r = (d + k) & 15;
        while (cur[r] < (int)deg && (L[cur[r]] & 15) != r) ++cur[r];
        if (cur[r] < (int)deg) pick = cur[r]++;
      }
      *at((uint32_t)p) = L[pick];
    }
  }
}

// damping: pack each canonical pair as (a_loc, b_loc) inside its anchor block
// record the block runs, the per-colour maxima that size
// each pass's LDS, and the pair geometry 2 V_a V_b (dW/dr)/r
__global__ void k_damp_pack(const uint32_t* __restrict__ akey, const int64_t* __restrict__ aoff,
                            const uint32_t* __restrict__ sa, const uint32_t* __restrict__ sb,
                            const uint32_t* __restrict__ slev, const uint32_t* __restrict__ cs,
                            const double* __restrict__ X, const double* __restrict__ V,
                            double inv_h, double c5, Grid g, int64_t n, int64_t n_anchors,
                            uint32_t* __restrict__ dpair,
                            float* __restrict__ dgeo32, double* __restrict__ dgeo64,
                            uint32_t* __restrict__ ablk, unsigned long long* bmax,
                            unsigned long long* pmax, int32_t* err) {
  int64_t ai = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (ai >= n_anchors) return;
  Block blk = anchor_block(akey[ai], g, cs);
  int64_t A[3];
  key_coords(akey[ai], g, A);
  const int col = (int)((A[0] & 1) | ((A[1] & 1) << 1) | ((A[2] & 1) << 2));
  int64_t lbase[4], acc = 0;
  for (int r = 0; r < 4; ++r) {
    ablk[8 * ai + 2 * r] = r < blk.nr ? (uint32_t)blk.beg[r] : 0u;
    ablk[8 * ai + 2 * r + 1] = r < blk.nr ? (uint32_t)(blk.end[r] - blk.beg[r]) : 0u;
  }
  for (int r = 0; r < blk.nr; ++r) {
    lbase[r] = acc;
    acc += blk.end[r] - blk.beg[r];
  }
  atomicMax(bmax + col, (unsigned long long)acc);
  atomicMax(pmax + col, (unsigned long long)(aoff[ai + 1] - aoff[ai]));
  if (acc > kDampMaxLocal) {
    atomicOr(err, 8);
    return;
  }
  for (int64_t i = aoff[ai]; i < aoff[ai + 1]; ++i) {
    int64_t loc[2] = {-1, -1};
    uint32_t pp[2] = {sa[i], sb[i]};
    for (int e = 0; e < 2; ++e)
      for (int r = 0; r < blk.nr; ++r)
        if ((int64_t)pp[e] >= blk.beg[r] && (int64_t)pp[e] < blk.end[r]) loc[e] = lbase[r] + (pp[e] - blk.beg[r]);
    if (loc[0] < 0 || loc[1] < 0 || slev[i] >= (uint32_t)kDampMaxLevel) {
      atomicOr(err, 16);
      continue;
    }
    dpair[i] = (uint32_t)loc[0] | ((uint32_t)loc[1] << kDampLocBits);
    double r2 = 0.0;
    for (int k = 0; k < g.dim; ++k) {
      double d = X[k * n + pp[0]] - X[k * n + pp[1]];
      r2 += d * d;
    }
    double q = sqrt(r2) * inv_h;
    double t = 1.0 - 0.5 * q;
    double geo = 2.0 * V[pp[0]] * V[pp[1]] * (c5 * t * t * t);
    dgeo64[i] = geo;
    dgeo32[i] = (float)geo;
  }
}

// level offsets of each anchor: dloff[base + L] = first pair of level L
// (relative to the anchor's first pair), dloff[base + nlev] = pair count
__global__ void k_lev_count(const uint32_t* __restrict__ anlev, int64_t n_anchors,
                            int64_t* __restrict__ cnt) {
  int64_t ai = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (ai < n_anchors) cnt[ai] = (int64_t)anlev[ai] + 1;
}

__global__ void k_lev_fill(const int64_t* __restrict__ aoff, const uint32_t* __restrict__ slev,
                           const int64_t* __restrict__ base, int64_t n_anchors,
                           uint16_t* __restrict__ dloff, uint32_t* __restrict__ dloff_base) {
  int64_t ai = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (ai >= n_anchors) return;
  const int64_t lo = aoff[ai], hi = aoff[ai + 1], b = base[ai];
  dloff_base[ai] = (uint32_t)b;
  uint32_t prev = 0xFFFFFFFFu;
  for (int64_t i = lo; i < hi; ++i) {
    const uint32_t L = slev[i];
    if (L != prev) dloff[b + L] = (uint16_t)(i - lo);
    prev = L;
  }
  dloff[b + prev + 1] = (uint16_t)(hi - lo);
}

// Joint rows of the damping sweep (setup, on the host).  A wavefront sweeps
// APW = 64 / G anchors of one colour together: each of its G-lane groups
// stages one anchor's block, and a row of the wavefront's schedule holds up
// to 64 pairs from any of its anchors, one per lane.  In a row an anchor
// contributes pairs of one level only (the pairs of a level share no
// particle, nor do the blocks of one colour), and its levels come in order,
// so the sweep is the canonical one; the lane order inside a row is free and
// is chosen so that each eighth of the wavefront's LDS accesses spreads over
// the banks.  Rows are filled by list scheduling:
// the anchors with the most levels still to go take their next level first,
// a level that does not fit the row's free lanes is split.  The anchors of a
// colour are grouped into wavefronts by descending level count, so anchors
// that need as many rows share one.  Per width G:
//   drow       row words first | end << 16, relative to the wavefront's first
//              record; each wavefront's list framed by kDampRowPad empty rows
//   drow_base  [n_waves + 1] start of each framed list
//   dwave      [n_waves][APW][8] block runs (begin, count) x 4 of each
//              wavefront's anchors (all counts 0: no anchor)
//   dwrec      [n_waves] first record of each wavefront, from its colour's
//              first pair
//   djinfo     [n_upairs] record position of each canonical pair | its
//              anchor's group << 28
// A wavefront's records must stay below 2^16 (the row words' range); a width
// whose wavefronts exceed it is marked unusable.
template <typename T>
static int dalloc(T** p, int64_t count);

static int build_joint_rows(sph_nbr* nb, hipStream_t s) {
  const int64_t na = nb->n_anchors, np = nb->n_upairs;
  std::vector<uint32_t> anlev(na), dloff_base(na);
  std::vector<int64_t> aoff(na + 1);
  int64_t nloff = 0;
  if (na > 0) {
    SPH_HIP(hipMemcpyAsync(anlev.data(), nb->anlev, na * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipMemcpyAsync(dloff_base.data(), nb->dloff_base, na * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
    SPH_HIP(hipMemcpyAsync(aoff.data(), nb->aoff, (na + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    nloff = (int64_t)dloff_base[na - 1] + anlev[na - 1] + 1;
  } else {
    aoff[0] = 0;
  }
  std::vector<uint16_t> dloff(std::max<int64_t>(nloff, 1));
  if (nloff > 0) {
    SPH_HIP(hipMemcpyAsync(dloff.data(), nb->dloff, nloff * sizeof(uint16_t), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
  }
  std::vector<uint32_t> info(std::max<int64_t>(np, 1)), dpair(std::max<int64_t>(np, 1));
  std::vector<uint32_t> ablk(8 * std::max<int64_t>(na, 1));
  if (np > 0) {
    SPH_HIP(hipMemcpyAsync(dpair.data(), nb->dpair, np * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
  }
  if (na > 0) {
    SPH_HIP(hipMemcpyAsync(ablk.data(), nb->ablk, 8 * na * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
  }
  struct RowPair {
    int64_t i;        // canonical pair
    uint32_t g;       // its anchor's group in the wavefront
    uint32_t qa, qb;  // LDS slot mod 8 of the two particles
  };
  std::vector<RowPair> rp;
  for (int gi = 0; gi < kDampWidths; ++gi) {
    const int apw = 64 / (8 << gi);
    std::vector<uint32_t> rows, wave, wrec;
    std::vector<int64_t> rbase;
    bool ok = true;
    int64_t nw = 0;
    for (int c = 0; c < 8; ++c) {
      nb->dwave_off[gi][c] = nw;
      const int64_t a0 = nb->color_off[c], a1 = nb->color_off[c + 1];
      std::vector<int64_t> order;
      for (int64_t a = a0; a < a1; ++a) order.push_back(a);
      std::stable_sort(order.begin(), order.end(),
                       [&](int64_t x, int64_t y) { return anlev[x] > anlev[y]; });
      const int64_t po = a0 < na ? aoff[a0] : np;
      const uint32_t per = (uint32_t)std::max<int64_t>(nb->damp_bmax[c], 1) + 1;  // slots per block
      int64_t rec_c = 0;  // records of the colour so far
      for (size_t w0 = 0; w0 < order.size(); w0 += apw, ++nw) {
        const int k = (int)std::min<size_t>(apw, order.size() - w0);
        int64_t wa[8];
        int lev[8], taken[8];
        for (int g = 0; g < apw; ++g) {
          for (int e = 0; e < 8; ++e) wave.push_back(g < k ? ablk[8 * order[w0 + g] + e] : 0u);
          if (g < k) {
            wa[g] = order[w0 + g];
            lev[g] = 0;
            taken[g] = 0;
          }
        }
        wrec.push_back((uint32_t)rec_c);
        rbase.push_back((int64_t)rows.size());
        for (int r = 0; r < kDampRowPad; ++r) rows.push_back(0u);
        int64_t cur = 0;  // records of this wavefront so far
        for (;;) {
          int idx[8], m = 0;
          for (int g = 0; g < k; ++g)
            if (lev[g] < (int)anlev[wa[g]]) idx[m++] = g;
          if (m == 0) break;
          std::stable_sort(idx, idx + m, [&](int x, int y) {
            return (int)anlev[wa[x]] - lev[x] > (int)anlev[wa[y]] - lev[y];
          });
          const int64_t first = cur;
          int free = 64;
          rp.clear();
          for (int j = 0; j < m && free > 0; ++j) {
            const int g = idx[j];
            const uint16_t* lo = dloff.data() + dloff_base[wa[g]];
            const int size = (int)lo[lev[g] + 1] - (int)lo[lev[g]];
            const int take = std::min(free, size - taken[g]);
            const int64_t p0 = aoff[wa[g]] + lo[lev[g]] + taken[g];
            for (int t = 0; t < take; ++t) {
              const uint32_t wd = dpair[p0 + t];
              const uint32_t sa_ = (uint32_t)g * per + (wd & 0xFFFFu), sb_ = (uint32_t)g * per + (wd >> 16);
              rp.push_back(RowPair{p0 + t, (uint32_t)g, sa_ & 7u, sb_ & 7u});
            }
            cur += take;
            free -= take;
            taken[g] += take;
            if (taken[g] == size) {
              ++lev[g];
              taken[g] = 0;
            }
          }
          // lanes in eighths of 8: within an eighth, pairs whose particles'
          // 16-byte LDS slots are distinct mod 8 first -- the pairs of a row
          // are independent, so their lane order is free.  (Groups of 16
          // distinct mod 16, which a 128-bit read alone would want, measured
          // slower: the row also writes 96 bits per particle.)
          {
            std::vector<char> used(rp.size(), 0);
            int64_t pos = first;
            size_t left = rp.size();
            while (left > 0) {
              const int q = (int)std::min<size_t>(8, left);
              uint32_t ma = 0, mb = 0;
              int got = 0;
              for (size_t j = 0; j < rp.size() && got < q; ++j)
                if (!used[j] && !((ma >> rp[j].qa) & 1u) && !((mb >> rp[j].qb) & 1u)) {
                  used[j] = 1;
                  ma |= 1u << rp[j].qa;
                  mb |= 1u << rp[j].qb;
                  info[rp[j].i] = (uint32_t)(po + rec_c + pos++) | (rp[j].g << 28);
                  ++got;
                }
              for (size_t j = 0; j < rp.size() && got < q; ++j)
                if (!used[j] && !(((ma >> rp[j].qa) & 1u) && ((mb >> rp[j].qb) & 1u))) {
                  used[j] = 1;
                  ma |= 1u << rp[j].qa;
                  mb |= 1u << rp[j].qb;
                  info[rp[j].i] = (uint32_t)(po + rec_c + pos++) | (rp[j].g << 28);
                  ++got;
                }
              for (size_t j = 0; j < rp.size() && got < q; ++j)
                if (!used[j]) {
                  used[j] = 1;
                  info[rp[j].i] = (uint32_t)(po + rec_c + pos++) | (rp[j].g << 28);
                  ++got;
                }
              left -= (size_t)q;
            }
          }
          if (cur > 65535) ok = false;
          rows.push_back((uint32_t)(first & 0xFFFF) | ((uint32_t)(cur & 0xFFFF) << 16));
        }
        for (int r = 0; r < kDampRowPad; ++r) rows.push_back(0u);
        rec_c += cur;
      }
    }
    nb->dwave_off[gi][8] = nw;
    rbase.push_back((int64_t)rows.size());
    if (np + 1 >= (int64_t)(1u << 28)) ok = false;
    nb->dwidth_ok[gi] = ok;
    if (wave.empty()) wave.push_back(0u);
    if (wrec.empty()) wrec.push_back(0u);
    if (rows.empty()) rows.push_back(0u);
    int rc;
    if ((rc = dalloc(&nb->drow[gi], (int64_t)rows.size())) ||
        (rc = dalloc(&nb->drow_base[gi], (int64_t)rbase.size())) ||
        (rc = dalloc(&nb->dwave[gi], (int64_t)wave.size())) ||
        (rc = dalloc(&nb->dwrec[gi], (int64_t)wrec.size())) ||
        (rc = dalloc(&nb->djinfo[gi], std::max<int64_t>(np, 1))))
      return rc;
    SPH_HIP(hipMemcpyAsync(nb->drow[gi], rows.data(), rows.size() * sizeof(uint32_t),
                           hipMemcpyHostToDevice, s));
    SPH_HIP(hipMemcpyAsync(nb->drow_base[gi], rbase.data(), rbase.size() * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    SPH_HIP(hipMemcpyAsync(nb->dwave[gi], wave.data(), wave.size() * sizeof(uint32_t),
                           hipMemcpyHostToDevice, s));
    SPH_HIP(hipMemcpyAsync(nb->dwrec[gi], wrec.data(), wrec.size() * sizeof(uint32_t),
                           hipMemcpyHostToDevice, s));
    if (np > 0)
      SPH_HIP(hipMemcpyAsync(nb->djinfo[gi], info.data(), np * sizeof(uint32_t),
                             hipMemcpyHostToDevice, s));
    SPH_HIP(hipStreamSynchronize(s));  // the host vectors are reused
  }
  return SPH_OK;
}

// host planning of row tiles (setup only)
// A tile's own particles are a run of cells along x in one row of cells, or
// in two stacked rows (the two z-rows of a slab two cells thick in 3D, pairs
// of y-rows in 2D), which then share one window: its neighbouring rows over
// the x-range widened by one cell.  Tiles grow along x while the window stays
// within `wmax` (the LDS budget that keeps two workgroups per CU); a single
// cell may exceed it up to `wmax_hard` (the whole LDS of a CU).
static int plan_tiles(const sph_nbr* nb, const std::vector<uint32_t>& cs,
                      const std::vector<int64_t>& off, int tmax, int64_t wmax, int64_t wmax_hard,
                      std::vector<TileDesc>& out, std::vector<uint32_t>& tslot,
                      int64_t& window_max, int64_t& ell_len) {
  const int dim = nb->dim;
  out.clear();
  tslot.clear();
  window_max = 0;
  ell_len = 0;
  auto own_index = [](const TileDesc& td, uint32_t t) -> int64_t {
    return t < td.count0 ? (int64_t)td.p0 + t : (int64_t)td.p1 + (t - td.count0);
  };
  std::vector<uint32_t> ord;
  auto emit = [&](TileDesc& td) {
    uint32_t width = 0;
    ord.resize(td.count);
    for (uint32_t t = 0; t < td.count; ++t) {
      const int64_t a = own_index(td, t);
      width = std::max<uint32_t>(width, (uint32_t)(off[a + 1] - off[a]));
      ord[t] = t;
    }
    auto deg = [&](uint32_t t) { return off[own_index(td, t) + 1] - off[own_index(td, t)]; };
    std::stable_sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) { return deg(x) > deg(y); });
    for (int t = 0; t < tmax; ++t)
      tslot.push_back((uint32_t)t < td.count
                          ? ord[t] | (uint32_t)((deg(ord[t]) + 3) / 4) << 16
                          : 0u);
    td.width = (width + 3) & ~3u;
    td.ell_off = (uint32_t)ell_len;
    ell_len += (int64_t)td.width * tmax;
    window_max = std::max<int64_t>(window_max, td.window);
    out.push_back(td);
  };
  for (const GridSeg& sg : nb->segs) {  // rows never cross segments (specimens)
    const int64_t nc0 = sg.nc0, nc1 = sg.nc1, nc2 = sg.nc2;
    auto key = [&](int64_t x, int64_t y, int64_t z) { return sg.koff + x + nc0 * (y + nc1 * z); };
    // rows of one tile: (y, z) of each own row; stacked rows share the window
    struct Rows {
      int n;
      int64_t y[2], z[2];
    };
    auto col_count = [&](const Rows& R, int64_t x) {
      int64_t c = 0;
      for (int r = 0; r < R.n; ++r) c += (int64_t)cs[key(x, R.y[r], R.z[r]) + 1] - cs[key(x, R.y[r], R.z[r])];
      return c;
    };
    // the tile of rows R over cells x0..x1; `chunk` (single row only) limits
    // the own particles to [c0, c0 + cn) of that one cell
    auto make = [&](const Rows& R, int64_t x0, int64_t x1, bool chunk, int64_t c0, int64_t cn,
                    TileDesc& td) -> int64_t {
      std::memset(&td, 0, sizeof(td));
      const int64_t xa = x0 > 0 ? x0 - 1 : 0, xb = x1 + 1 < nc0 ? x1 + 1 : nc0 - 1;
      int64_t ylo = R.y[0], yhi = R.y[R.n - 1], zlo = R.z[0], zhi = R.z[R.n - 1];
      ylo = std::max<int64_t>(ylo - 1, 0);
      yhi = std::min<int64_t>(yhi + 1, nc1 - 1);
      if (dim == 3) {
        zlo = std::max<int64_t>(zlo - 1, 0);
        zhi = std::min<int64_t>(zhi + 1, nc2 - 1);
      }
      int64_t op[2] = {0, 0}, oc[2] = {0, 0}, ob[2] = {0, 0};
      for (int r = 0; r < R.n; ++r) {
        op[r] = cs[key(x0, R.y[r], R.z[r])];
        oc[r] = (int64_t)cs[key(x1, R.y[r], R.z[r]) + 1] - op[r];
        if (chunk) {
          op[r] += c0;
          oc[r] = cn;
        }
      }
      int64_t w = 0;
      for (int64_t zz = zlo; zz <= zhi; ++zz)
        for (int64_t yy = ylo; yy <= yhi; ++yy) {
          const int64_t s0 = cs[key(xa, yy, zz)], s1 = cs[key(xb, yy, zz) + 1];
          for (int r = 0; r < R.n; ++r)
            if (yy == R.y[r] && zz == R.z[r]) ob[r] = w + (op[r] - s0);
          td.run_start[td.nruns] = (uint32_t)s0;
          td.run_count[td.nruns] = (uint32_t)(s1 - s0);
          ++td.nruns;
          w += s1 - s0;
        }
      // an empty first row: the second one alone (p0 stays a valid own particle)
      const int f = (R.n == 2 && oc[0] == 0) ? 1 : 0;
      td.p0 = (uint32_t)op[f];
      td.own_base = (uint32_t)ob[f];
      td.count0 = (uint32_t)oc[f];
      td.p1 = (uint32_t)(R.n == 2 && f == 0 ? op[1] : op[f]);
      td.own_base1 = (uint32_t)(R.n == 2 && f == 0 ? ob[1] : ob[f]);
      td.count = (uint32_t)(oc[f] + (R.n == 2 && f == 0 ? oc[1] : 0));
      td.window = (uint32_t)w;
      return w;
    };
    auto walk = [&](const Rows& R) -> int {
      int64_t x = 0;
      while (x < nc0) {
        int64_t cnt = col_count(R, x);
        if (cnt == 0) {
          ++x;
          continue;
        }
        TileDesc td;
        if (cnt > tmax) {  // one dense column: each row's cell in chunks
          for (int r = 0; r < R.n; ++r) {
            const Rows R1{1, {R.y[r], 0}, {R.z[r], 0}};
            const int64_t cc = col_count(R1, x);
            for (int64_t c0 = 0; c0 < cc; c0 += tmax) {
              if (make(R1, x, x, true, c0, std::min<int64_t>(tmax, cc - c0), td) > wmax_hard)
                return SPH_E_CAPACITY;
              emit(td);
            }
          }
          ++x;
          continue;
        }
        int64_t x1 = x;
        while (x1 + 1 < nc0) {
          const int64_t nxt = col_count(R, x1 + 1);
          if (cnt + nxt > tmax) break;
          if (make(R, x, x1 + 1, false, 0, 0, td) > wmax) break;
          cnt += nxt;
          ++x1;
        }
        if (make(R, x, x1, false, 0, 0, td) > (x1 == x ? wmax_hard : wmax)) return SPH_E_CAPACITY;
        emit(td);
        x = x1 + 1;
      }
      return SPH_OK;
    };
    int rc;
    if (dim == 3 && nc2 == 2) {
      // a slab two cells thick: both z-rows of each y share one window
      for (int64_t y = 0; y < nc1; ++y)
        if ((rc = walk(Rows{2, {y, y}, {0, 1}}))) return rc;
    } else if (dim == 2) {
      // pairs of y-rows: four window rows for two own rows
      for (int64_t y = 0; y < nc1; y += 2)
        if ((rc = walk(y + 1 < nc1 ? Rows{2, {y, y + 1}, {0, 0}} : Rows{1, {y, 0}, {0, 0}})))
          return rc;
    } else {
      // rows in (y, z) order: the z-neighbour rows a tile's window needs were
      // just staged by the previous rows' tiles, so they are still in L2
      for (int64_t y = 0; y < nc1; ++y)
        for (int64_t z = 0; z < nc2; ++z)
          if ((rc = walk(Rows{1, {y, 0}, {z, 0}}))) return rc;
    }
  }
  if (ell_len >= (1LL << 32)) return SPH_E_CAPACITY;
  return SPH_OK;
}

// ---------------------------------------------------------------------------
// the per-step scratch: (pair word, q) damping records of both precisions
// (8 B in FP32, 16 B (word, pad, q) in FP64, and a sentinel record after the
// last pair), the inverse masses of both precisions, the kinetic-energy block
// partials and the gradient partials, each at a 256-byte boundary
constexpr int kWsParts = 6;
static int64_t ws_layout(const sph_nbr* nb, int64_t off[kWsParts + 1]) {
  const int64_t n1 = std::max<int64_t>(nb->n, 1);
  const int64_t part[kWsParts] = {(nb->n_upairs + 1) * 8, (nb->n_upairs + 1) * 16,
                                  n1 * (int64_t)sizeof(float), n1 * (int64_t)sizeof(double),
                                  kKeMaxBlocks * (int64_t)sizeof(double),
                                  nb->gpart_slots * SPH_NGRAD * (int64_t)sizeof(double)};
  off[0] = 0;
  for (int i = 0; i < kWsParts; ++i) off[i + 1] = (off[i] + part[i] + 255) & ~int64_t(255);
  return off[kWsParts];
}

// point the handle's scratch into `base` and clear what must start at zero
static int ws_attach(sph_nbr* nb, char* base, hipStream_t s) {
  int64_t off[kWsParts + 1];
  ws_layout(nb, off);
  nb->dwq[SPH_F32] = base + off[0];
  nb->dwq[SPH_F64] = base + off[1];
  nb->imass[SPH_F32] = base + off[2];
  nb->imass[SPH_F64] = base + off[3];
  nb->ke_partial = reinterpret_cast<double*>(base + off[4]);
  nb->gpart = reinterpret_cast<double*>(base + off[5]);
  SPH_HIP(hipMemsetAsync(nb->gpart, 0, nb->gpart_slots * SPH_NGRAD * sizeof(double), s));
  nb->damp_pre = false;
  for (int p = 0; p < 2; ++p)
    for (int c = 0; c < 8; ++c) nb->damp_g_used[p][c] = 0;
  return SPH_OK;
}

static void free_nbr(sph_nbr* h) {
  if (!h) return;
  void* ptrs[] = {h->key, h->perm, h->cell_start, h->nbr_off, h->nbr_idx, h->X,   h->V,
                  h->B0,  h->Vf,   h->B0f,        h->gsum, h->gsumf, h->sa,      h->sb,      h->slev, h->akey,
                  h->aoff, h->anlev, h->ctrl,     h->ws_own, h->dpair, h->ablk,
                  h->dgeo32, h->dgeo64, h->dloff, h->dloff_base,
                  h->tiling[0].tiles, h->tiling[0].ell, h->tiling[1].tiles, h->tiling[1].ell,
                  h->tiling[0].tslot, h->tiling[1].tslot};
  for (void* p : ptrs)
    if (p) hipFree(p);
  for (void* p : {(void*)h->spec, (void*)h->spec_off_dev, (void*)h->bt32, (void*)h->bt64,
                  (void*)h->gdiff, (void*)h->dsegs, (void*)h->cell_seg})
    if (p) hipFree(p);
  for (int gi = 0; gi < kDampWidths; ++gi)
    for (void* p : {(void*)h->drow[gi], (void*)h->drow_base[gi], (void*)h->dwave[gi],
                    (void*)h->dwrec[gi], (void*)h->djinfo[gi]})
      if (p) hipFree(p);
  free_graph_cache(h);
  if (h->ctrl_host) hipHostFree(h->ctrl_host);
  if (h->prof) {
    prof_resolve(h);
    for (hipEvent_t e : h->prof->pool) hipEventDestroy(e);
    delete h->prof;
  }
  delete h;
}

template <typename T>
static int dalloc(T** p, int64_t count) {
  *p = nullptr;
  SPH_HIP(hipMalloc((void**)p, (size_t)std::max<int64_t>(count, 1) * sizeof(T)));
  return SPH_OK;
}

static inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

static int build(int dim, int64_t n, const double* X, const double* V, double h, int32_t nseg,
                 const int32_t* spec_in, hipStream_t s, sph_nbr* nb) {
  nb->dim = dim;
  nb->n = n;
  nb->h = h;
  const double rc = 2.0 * h;
  const double rc2 = rc * rc;
  nb->inv_rc = 1.0 / rc;
  const double pi = 3.14159265358979323846;
  double alpha = dim == 2 ? 7.0 / (4.0 * pi * h * h) : 21.0 / (16.0 * pi * h * h * h);
  nb->c5 = -5.0 * alpha / (h * h);
  nb->inv_h = 1.0 / h;
  SPH_HIP(hipGetDevice(&nb->device));

  // bounds: of the whole cloud, or of each specimen (contiguous input ranges)
  std::vector<double> hb(6 * (size_t)nseg, 0.0);
  double* dbounds = nullptr;
  SPH_HIP(hipMalloc(&dbounds, 6 * (size_t)nseg * sizeof(double)));
  if (nseg == 1) {
    k_bounds<<<1, 1024, 0, s>>>(X, n, dim, dbounds);
    SPH_LAUNCH_CHECK();
  } else {
    std::vector<int32_t> hs(n);
    SPH_HIP(hipMemcpy(hs.data(), spec_in, n * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int64_t> in_off(nseg + 1, 0);
    if (hs[0] != 0) {
      hipFree(dbounds);
      set_error("specimen ids must start at 0");
      return SPH_E_ARG;
    }
    for (int64_t i = 1; i < n; ++i) {
      if (hs[i] != hs[i - 1] && hs[i] != hs[i - 1] + 1) {
        hipFree(dbounds);
        set_error("specimen ids must be contiguous ascending runs (particle %lld)", (long long)i);
        return SPH_E_ARG;
      }
      if (hs[i] != hs[i - 1]) in_off[hs[i]] = i;
    }
    if (hs[n - 1] != nseg - 1) {
      hipFree(dbounds);
      set_error("specimen ids must cover 0..%d", nseg - 1);
      return SPH_E_ARG;
    }
    in_off[nseg] = n;
    int64_t* din = nullptr;
    SPH_HIP(hipMalloc(&din, (nseg + 1) * sizeof(int64_t)));
    SPH_HIP(hipMemcpy(din, in_off.data(), (nseg + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    k_bounds_seg<<<(unsigned)nseg, 256, 0, s>>>(X, n, dim, din, dbounds);
    SPH_LAUNCH_CHECK();
    SPH_HIP(hipStreamSynchronize(s));
    hipFree(din);
  }
  SPH_HIP(hipMemcpyAsync(hb.data(), dbounds, (nseg == 1 ? 2 * dim : 6 * nseg) * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  hipFree(dbounds);
  nb->segs.assign(nseg, GridSeg{1, 1, 1, 0.0, 0.0, 0.0, 0});
  int64_t koff = 0;
  for (int sgi = 0; sgi < nseg; ++sgi) {
    const double* b = hb.data() + (nseg == 1 ? 0 : 6 * sgi);
    int64_t nc[3] = {1, 1, 1};
    double org[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k) {
      if (!std::isfinite(b[2 * k]) || !std::isfinite(b[2 * k + 1])) {
        set_error("non-finite reference positions");
        return SPH_E_ARG;
      }
      nc[k] = (int64_t)floor((b[2 * k + 1] - b[2 * k]) * nb->inv_rc) + 1;
      // the cloud is centred in the cell grid (equal margins on both sides)
      org[k] = b[2 * k] - 0.5 * ((double)nc[k] * rc - (b[2 * k + 1] - b[2 * k]));
    }
    nb->segs[sgi] = GridSeg{nc[0], nc[1], nc[2], org[0], org[1], org[2], koff};
    koff += nc[0] * nc[1] * nc[2];
    if (koff > 0xFFFFFFF0LL) break;
  }
  for (int k = 0; k < 3; ++k) {
    nb->nc[k] = k == 0 ? nb->segs[0].nc0 : (k == 1 ? nb->segs[0].nc1 : nb->segs[0].nc2);
    nb->origin[k] = k == 0 ? nb->segs[0].o0 : (k == 1 ? nb->segs[0].o1 : nb->segs[0].o2);
  }
  nb->n_cells = koff;
  if (nb->n_cells > 0xFFFFFFF0LL || n > 0xFFFFFFF0LL) {
    set_error("too many cells (%lld) or particles", (long long)nb->n_cells);
    return SPH_E_CAPACITY;
  }
  SPH_HIP(hipMalloc(&nb->dsegs, nseg * sizeof(GridSeg)));
  SPH_HIP(hipMemcpy(nb->dsegs, nb->segs.data(), nseg * sizeof(GridSeg), hipMemcpyHostToDevice));
  if (nseg > 1) {
    SPH_HIP(hipMalloc(&nb->cell_seg, nb->n_cells * sizeof(uint16_t)));
    k_cell_seg<<<nblocks(nb->n_cells, 256), 256, 0, s>>>(nb->dsegs, nseg, nb->n_cells, nb->cell_seg);
    SPH_LAUNCH_CHECK();
  }
  Grid g{dim, nseg, nb->segs[0], nb->dsegs, nb->cell_seg, nb->inv_rc};

  // keys and stable sort
  uint32_t *kalt = nullptr, *valt = nullptr;
  int rc_ = SPH_OK;
  if ((rc_ = dalloc(&nb->key, n)) || (rc_ = dalloc(&nb->perm, n)) || (rc_ = dalloc(&kalt, n)) ||
      (rc_ = dalloc(&valt, n)))
    return rc_;
  k_cellkey<<<nblocks(n, 256), 256, 0, s>>>(X, n, g, spec_in, nb->key, nb->perm);
  SPH_LAUNCH_CHECK();
  rc_ = radix_sort(nb->key, nb->perm, kalt, valt, n, (uint32_t)(nb->n_cells - 1), s);
  hipFree(kalt);
  hipFree(valt);
  if (rc_) return rc_;

  if ((rc_ = dalloc(&nb->X, dim * n)) || (rc_ = dalloc(&nb->V, n)) || (rc_ = dalloc(&nb->Vf, n)) ||
      (rc_ = dalloc(&nb->cell_start, nb->n_cells + 1)))
    return rc_;
  k_gather_sorted<<<nblocks(n, 256), 256, 0, s>>>(X, V, nb->perm, n, dim, nb->X, nb->V, nb->Vf);
  SPH_LAUNCH_CHECK();
  k_cell_start<<<nblocks(nb->n_cells + 1, 256), 256, 0, s>>>(nb->key, n, nb->n_cells,
                                                              nb->cell_start);
  SPH_LAUNCH_CHECK();

  // neighbours
  int64_t* deg = nullptr;
  unsigned long long* dmax = nullptr;
  if ((rc_ = dalloc(&deg, n + 1)) || (rc_ = dalloc(&nb->nbr_off, n + 1)) || (rc_ = dalloc(&dmax, 4)))
    return rc_;
  SPH_HIP(hipMemsetAsync(dmax, 0, 4 * sizeof(unsigned long long), s));
  k_nbr<false><<<nblocks(n, 128), 128, 0, s>>>(nb->X, nb->key, nb->cell_start, n, g, rc2, deg,
                                               nullptr, nullptr, dmax);
  SPH_LAUNCH_CHECK();
  rc_ = scan_exclusive(deg, nb->nbr_off, n, nb->nbr_off + n, s);
  hipFree(deg);
  if (rc_) return rc_;
  int64_t P = 0;
  unsigned long long maxdeg = 0;
  SPH_HIP(hipMemcpyAsync(&P, nb->nbr_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipMemcpyAsync(&maxdeg, dmax, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  nb->n_pairs = P;
  nb->n_upairs = P / 2;
  nb->max_deg = (int64_t)maxdeg;
  if ((rc_ = dalloc(&nb->nbr_idx, P))) return rc_;
  k_nbr<true><<<nblocks(n, 128), 128, 0, s>>>(nb->X, nb->key, nb->cell_start, n, g, rc2, nullptr,
                                              nb->nbr_off, nb->nbr_idx, nullptr);
  SPH_LAUNCH_CHECK();

  // correction matrices
  int32_t* dstat = nullptr;
  if ((rc_ = dalloc(&nb->B0, dim * dim * n)) || (rc_ = dalloc(&nb->B0f, dim * dim * n)) ||
      (rc_ = dalloc(&dstat, 2)))
    return rc_;
  SPH_HIP(hipMemsetAsync(dstat, 0, 2 * sizeof(int32_t), s));
  k_B0<<<nblocks(n, 128), 128, 0, s>>>(nb->X, nb->V, nb->nbr_off, nb->nbr_idx, n, dim, nb->inv_h,
                                       nb->c5, nb->B0, nb->B0f, dstat);
  SPH_LAUNCH_CHECK();
  int32_t hstat = 0;
  SPH_HIP(hipMemcpyAsync(&hstat, dstat, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  if (hstat) {
    hipFree(dstat);
    hipFree(dmax);
    set_error("singular correction matrix (particle without a full-rank neighbourhood)");
    return SPH_E_NUMERIC;
  }

  // damping schedule
  const int64_t nc = nb->n_cells;
  int64_t *cnt = nullptr, *flag = nullptr, *pos = nullptr, *acnt = nullptr;
  if ((rc_ = dalloc(&cnt, nc)) || (rc_ = dalloc(&flag, nc)) || (rc_ = dalloc(&pos, nc + 1)) ||
      (rc_ = dalloc(&nb->akey, nc)) || (rc_ = dalloc(&acnt, nc + 1)))
    return rc_;
  SPH_HIP(hipMemsetAsync(dmax, 0, 4 * sizeof(unsigned long long), s));
  k_sched_count<<<nblocks(nc, 128), 128, 0, s>>>(nb->key, nb->cell_start, nb->nbr_off,
                                                 nb->nbr_idx, g, nc, cnt, dmax);
  SPH_LAUNCH_CHECK();
  int64_t ncol = 1LL << dim;
  int64_t base = 0;
  for (int col = 0; col < ncol; ++col) {
    nb->color_off[col] = base;
    k_color_flags<<<nblocks(nc, 256), 256, 0, s>>>(cnt, g, nc, col, flag);
    SPH_LAUNCH_CHECK();
    if ((rc_ = scan_exclusive(flag, pos, nc, pos + nc, s))) return rc_;
    k_color_emit<<<nblocks(nc, 256), 256, 0, s>>>(cnt, flag, pos, nc, base, nb->akey, acnt);
    SPH_LAUNCH_CHECK();
    int64_t tot = 0;
    SPH_HIP(hipMemcpyAsync(&tot, pos + nc, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    base += tot;
  }
  for (int col = (int)ncol; col < 9; ++col) nb->color_off[col] = base;
  nb->n_anchors = base;
  unsigned long long hbmax = 0;
  SPH_HIP(hipMemcpyAsync(&hbmax, dmax, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  if ((rc_ = dalloc(&nb->aoff, base + 1))) return rc_;
  if ((rc_ = scan_exclusive(acnt, nb->aoff, base, nb->aoff + base, s))) return rc_;
  int64_t npu = 0;
  SPH_HIP(hipMemcpyAsync(&npu, nb->aoff + base, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  hipFree(cnt);
  hipFree(flag);
  hipFree(pos);
  hipFree(acnt);
  if (npu != nb->n_upairs) {
    set_error("schedule pair count %lld != %lld", (long long)npu, (long long)nb->n_upairs);
    return SPH_E_DEVICE;
  }
  uint32_t *ta = nullptr, *tb = nullptr, *tl = nullptr;
  if ((rc_ = dalloc(&nb->sa, npu)) || (rc_ = dalloc(&nb->sb, npu)) || (rc_ = dalloc(&nb->slev, npu)) ||
      (rc_ = dalloc(&nb->anlev, base)) || (rc_ = dalloc(&ta, npu)) || (rc_ = dalloc(&tb, npu)) ||
      (rc_ = dalloc(&tl, npu)))
    return rc_;
  const int words = (int)((2 * nb->max_deg) / 64 + 1);
  const int64_t bmax = std::max<int64_t>((int64_t)hbmax, 1);
  const int64_t batch = std::max<int64_t>(1, std::min<int64_t>(16384, (int64_t)(512ll << 20) /
                                                                          (bmax * words * 8)));
  unsigned long long* scratch = nullptr;
  if ((rc_ = dalloc(&scratch, batch * bmax * words))) return rc_;
  SPH_HIP(hipMemsetAsync(dmax, 0, 4 * sizeof(unsigned long long), s));
  for (int64_t a0 = 0; a0 < base; a0 += batch) {
    int64_t a1 = std::min(base, a0 + batch);
    k_sched_fill<<<nblocks(a1 - a0, 64), 64, 0, s>>>(
        nb->key, nb->cell_start, nb->nbr_off, nb->nbr_idx, g, nb->akey, nb->aoff, a0, a1, words,
        bmax, scratch, ta, tb, tl, nb->sa, nb->sb, nb->slev, nb->anlev, dmax, dstat + 1);
    SPH_LAUNCH_CHECK();
  }
  unsigned long long hmaxlev = 0;
  int32_t herr = 0;
  SPH_HIP(hipMemcpyAsync(&hmaxlev, dmax, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipMemcpyAsync(&herr, dstat + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  hipFree(scratch);
  hipFree(ta);
  hipFree(tb);
  hipFree(tl);
  hipFree(dmax);
  hipFree(dstat);
  if (herr) {
    set_error("schedule builder failed (code %d)", herr);
    return SPH_E_CAPACITY;
  }
  nb->max_level = (int64_t)hmaxlev;

  // damping pairs packed inside their anchor blocks
  {
    unsigned long long* mx = nullptr;
    int32_t* derr = nullptr;
    if ((rc_ = dalloc(&nb->dpair, npu)) ||
        (rc_ = dalloc(&nb->dgeo32, npu)) || (rc_ = dalloc(&nb->dgeo64, npu)) ||
        (rc_ = dalloc(&nb->ablk, 8 * std::max<int64_t>(base, 1))) ||
        (rc_ = dalloc(&mx, 16)) || (rc_ = dalloc(&derr, 1)))
      return rc_;
    SPH_HIP(hipMemsetAsync(mx, 0, 16 * sizeof(unsigned long long), s));
    SPH_HIP(hipMemsetAsync(derr, 0, sizeof(int32_t), s));
    if (base > 0) {
      k_damp_pack<<<nblocks(base, 64), 64, 0, s>>>(
          nb->akey, nb->aoff, nb->sa, nb->sb, nb->slev, nb->cell_start, nb->X, nb->V, nb->inv_h,
          nb->c5, g, n, base, nb->dpair, nb->dgeo32, nb->dgeo64, nb->ablk, mx, mx + 8,
          derr);
      SPH_LAUNCH_CHECK();
    }
    unsigned long long hm[16] = {0};
    int32_t he = 0;
    SPH_HIP(hipMemcpyAsync(hm, mx, 16 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipMemcpyAsync(&he, derr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    hipFree(mx);
    hipFree(derr);
    if (he) {
      set_error("damping schedule exceeds %d block particles or %d levels", kDampMaxLocal,
                kDampMaxLevel);
      return SPH_E_CAPACITY;
    }
    nb->damp_block_max = 0;
    nb->damp_pairs_max = 0;
    for (int c = 0; c < 8; ++c) {
      nb->damp_bmax[c] = (int64_t)hm[c];
      nb->damp_pmax[c] = (int64_t)hm[8 + c];
      nb->damp_block_max = std::max(nb->damp_block_max, nb->damp_bmax[c]);
      nb->damp_pairs_max = std::max(nb->damp_pairs_max, nb->damp_pmax[c]);
    }
    // LDS of one anchor in the FP64 sweep: its block (v, inverse mass) and a
    // spare slot, addressed by 16-bit byte offsets
    const int64_t need = (nb->damp_block_max + 1) * (4 * 8);
    if (need > std::min<int64_t>(kDampLdsBudget, 65536) || nb->damp_pairs_max > 65535) {
      set_error("an anchor block needs %lld B of LDS for the damping sweep (limit %lld): "
                "neighbourhoods this dense are not supported", (long long)need,
                (long long)kDampLdsBudget);
      return SPH_E_CAPACITY;
    }
    // per-anchor level offsets
    int64_t* lcnt = nullptr;
    int64_t* lbase = nullptr;
    if ((rc_ = dalloc(&lcnt, base + 1)) || (rc_ = dalloc(&lbase, base + 1)) ||
        (rc_ = dalloc(&nb->dloff_base, std::max<int64_t>(base, 1))))
      return rc_;
    if (base > 0) {
      k_lev_count<<<nblocks(base, 256), 256, 0, s>>>(nb->anlev, base, lcnt);
      SPH_LAUNCH_CHECK();
    }
    if ((rc_ = scan_exclusive(lcnt, lbase, base, lbase + base, s))) return rc_;
    int64_t nloff = 0;
    SPH_HIP(hipMemcpyAsync(&nloff, lbase + base, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    if ((rc_ = dalloc(&nb->dloff, nloff))) return rc_;
    if (base > 0) {
      k_lev_fill<<<nblocks(base, 64), 64, 0, s>>>(nb->aoff, nb->slev, lbase, base, nb->dloff,
                                                  nb->dloff_base);
      SPH_LAUNCH_CHECK();
    }
    if ((rc_ = build_joint_rows(nb, s))) return rc_;
    // first pair of every colour
    for (int c = 0; c < 9; ++c) {
      const int64_t a = std::min<int64_t>(nb->color_off[c], base);
      SPH_HIP(hipMemcpy(&nb->damp_pair_off[c], nb->aoff + a, sizeof(int64_t), hipMemcpyDeviceToHost));
    }
    SPH_HIP(hipStreamSynchronize(s));
    hipFree(lcnt);
    hipFree(lbase);
  }

  // row tiles for the LDS-staged gathers, one tiling per precision
  {
    std::vector<uint32_t> hcs(nb->n_cells + 1);
    std::vector<int64_t> hoff(n + 1);
    SPH_HIP(hipMemcpyAsync(hcs.data(), nb->cell_start, (nb->n_cells + 1) * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
    SPH_HIP(hipMemcpyAsync(hoff.data(), nb->nbr_off, (n + 1) * sizeof(int64_t),
                           hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    int32_t* terr = nullptr;
    if ((rc_ = dalloc(&terr, 1))) return rc_;
    for (int prec = 0; prec < 2; ++prec) {
      Tiling& T = nb->tiling[prec];
      T.tmax = tile_tmax(prec);
      std::vector<TileDesc> tv;
      std::vector<uint32_t> ts;
      rc_ = plan_tiles(nb, hcs, hoff, T.tmax, tile_wmax(prec, dim), tile_wmax_hard(prec, dim), tv,
                       ts, T.window_max, T.ell_len);
      if (rc_) {
        hipFree(terr);
        set_error("tile planning failed (a cell row window exceeds the LDS budget)");
        return rc_;
      }
      T.n_tiles = (int64_t)tv.size();
      if ((rc_ = dalloc(&T.tiles, T.n_tiles)) || (rc_ = dalloc(&T.ell, T.ell_len)) ||
          (rc_ = dalloc(&T.tslot, std::max<int64_t>((int64_t)ts.size(), 1))))
        return rc_;
      SPH_HIP(hipMemcpyAsync(T.tiles, tv.data(), T.n_tiles * sizeof(TileDesc),
                             hipMemcpyHostToDevice, s));
      if (!ts.empty())
        SPH_HIP(hipMemcpyAsync(T.tslot, ts.data(), ts.size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice, s));
      SPH_HIP(hipMemsetAsync(terr, 0, sizeof(int32_t), s));
      if (T.n_tiles > 0) {
        k_tile_ell<<<(unsigned)T.n_tiles, 128, 0, s>>>(T.tiles, T.tslot, nb->nbr_off, nb->nbr_idx,
                                                       T.tmax, T.ell, terr);
        SPH_LAUNCH_CHECK();
      }
      int32_t he = 0;
      SPH_HIP(hipMemcpyAsync(&he, terr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      SPH_HIP(hipStreamSynchronize(s));
      if (he) {
        hipFree(terr);
        set_error("tile ELL build failed (code %d)", he);
        return SPH_E_DEVICE;
      }
    }
    // the kernel-gradient sums of both precisions, with the tiled gathers'
    // arithmetic
    if ((rc_ = dalloc(&nb->gsum, dim * n)) || (rc_ = dalloc(&nb->gsumf, dim * n)) ||
        (rc_ = tile_gsum(nb, s))) {
      hipFree(terr);
      return rc_;
    }
    hipFree(terr);
  }

  // inner-loop control block
  SPH_HIP(hipMalloc(&nb->ctrl, sizeof(Ctrl)));
  SPH_HIP(hipMemsetAsync(nb->ctrl, 0, sizeof(Ctrl), s));
  SPH_HIP(hipHostMalloc((void**)&nb->ctrl_host, sizeof(Ctrl), hipHostMallocDefault));
  // per-workgroup partial sums of the parameter gradients (reverse mode)
  {
    int64_t slots = (n + kDiffPerBlock - 1) / kDiffPerBlock;
    for (int prec = 0; prec < 2; ++prec)
      slots = std::max<int64_t>(slots, 8 * ((nb->tiling[prec].n_tiles + 7) / 8));
    nb->gpart_slots = std::max<int64_t>(slots, 1);
  }
  // the per-step scratch, in one block of the handle's own
  int64_t off[kWsParts + 1];
  SPH_HIP(hipMalloc(&nb->ws_own, ws_layout(nb, off)));
  if ((rc_ = ws_attach(nb, static_cast<char*>(nb->ws_own), s))) return rc_;
  SPH_HIP(hipStreamSynchronize(s));
  return SPH_OK;
}

}  // namespace sph

using namespace sph;

static int build_entry(int dim, int64_t n, const double* X, const double* V, double h,
                       int32_t n_spec, const int32_t* spec_id, void* stream, sph_nbr** out) {
  clear_error();
  if (!out) {
    set_error("out is NULL");
    return SPH_E_ARG;
  }
  *out = nullptr;
  if (dim != 2 && dim != 3) {
    set_error("dim must be 2 or 3");
    return SPH_E_UNSUPPORTED;
  }
  if (n < 1 || !X || !V || !(h > 0.0) || !std::isfinite(h)) {
    set_error("bad arguments (n=%lld, h=%g)", (long long)n, h);
    return SPH_E_ARG;
  }
  if (n_spec < 1 || (n_spec > 1 && !spec_id) || n_spec > n) {
    set_error("bad specimen count %d", n_spec);
    return SPH_E_ARG;
  }
  if (n_spec > 65535) {
    set_error("at most 65535 specimens");
    return SPH_E_CAPACITY;
  }
  sph_nbr* nb = new sph_nbr();
  hipStream_t s = (hipStream_t)stream;
  int rc = build(dim, n, X, V, h, n_spec, n_spec > 1 ? spec_id : nullptr, s, nb);
  if (rc == SPH_OK && n_spec > 1) rc = batch_finish(nb, n_spec, spec_id, s);
  if (rc != SPH_OK) {
    hipStreamSynchronize(s);
    free_nbr(nb);
    return rc;
  }
  *out = nb;
  return SPH_OK;
}

extern "C" int sph_build_neighbors(int dim, int64_t n, const double* X, const double* V, double h,
                                   void* stream, sph_nbr** out) {
  return build_entry(dim, n, X, V, h, 1, nullptr, stream, out);
}

extern "C" int sph_build_neighbors_batched(int dim, int64_t n, const double* X, const double* V,
                                           double h, int32_t n_spec, const int32_t* spec_id,
                                           void* stream, sph_nbr** out) {
  if (n_spec > 1 && !spec_id) {
    clear_error();
    set_error("spec_id is NULL");
    return SPH_E_ARG;
  }
  return build_entry(dim, n, X, V, h, n_spec, spec_id, stream, out);
}

extern "C" int sph_nbr_destroy(sph_nbr* nb) {
  if (!nb) return SPH_OK;
  hipDeviceSynchronize();
  free_nbr(nb);
  return SPH_OK;
}

extern "C" int sph_workspace_size(const sph_nbr* nb, int64_t* bytes) {
  clear_error();
  if (!nb || !bytes) {
    set_error("null argument");
    return SPH_E_ARG;
  }
  int64_t off[kWsParts + 1];
  *bytes = ws_layout(nb, off);
  return SPH_OK;
}

extern "C" int sph_set_workspace(sph_nbr* nb, void* ws, int64_t bytes, void* stream) {
  clear_error();
  if (!nb) {
    set_error("null handle");
    return SPH_E_ARG;
  }
  int64_t off[kWsParts + 1];
  const int64_t need = ws_layout(nb, off);
  if (ws && (bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255u))) {
    set_error("workspace of %lld bytes at %p: need %lld bytes at a 256-byte boundary",
              (long long)bytes, ws, (long long)need);
    return SPH_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  SPH_HIP(hipStreamSynchronize(s));
  SPH_HIP(hipDeviceSynchronize());
  free_graph_cache(nb);  // its launches hold the old scratch addresses
  char* base = static_cast<char*>(ws);
  if (ws) {
    if (nb->ws_own) {
      SPH_HIP(hipFree(nb->ws_own));
      nb->ws_own = nullptr;
    }
  } else {
    if (!nb->ws_own) SPH_HIP(hipMalloc(&nb->ws_own, need));
    base = static_cast<char*>(nb->ws_own);
  }
  int rc = ws_attach(nb, base, s);
  if (rc) return rc;
  SPH_HIP(hipStreamSynchronize(s));
  return SPH_OK;
}

extern "C" int sph_nbr_query(const sph_nbr* nb, sph_nbr_info* info) {
  if (!nb || !info) {
    set_error("null argument");
    return SPH_E_ARG;
  }
  std::memset(info, 0, sizeof(*info));
  info->dim = nb->dim;
  info->n_colors = 1 << nb->dim;
  info->n = nb->n;
  info->n_pairs = nb->n_pairs;
  info->n_upairs = nb->n_upairs;
  info->n_cells = nb->n_cells;
  for (int k = 0; k < 3; ++k) {
    info->ncell[k] = nb->nc[k];
    info->origin[k] = nb->origin[k];
  }
  info->n_anchors = nb->n_anchors;
  info->max_deg = nb->max_deg;
  info->max_level = nb->max_level;
  for (int k = 0; k < 9; ++k) info->color_off[k] = nb->color_off[k];
  info->h = nb->h;
  info->inv_rc = nb->inv_rc;
  info->key = nb->key;
  info->perm = nb->perm;
  info->cell_start = nb->cell_start;
  info->nbr_off = nb->nbr_off;
  info->nbr_idx = nb->nbr_idx;
  info->X = nb->X;
  info->V = nb->V;
  info->B0 = nb->B0;
  info->sched_a = nb->sa;
  info->sched_b = nb->sb;
  info->sched_level = nb->slev;
  info->anchor_key = nb->akey;
  info->anchor_off = nb->aoff;
  info->anchor_nlev = nb->anlev;
  return SPH_OK;
}

extern "C" const char* sph_last_error(void) { return sph::g_err.c_str(); }
