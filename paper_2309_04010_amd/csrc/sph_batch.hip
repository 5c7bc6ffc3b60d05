// sph_batch.hip -- batches of independent specimens in one particle set.
//
// The specimens of a parameter sweep share one particle set, one neighbour
// structure, one tiling and one damping schedule, so every kernel runs over
// all of them in a single launch.  Each specimen has its own segment of the
// cell grid (built by sph_build_neighbors_batched), so its cells, sorted
// order, neighbour lists, correction matrices and damping order are those
// of the specimen alone; a tile, an anchor and a neighbour list each belong
// to one specimen.  Kernels look up the per-specimen scalars (mu, K, lambda,
// dt_s, dt_slow, D, eta dt_s) through the specimen id of each sorted particle.
#include <hip/hip_runtime.h>

#include <vector>

#include "sph_common.h"

namespace sph {

__global__ void k_spec_gather(int64_t n, int32_t n_spec, const int32_t* __restrict__ spec_in,
                              const uint32_t* __restrict__ perm, uint16_t* __restrict__ spec,
                              int32_t* err) {
  const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  const int32_t s = spec_in[perm[a]];
  if (s < 0 || s >= n_spec) {
    atomicOr(err, 1);
    spec[a] = 0;
    return;
  }
  spec[a] = (uint16_t)s;
}

// per-specimen sums of the gradient partials: workgroup slots of the tiled
// reverse kernels (each tile lies in one specimen) and per-particle partials
// of the diffusion reverse; fixed order, then cleared
__global__ __launch_bounds__(256) void k_grad_reduce_batched(
    double* __restrict__ gpart, int64_t slots, const TileDesc* __restrict__ tiles, int64_t n_tiles,
    const uint16_t* __restrict__ spec, double* __restrict__ gdiff, int64_t n,
    const int64_t* __restrict__ spec_off, double* __restrict__ out) {
  __shared__ double red[256];
  const int s = blockIdx.x;
  const int64_t per = (n_tiles + 7) / 8;
  const int64_t q0 = spec_off[s], q1 = spec_off[s + 1];
  for (int gi = 0; gi < SPH_NGRAD; ++gi) {
    double acc = 0.0;
    if (gi == SPH_GRAD_D || gi == SPH_GRAD_C) {
      double* g = gdiff + (gi == SPH_GRAD_D ? 0 : n);
      for (int64_t a = q0 + threadIdx.x; a < q1; a += 256) {
        acc += g[a];
        g[a] = 0.0;
      }
    } else {
      for (int64_t j = threadIdx.x; j < slots; j += 256) {
        const int64_t tile = (j & 7) * per + (j >> 3);
        if (tile >= n_tiles || spec[tiles[tile].p0] != s) continue;
        acc += gpart[j * SPH_NGRAD + gi];
        gpart[j * SPH_NGRAD + gi] = 0.0;
      }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0 && out) out[(int64_t)s * SPH_NGRAD + gi] += red[0];
    __syncthreads();
  }
}

int batch_check(const sph_nbr* nb, const sph_multirate_cfg* cfg) {
  const sph_batch* b = cfg->batch;
  if (!b) return SPH_OK;
  if (nb->n_spec == 0 || b->n_spec != nb->n_spec) {
    set_error("cfg->batch has %d specimens, the handle %lld (build it with sph_build_neighbors_batched)", b->n_spec,
              (long long)nb->n_spec);
    return SPH_E_ARG;
  }
  if (!b->E || (cfg->slow_kind != SPH_SLOW_LOAD && !b->D)) {
    set_error("cfg->batch arrays missing");
    return SPH_E_ARG;
  }
  if (cfg->k_sched == nullptr && cfg->fixed_inner <= 0) {
    set_error("a batched run needs fixed inner counts (fixed_inner or k_sched)");
    return SPH_E_ARG;
  }
  return SPH_OK;
}

// per-specimen tables, in both precisions, uploaded before a batched run
int batch_upload(const sph_nbr* nb, const sph_material* m, const sph_multirate_cfg* cfg,
                 hipStream_t s) {
  const sph_batch* b = cfg->batch;
  const int64_t ns = nb->n_spec;
  std::vector<double> t64(BT_COUNT * ns);
  std::vector<float> t32(BT_COUNT * ns);
  for (int64_t i = 0; i < ns; ++i) {
    const double E = b->E[i];
    const double mu = E / (2.0 * (1.0 + m->nu));
    const double K = E / (3.0 * (1.0 - 2.0 * m->nu));
    const double D = b->D ? b->D[i] : cfg->D;
    sph_material mi = *m;
    mi.E = E;
    double dt_rest = 0.0, dt_diff = 0.0;
    rest_steps(nb->h, &mi, D, &dt_rest, &dt_diff);
    const double dt = b->dt_s && b->dt_s[i] > 0.0 ? b->dt_s[i] : dt_rest;
    double dtd = b->dt_slow ? b->dt_slow[i] : 0.0;
    if (!(dtd > 0.0)) dtd = cfg->slow_kind != SPH_SLOW_LOAD ? dt_diff : cfg->dt_slow;
    const double v[BT_COUNT] = {mu, K, K - 2.0 * mu / 3.0, dt, dtd, D, cfg->eta * dt};
    for (int f = 0; f < BT_COUNT; ++f) {
      t64[f * ns + i] = v[f];
      // the same roundings as the uniform path: mu, K, lam and eta dt go to
      // float from double, as the launchers do
      t32[f * ns + i] = (float)v[f];
    }
    if (!(E > 0.0) || !(dt > 0.0) || !(dtd > 0.0)) {
      set_error("specimen %lld: E, dt_s and dt_slow must be positive", (long long)i);
      return SPH_E_ARG;
    }
  }
  SPH_HIP(hipMemcpyAsync(nb->bt64, t64.data(), t64.size() * sizeof(double), hipMemcpyHostToDevice, s));
  SPH_HIP(hipMemcpyAsync(nb->bt32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice, s));
  SPH_HIP(hipStreamSynchronize(s));
  return SPH_OK;
}

int grad_reduce_batched(const sph_nbr* nb, int prec, double* out, hipStream_t s) {
  const Tiling& t = nb->tiling[prec];
  k_grad_reduce_batched<<<(unsigned)nb->n_spec, 256, 0, s>>>(nb->gpart, nb->gpart_slots, t.tiles,
                                                             t.n_tiles, nb->spec, nb->gdiff, nb->n,
                                                             nb->spec_off_dev, out);
  SPH_LAUNCH_CHECK();
  return SPH_OK;
}

// specimen ids of the sorted particles, their ranges, the parameter tables
int batch_finish(sph_nbr* nb, int32_t n_spec, const int32_t* spec_id, hipStream_t s) {
  const int64_t n = nb->n;
  int32_t* err = nullptr;
  SPH_HIP(hipMalloc(&nb->spec, std::max<int64_t>(n, 1) * sizeof(uint16_t)));
  SPH_HIP(hipMalloc(&err, sizeof(int32_t)));
  SPH_HIP(hipMemsetAsync(err, 0, sizeof(int32_t), s));
  k_spec_gather<<<(unsigned)std::max<int64_t>(1, (n + 255) / 256), 256, 0, s>>>(
      n, n_spec, spec_id, nb->perm, nb->spec, err);
  SPH_LAUNCH_CHECK();
  int32_t he = 0;
  SPH_HIP(hipMemcpyAsync(&he, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SPH_HIP(hipStreamSynchronize(s));
  hipFree(err);
  if (he) {
    set_error("specimen id out of range");
    return SPH_E_ARG;
  }
  // specimen k owns cell keys [koff_k, koff_k+1), hence sorted positions
  // [cell_start[koff_k], cell_start[koff_k+1])
  std::vector<int64_t> off(n_spec + 1);
  for (int k = 0; k <= n_spec; ++k) {
    const int64_t key = k < n_spec ? nb->segs[k].koff : nb->n_cells;
    uint32_t v = 0;
    SPH_HIP(hipMemcpy(&v, nb->cell_start + key, sizeof(uint32_t), hipMemcpyDeviceToHost));
    off[k] = v;
  }
  SPH_HIP(hipMalloc(&nb->spec_off_dev, (n_spec + 1) * sizeof(int64_t)));
  SPH_HIP(hipMemcpy(nb->spec_off_dev, off.data(), (n_spec + 1) * sizeof(int64_t),
                    hipMemcpyHostToDevice));
  SPH_HIP(hipMalloc(&nb->bt32, BT_COUNT * n_spec * sizeof(float)));
  SPH_HIP(hipMalloc(&nb->bt64, BT_COUNT * n_spec * sizeof(double)));
  SPH_HIP(hipMalloc(&nb->gdiff, 2 * std::max<int64_t>(n, 1) * sizeof(double)));
  SPH_HIP(hipMemset(nb->gdiff, 0, 2 * std::max<int64_t>(n, 1) * sizeof(double)));
  nb->spec_off = off;
  nb->n_spec = n_spec;
  return SPH_OK;
}

}  // namespace sph
