// qv_filter.hip -- batched Bayes filter step on gfx950 (Sec. III, posterior
// belief update): prediction through the slip stencil, the likelihood of
// the given observation, and normalisation.  Two passes over bands of rows:
// the first reduces P(z|b,a) per (belief, band) into the workspace, the
// second sums those partials in band order and writes the posterior.
#include <algorithm>

#include "qv_internal.h"

namespace qv {

// Rows y0-1 .. y0+th of b into LDS; off-grid, blocked and goal cells are zero
// (none of them sends mass to a neighbour).
__device__ __forceinline__ void load_fband(const DevModel &m, const uint32_t *sig,
                                           const float *b, int y0, int th, float *band,
                                           int BW) {
  const int n = (th + 2) * BW;
  const float rBW = 1.0f / (float)BW;
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const int r = fdiv(i, BW, rBW);
    const int gy = y0 - 1 + r, gx = i - r * BW - 1;
    float v = 0.f;
    if (gy >= 0 && gy < m.H && gx >= 0 && gx < m.W) {
      const int s = gy * m.W + gx;
      if ((sig[s] & (kSigFree | kSigGoal)) == kSigFree) v = b[s];
    }
    band[i] = v;
  }
}

__device__ __forceinline__ float fpredict(const DevModel &m, const float *band, int BW, int ly,
                                          int lx, uint32_t sg, const float *sl,
                                          const float *stay_a, const float *b, int t) {
  if (!(sg & kSigFree)) return 0.f;
  const float *c = band + (ly + 1) * BW + lx + 1;
  if (sg & kSigGoal) return stencil(c, BW, sl, 1.f, b[t]);
  return stencil(c, BW, sl, stay_a[sig_out8(sg)], c[0]);
}

__device__ __forceinline__ bool bu_item_ok(const DevModel &m, int a, int z) {
  return a >= 0 && a < m.A && z >= 0 && z < 16 * (m.L + 1);
}

__global__ __launch_bounds__(kBlock) void k_bu_lik(DevModel m, const uint32_t *sig,
                                                   const float *staytab, int TH, int tiles,
                                                   const float *b, const int32_t *acts,
                                                   const int32_t *obs, float *part,
                                                   int32_t *err) {
  extern __shared__ float smem[];
  __shared__ float red[kBlock / kWave];
  const int item = blockIdx.x / tiles, tile = blockIdx.x - item * tiles;
  const int a = acts[item], z = obs[item];
  if (!bu_item_ok(m, a, z)) {
    if (tile == 0 && threadIdx.x == 0) atomicOr(err, 4);
    return;
  }
  const int W = m.W, BW = W + 2;
  const int y0 = tile * TH, th = min(TH, m.H - y0);
  const float *bi = b + (size_t)item * m.S;
  float *band = smem;
  load_fband(m, sig, bi, y0, th, band, BW);
  __syncthreads();
  const float rW = 1.0f / (float)W;
  const float *sl = &m.slip[a * 9];
  const float *stay_a = staytab + a * 256;
  const uint32_t zw = (uint32_t)(z & 15), zl = (uint32_t)(z >> 4);
  float acc = 0.f;
  for (int i = threadIdx.x; i < th * W; i += kBlock) {
    const int ly = fdiv(i, W, rW), lx = i - ly * W;
    const int t = (y0 + ly) * W + lx;
    const uint32_t sg = sig[t];
    const float bp = fpredict(m, band, BW, ly, lx, sg, sl, stay_a, bi, t);
    const float o = wall_lik(m.flip, zw, sig_wall(sg)) * lm_lik(m.lm_p, zl, sig_lm(sg));
    acc = fmaf(o, bp, acc);
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int w = 0; w < kBlock / kWave; ++w) s += red[w];
    part[(size_t)item * tiles + tile] = s;
  }
}

__global__ __launch_bounds__(kBlock) void k_bu_write(DevModel m, const uint32_t *sig,
                                                     const float *staytab, int TH, int tiles,
                                                     const float *b, const int32_t *acts,
                                                     const int32_t *obs, const float *part,
                                                     float *b_out, float *p_out,
                                                     int32_t *err) {
  extern __shared__ float smem[];
  const int item = blockIdx.x / tiles, tile = blockIdx.x - item * tiles;
  const int a = acts[item], z = obs[item];
  if (!bu_item_ok(m, a, z)) {
    if (tile == 0 && threadIdx.x == 0) p_out[item] = 0.f;
    return;
  }
  float p = 0.f;
  for (int t = 0; t < tiles; ++t) p += part[(size_t)item * tiles + t];
  if (tile == 0 && threadIdx.x == 0) {
    p_out[item] = p;
    if (!(p > 0.f)) atomicOr(err, 8);
  }
  if (!(p > 0.f)) return;
  const float inv = 1.0f / p;
  const int W = m.W, BW = W + 2;
  const int y0 = tile * TH, th = min(TH, m.H - y0);
  const float *bi = b + (size_t)item * m.S;
  float *band = smem;
  load_fband(m, sig, bi, y0, th, band, BW);
  __syncthreads();
  const float rW = 1.0f / (float)W;
  const float *sl = &m.slip[a * 9];
  const float *stay_a = staytab + a * 256;
  const uint32_t zw = (uint32_t)(z & 15), zl = (uint32_t)(z >> 4);
  float *bo = b_out + (size_t)item * m.S;
  for (int i = threadIdx.x; i < th * W; i += kBlock) {
    const int ly = fdiv(i, W, rW), lx = i - ly * W;
    const int t = (y0 + ly) * W + lx;
    const uint32_t sg = sig[t];
    const float bp = fpredict(m, band, BW, ly, lx, sg, sl, stay_a, bi, t);
    const float o = wall_lik(m.flip, zw, sig_wall(sg)) * lm_lik(m.lm_p, zl, sig_lm(sg));
    bo[t] = o * bp * inv;
  }
}

size_t belief_update_ws(const qv_model *m, int batch) {
  const size_t S = (size_t)m->W * m->H;
  const int TH = tile_rows(m->W, m->H);
  const int tiles = (m->H + TH - 1) / TH;
  size_t off = 0;
  off += align_up(S * 4, 256);                        // sig
  off += align_up((size_t)m->A * 256 * 4, 256);       // staytab
  off += align_up((size_t)batch * tiles * 4, 256);    // partial likelihoods
  off += 256;                                         // err
  return off;
}

hipError_t launch_belief_update(const DevModel &m, int batch, const float *b,
                                const int32_t *a, const int32_t *z, float *b_out,
                                float *p_out, char *ws, hipStream_t st) {
  const size_t S = (size_t)m.S;
  const int TH = tile_rows(m.W, m.H);
  const int tiles = (m.H + TH - 1) / TH;
  size_t off = 0;
  uint32_t *sig = (uint32_t *)(ws + off);
  off += align_up(S * 4, 256);
  float *staytab = (float *)(ws + off);
  off += align_up((size_t)m.A * 256 * 4, 256);
  float *part = (float *)(ws + off);
  off += align_up((size_t)batch * tiles * 4, 256);
  int32_t *err = (int32_t *)(ws + off);
  hipError_t e = launch_prep(m, sig, staytab, err, st);
  if (e != hipSuccess) return e;
  if (batch == 0) return hipSuccess;
  const size_t lds = (size_t)(TH + 2) * (m.W + 2) * sizeof(float);
  const dim3 grid((unsigned)((size_t)batch * tiles));
  QV_LAUNCH(k_bu_lik, grid, dim3(kBlock), lds, st, m, sig, staytab, TH, tiles, b, a, z,
                     part, err);
  QV_LAUNCH(k_bu_write, grid, dim3(kBlock), lds, st, m, sig, staytab, TH, tiles, b, a,
                     z, part, b_out, p_out, err);
  return hipGetLastError();
}

}  // namespace qv
