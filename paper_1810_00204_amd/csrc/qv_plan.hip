// qv_plan.hip -- level-synchronous QV-tree expansion on gfx950.
//
// One planning step builds the depth-D tree of Alg. 1-7 (Sec. IV-C) one
// frontier at a time.  For every level d < D, over all capacity slots of
// the level at once:
//   k_stats    predicted belief b' = T_a^T b per action (slip stencil, Sec. V)
//              reduced to a 16-bin histogram by true wall reading, the
//              predicted mass on each landmark cell, and R(b,a) (Sec. III);
//   k_sample   P(z|b,a) over all z from those sums, n inverse-CDF draws with
//              Philox uniforms (Alg. 3/4), distinct z with frequencies;
//   k_update   child beliefs Phi(b,a,z) (posterior belief update, Sec. III)
//              written to HBM for the next level, or at d = D-1
//   k_leaf     the same posterior values scored on the fly against the
//              Q-MDP vectors, sum_s b(s) Q(s,a') (Alg. 5), never stored.
// Then k_leaf_reduce and k_backup run the expectimax backup (Alg. 6/7).
// Beliefs stream through LDS in bands of whole rows with a one-cell halo.
#include <algorithm>

#include "qv_internal.h"

namespace qv {

// ---------------------------------------------------------------------------
// map signature and stay table
// ---------------------------------------------------------------------------
// root != nullptr: also define the root's records (valid, no observation)
struct RootRecords {
  int32_t *valid, *z, *count;
  float *pz;
};

__global__ void k_prep_sig(DevModel m, uint32_t *sig, float *staytab, int32_t *err,
                           RootRecords root) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0) {
    err[0] = 0;
    if (root.valid) {
      root.valid[0] = 1;
      root.z[0] = -1;
      root.count[0] = 0;
      root.pz[0] = 0.f;
    }
  }
  if (s < m.A * 256) {
    // stay(a, pattern): T'(a,4) plus the slip mass of every move whose
    // target is blocked or off-grid (bit clear in the 8-neighbour pattern)
    const int a = s >> 8, pat = s & 255;
    float st = m.slip[a * 9 + 4];
    int bit = 0;
    for (int k = 0; k < 9; ++k) {
      if (k == 4) continue;
      if (!((pat >> bit) & 1)) st += m.slip[a * 9 + k];
      ++bit;
    }
    staytab[s] = st;
  }
  if (s >= m.S) return;
  const int y = s / m.W, x = s - y * m.W;
  uint32_t v = 0;
  int bit = 0;
  for (int k = 0; k < 9; ++k) {
    if (k == 4) continue;
    const int ny = y + k / 3 - 1, nx = x + k % 3 - 1;
    const bool ok = ny >= 0 && ny < m.H && nx >= 0 && nx < m.W && m.occ[ny * m.W + nx] == 0;
    if (ok) v |= 1u << bit;
    ++bit;
  }
  if (m.occ[s] == 0) v |= kSigFree;
  if (s == m.goal) v |= kSigGoal;
  // wall bits up/left/right/down are neighbours k = 1, 3, 5, 7 -> bits 1, 3, 4, 6
  const uint32_t w = (((v >> 1) & 1u) ^ 1u) | ((((v >> 3) & 1u) ^ 1u) << 1) |
                     ((((v >> 4) & 1u) ^ 1u) << 2) | ((((v >> 6) & 1u) ^ 1u) << 3);
  sig[s] = v | (w << 10);
}

__global__ void k_prep_landmarks(DevModel m, uint32_t *sig, int32_t *err) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= m.L) return;
  const int c = m.lm_cell[l];
  if (c < 0 || c >= m.S) {
    atomicOr(err, 1);
    return;
  }
  // a cell carries at most one landmark id: a second one is refused and flagged
  uint32_t cur = sig[c];
  while (sig_lm(cur) == 0u) {
    const uint32_t prev = atomicCAS(&sig[c], cur, cur | ((uint32_t)(l + 1) << 14));
    if (prev == cur) return;
    cur = prev;
  }
  atomicOr(err, 2);
}

hipError_t launch_prep(const DevModel &dm, uint32_t *sig, float *staytab, int32_t *err,
                       hipStream_t st) {
  const int n = std::max(dm.S, dm.A * 256);
  const RootRecords none = {nullptr, nullptr, nullptr, nullptr};
  QV_LAUNCH(k_prep_sig, dim3((n + 255) / 256), dim3(256), 0, st, dm, sig, staytab,
                     err, none);
  if (dm.L > 0)
    QV_LAUNCH(k_prep_landmarks, dim3((dm.L + 255) / 256), dim3(256), 0, st, dm, sig,
                       err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// shared pieces of the tiled kernels
// ---------------------------------------------------------------------------

// Rows y0-1 .. y0+th of belief b, columns -1 .. W, into LDS (pitch BW=W+2).
// Off-grid, blocked and goal cells read as zero: none of them is a source of
// moving mass (the goal is absorbing and keeps its own mass).
__device__ __forceinline__ void load_band(const DevModel &m, const uint32_t *sig,
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

// b'(t) for cell t = (y0+ly)*W + lx of the tile.
__device__ __forceinline__ float predict_cell(const DevModel &m, const float *band, int BW,
                                              int ly, int lx, uint32_t sg, const float *sl,
                                              const float *stay_a, const float *b, int t) {
  if (!(sg & kSigFree)) return 0.f;
  const float *c = band + (ly + 1) * BW + lx + 1;
  float stay, self;
  if (sg & kSigGoal) {
    stay = 1.f;
    self = b[t];
  } else {
    stay = stay_a[sig_out8(sg)];
    self = c[0];
  }
  return stencil(c, BW, sl, stay, self);
}

// Sum NV per-thread values over the workgroup; thread i < NV gets the total
// of value i (fixed order: wavefront butterfly, then waves 0..3).
template <int NV>
__device__ __forceinline__ float block_sum_to_thread(float (&v)[NV], float *red) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const float s = wave_sum(v[i]);
    if (lane == 0) red[wave * NV + i] = s;
  }
  __syncthreads();
  float out = 0.f;
  if (threadIdx.x < NV) {
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) out += red[w * NV + threadIdx.x];
  }
  __syncthreads();
  return out;
}

// ---------------------------------------------------------------------------
// k_stats: per (parent slot, tile)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_stats(DevModel m, LevelArgs lv) {
  extern __shared__ float smem[];
  const int p = blockIdx.x / lv.tiles;
  const int tile = blockIdx.x - p * lv.tiles;
  if (!lv.pvalid[p]) return;
  const int W = m.W, BW = W + 2, A = m.A;
  const int y0 = tile * lv.TH;
  const int th = min(lv.TH, m.H - y0);
  float *band = smem;
  float *hist = band + (lv.TH + 2) * BW;   // [16][kBlock], per-thread bins
  float *red = hist + 16 * kBlock;         // [4][QV_MAX_ACTIONS]
  const float *b = lv.pbel + (size_t)p * m.S;
  load_band(m, lv.sig, b, y0, th, band, BW);
  __syncthreads();
  const int tid = threadIdx.x;
  const int ncell = th * W;
  const float rW = 1.0f / (float)W;
  float *part = lv.part + (size_t)p * A * lv.tiles * 17;

  // R(b,a) = sum_x R(x,a) b(x) for every action (Sec. III)
  float racc[QV_MAX_ACTIONS];
#pragma unroll
  for (int a = 0; a < QV_MAX_ACTIONS; ++a) racc[a] = 0.f;
  for (int i = tid; i < ncell; i += kBlock) {
    const int t = y0 * W + i;
    const float bt = b[t];
    const float *Rr = m.R + (size_t)t * A;
#pragma unroll
    for (int a = 0; a < QV_MAX_ACTIONS; ++a)
      if (a < A) racc[a] = fmaf(bt, Rr[a], racc[a]);
  }
  {
    const float tot = block_sum_to_thread<QV_MAX_ACTIONS>(racc, red);
    if (tid < A) part[((size_t)tid * lv.tiles + tile) * 17 + 16] = tot;
  }

  const float rho = m.lm_p;
  for (int a = 0; a < A; ++a) {
    const float *sl = &m.slip[a * 9];
    const float *stay_a = lv.staytab + a * 256;
    float h0 = 0.f;
#pragma unroll
    for (int w = 1; w < 16; ++w) hist[w * kBlock + tid] = 0.f;
    for (int i = tid; i < ncell; i += kBlock) {
      const int ly = fdiv(i, W, rW), lx = i - ly * W;
      const int t = (y0 + ly) * W + lx;
      const uint32_t sg = lv.sig[t];
      const float bp = predict_cell(m, band, BW, ly, lx, sg, sl, stay_a, b, t);
      const uint32_t lm = sig_lm(sg);
      float contrib = bp;
      if (lm && lm <= (uint32_t)m.L) {
        contrib = bp * (1.f - rho);
        lv.lmv[((size_t)p * A + a) * m.L + lm - 1] = bp;
      }
      const uint32_t w = sig_wall(sg);
      if (w == 0u)
        h0 += contrib;
      else
        hist[w * kBlock + tid] += contrib;
    }
    hist[tid] = h0;
    __syncthreads();
    // bin = tid/16 sums 16 consecutive per-thread entries, then 16 lanes combine
    const float *hb = hist + (tid >> 4) * kBlock + (tid & 15) * 16;
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += hb[i];
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
    if ((tid & 15) == 0) part[((size_t)a * lv.tiles + tile) * 17 + (tid >> 4)] = s;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// k_sample: one wavefront per (parent slot, action)
// ---------------------------------------------------------------------------
struct ObsSource {
  float p0;               // lanes 0..15: P(zw, no landmark)
  const float *lmv;       // predicted mass on landmark cells of this (slot, action)
};

// P(z|b,a) for z = zw + 16 zl.  Must be called by every lane of the wave
// (it reads lane zw's no-landmark value with a shuffle).
__device__ __forceinline__ float obs_prob(const DevModel &m, const uint32_t *sig,
                                          const ObsSource &src, int z) {
  const int zw = z & 15, zl = z >> 4;
  const float from_p0 = __shfl(src.p0, zw, kWave);
  if (zl == 0) return from_p0;
  if (zl > m.L) return 0.f;
  const int c = m.lm_cell[zl - 1];
  if (c < 0 || c >= m.S) return 0.f;
  return wall_lik(m.flip, (uint32_t)zw, sig_wall(sig[c])) * m.lm_p * src.lmv[zl - 1];
}

__global__ __launch_bounds__(256) void k_sample(DevModel m, LevelArgs lv) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int idx = blockIdx.x * (256 / kWave) + wave;
  if (idx >= lv.nslots * m.A) return;
  const int p = idx / m.A, a = idx - p * m.A;
  const int n = lv.n;
  const int cb = p * lv.K + a * n;
  if (!lv.pvalid[p]) {
    if (lane < n) {
      lv.cvalid[cb + lane] = 0;
      lv.cz[cb + lane] = -1;
      lv.ccount[cb + lane] = 0;
      lv.cpz[cb + lane] = 0.f;
    }
    return;
  }
  // totals over tiles of the 16 wall bins and of R(b,a), tile order fixed
  float hs = 0.f;
  if (lane < 17) {
    const float *pp = lv.part + (size_t)idx * lv.tiles * 17 + lane;
    for (int t = 0; t < lv.tiles; ++t) hs += pp[t * 17];
  }
  if (lane == 16) lv.reward[idx] = hs;
  // P(zw, no landmark) = sum_w O_w(zw|w) H[w]; landmark cells entered H with
  // their "no landmark" factor already
  ObsSource src;
  src.p0 = 0.f;
  src.lmv = lv.lmv + (size_t)idx * m.L;
  for (int w = 0; w < 16; ++w) {
    const float hw = __shfl(hs, w, kWave);
    src.p0 = fmaf(wall_lik(m.flip, (uint32_t)(lane & 15), (uint32_t)w), hw, src.p0);
  }
  // running totals over z in ascending order: lane j owns z in [j*CH, (j+1)*CH)
  const int Z = 16 * (m.L + 1);
  const int CH = (Z + kWave - 1) / kWave;
  float loc = 0.f;
  for (int j = 0; j < CH; ++j) {
    const int z = lane * CH + j;
    const float v = obs_prob(m, lv.sig, src, min(z, Z - 1));
    loc += (z < Z) ? v : 0.f;
  }
  // exclusive prefix of the lane totals, summed in lane order
  float exc = 0.f, P = 0.f;
  for (int i = 0; i < kWave; ++i) {
    const float s = __shfl(loc, i, kWave);
    if (i == lane) exc = P;
    P += s;
  }
  // n uniforms: Philox counter (a*ceil(n/4) + k/4, slot, level, query), word k%4
  float tgt[QV_MAX_SAMPLES];
  const int ng = (n + 3) / 4;
#pragma unroll
  for (int g = 0; g < QV_MAX_SAMPLES / 4; ++g) {
    if (g < ng) {
      const uint4 r = philox4x32_10(
          make_uint4((uint32_t)(a * ng + g), (uint32_t)p, (uint32_t)lv.d, lv.qid), lv.key0,
          lv.key1);
      tgt[4 * g + 0] = u24(r.x) * P;
      tgt[4 * g + 1] = u24(r.y) * P;
      tgt[4 * g + 2] = u24(r.z) * P;
      tgt[4 * g + 3] = u24(r.w) * P;
    }
  }
  // first z of positive mass whose running total exceeds the target
  constexpr int kNone = 0x7fffffff;
  int cand[QV_MAX_SAMPLES];
#pragma unroll
  for (int k = 0; k < QV_MAX_SAMPLES; ++k) cand[k] = kNone;
  int lastpos = -1;
  float run = 0.f;
  for (int j = 0; j < CH; ++j) {
    const int z = lane * CH + j;
    float v = obs_prob(m, lv.sig, src, min(z, Z - 1));
    if (z >= Z) v = 0.f;
    run += v;
    const float F = exc + run;
    if (v > 0.f) {
      lastpos = z;
#pragma unroll
      for (int k = 0; k < QV_MAX_SAMPLES; ++k)
        if (k < n && cand[k] == kNone && tgt[k] < F) cand[k] = z;
    }
  }
  // the last z of positive mass catches a target that rounding left beyond it
  int lastz = lastpos;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) lastz = max(lastz, __shfl_xor(lastz, o, kWave));
  int zk[QV_MAX_SAMPLES];
  float pk[QV_MAX_SAMPLES];
#pragma unroll
  for (int k = 0; k < QV_MAX_SAMPLES; ++k) {
    if (k < n) {
      int zz = wave_min(cand[k]);
      if (zz == kNone) zz = lastz;
      zk[k] = zz;
      pk[k] = zz >= 0 ? obs_prob(m, lv.sig, src, zz) : 0.f;
    }
  }
  if (lane == 0) {
    // ascending z, then one child per distinct z with its frequency
    for (int i = 1; i < n; ++i)
      for (int j = i; j > 0 && zk[j - 1] > zk[j]; --j) {
        const int tz = zk[j];
        zk[j] = zk[j - 1];
        zk[j - 1] = tz;
        const float tp = pk[j];
        pk[j] = pk[j - 1];
        pk[j - 1] = tp;
      }
    int r = 0;
    for (int i = 0; i < n;) {
      int j = i;
      while (j < n && zk[j] == zk[i]) ++j;
      const bool ok = zk[i] >= 0 && pk[i] > 0.f;
      lv.cvalid[cb + r] = ok ? 1 : 0;
      lv.cz[cb + r] = zk[i];
      lv.ccount[cb + r] = j - i;
      lv.cpz[cb + r] = pk[i];
      r += ok ? 1 : 0;
      i = j;
    }
    for (; r < n; ++r) {
      lv.cvalid[cb + r] = 0;
      lv.cz[cb + r] = -1;
      lv.ccount[cb + r] = 0;
      lv.cpz[cb + r] = 0.f;
    }
  }
}

// ---------------------------------------------------------------------------
// k_update: per (parent slot, tile); writes Phi(b,a,z) for every child
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_update(DevModel m, LevelArgs lv) {
  extern __shared__ float smem[];
  const int p = blockIdx.x / lv.tiles;
  const int tile = blockIdx.x - p * lv.tiles;
  if (!lv.pvalid[p]) return;
  const int W = m.W, BW = W + 2, A = m.A, S = m.S;
  const int y0 = tile * lv.TH;
  const int th = min(lv.TH, m.H - y0);
  float *band = smem;
  const float *b = lv.pbel + (size_t)p * S;
  load_band(m, lv.sig, b, y0, th, band, BW);
  __syncthreads();
  const int ncell = th * W;
  const float rW = 1.0f / (float)W;
  for (int a = 0; a < A; ++a) {
    const int cb = p * lv.K + a * lv.n;
    int U = 0;
    int zr[QV_MAX_SAMPLES];
    float inv[QV_MAX_SAMPLES];
#pragma unroll
    for (int r = 0; r < QV_MAX_SAMPLES; ++r) {
      zr[r] = 0;
      inv[r] = 0.f;
      if (r < lv.n && lv.cvalid[cb + r]) {
        zr[r] = lv.cz[cb + r];
        inv[r] = 1.0f / lv.cpz[cb + r];
        ++U;
      }
    }
    if (U == 0) continue;
    const float *sl = &m.slip[a * 9];
    const float *stay_a = lv.staytab + a * 256;
    for (int i = threadIdx.x; i < ncell; i += kBlock) {
      const int ly = fdiv(i, W, rW), lx = i - ly * W;
      const int t = (y0 + ly) * W + lx;
      const uint32_t sg = lv.sig[t];
      const float bp = predict_cell(m, band, BW, ly, lx, sg, sl, stay_a, b, t);
      const uint32_t w = sig_wall(sg), lm = sig_lm(sg);
#pragma unroll
      for (int r = 0; r < QV_MAX_SAMPLES; ++r) {
        if (r < U) {
          const float o = wall_lik(m.flip, (uint32_t)(zr[r] & 15), w) *
                          lm_lik(m.lm_p, (uint32_t)(zr[r] >> 4), lm);
          lv.cbel[(size_t)(cb + r) * S + t] = o * bp * inv[r];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// k_leaf: per (parent slot, tile) at the last level: each child belief
// value is formed as in k_update and immediately dotted with Q(.,a')
// ---------------------------------------------------------------------------
constexpr int kLeafGroup = 4;

__global__ __launch_bounds__(kBlock) void k_leaf(DevModel m, LevelArgs lv) {
  extern __shared__ float smem[];
  const int p = blockIdx.x / lv.tiles;
  const int tile = blockIdx.x - p * lv.tiles;
  if (!lv.pvalid[p]) return;
  const int W = m.W, BW = W + 2, A = m.A, S = m.S;
  const int y0 = tile * lv.TH;
  const int th = min(lv.TH, m.H - y0);
  float *band = smem;
  float *red = band + (lv.TH + 2) * BW;    // [4][kLeafGroup*QV_MAX_ACTIONS]
  const float *b = lv.pbel + (size_t)p * S;
  load_band(m, lv.sig, b, y0, th, band, BW);
  __syncthreads();
  const int ncell = th * W;
  const float rW = 1.0f / (float)W;
  for (int a = 0; a < A; ++a) {
    const int cb = p * lv.K + a * lv.n;
    int U = 0;
    for (int r = 0; r < lv.n; ++r) U += lv.cvalid[cb + r] ? 1 : 0;
    const float *sl = &m.slip[a * 9];
    const float *stay_a = lv.staytab + a * 256;
    for (int r0 = 0; r0 < U; r0 += kLeafGroup) {
      int zr[kLeafGroup];
      float inv[kLeafGroup];
#pragma unroll
      for (int r = 0; r < kLeafGroup; ++r) {
        zr[r] = 0;
        inv[r] = 0.f;
        if (r0 + r < U) {
          zr[r] = lv.cz[cb + r0 + r];
          inv[r] = 1.0f / lv.cpz[cb + r0 + r];
        }
      }
      float acc[kLeafGroup * QV_MAX_ACTIONS];
#pragma unroll
      for (int i = 0; i < kLeafGroup * QV_MAX_ACTIONS; ++i) acc[i] = 0.f;
      for (int i = threadIdx.x; i < ncell; i += kBlock) {
        const int ly = fdiv(i, W, rW), lx = i - ly * W;
        const int t = (y0 + ly) * W + lx;
        const uint32_t sg = lv.sig[t];
        const float bp = predict_cell(m, band, BW, ly, lx, sg, sl, stay_a, b, t);
        const uint32_t w = sig_wall(sg), lm = sig_lm(sg);
        float q[QV_MAX_ACTIONS];
        const float *Qr = lv.Q + (size_t)t * A;
#pragma unroll
        for (int c = 0; c < QV_MAX_ACTIONS; ++c) q[c] = (c < A) ? Qr[c] : 0.f;
#pragma unroll
        for (int r = 0; r < kLeafGroup; ++r) {
          if (r0 + r < U) {
            const float o = wall_lik(m.flip, (uint32_t)(zr[r] & 15), w) *
                            lm_lik(m.lm_p, (uint32_t)(zr[r] >> 4), lm);
            const float v = o * bp * inv[r];
#pragma unroll
            for (int c = 0; c < QV_MAX_ACTIONS; ++c)
              acc[r * QV_MAX_ACTIONS + c] = fmaf(v, q[c], acc[r * QV_MAX_ACTIONS + c]);
          }
        }
      }
      const float tot = block_sum_to_thread<kLeafGroup * QV_MAX_ACTIONS>(acc, red);
      const int r = threadIdx.x / QV_MAX_ACTIONS, c = threadIdx.x - r * QV_MAX_ACTIONS;
      if (threadIdx.x < kLeafGroup * QV_MAX_ACTIONS && r0 + r < U && c < A)
        lv.leafpart[((size_t)(cb + r0 + r) * lv.tiles + tile) * A + c] = tot;
    }
  }
}

// ---------------------------------------------------------------------------
// k_leaf_score: per (stored leaf slot, tile), sum_s b(s) Q(s,a')
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_leaf_score(DevModel m, const float *bel,
                                                       const int32_t *valid, int tiles, int TH,
                                                       const float *Q, float *leafpart) {
  __shared__ float red[4 * QV_MAX_ACTIONS];
  const int c = blockIdx.x / tiles;
  const int tile = blockIdx.x - c * tiles;
  if (!valid[c]) return;
  const int W = m.W, A = m.A;
  const int y0 = tile * TH;
  const int th = min(TH, m.H - y0);
  const float *b = bel + (size_t)c * m.S;
  float acc[QV_MAX_ACTIONS];
#pragma unroll
  for (int a = 0; a < QV_MAX_ACTIONS; ++a) acc[a] = 0.f;
  for (int i = threadIdx.x; i < th * W; i += kBlock) {
    const int t = y0 * W + i;
    const float v = b[t];
    const float *Qr = Q + (size_t)t * A;
#pragma unroll
    for (int a = 0; a < QV_MAX_ACTIONS; ++a)
      if (a < A) acc[a] = fmaf(v, Qr[a], acc[a]);
  }
  const float tot = block_sum_to_thread<QV_MAX_ACTIONS>(acc, red);
  if (threadIdx.x < A) leafpart[((size_t)c * tiles + tile) * A + threadIdx.x] = tot;
}

// V(leaf) = max_a' sum over tiles (tile order fixed).  With is_root the leaf
// is the root itself (depth 0) and its per-action sums are its Q-values.
__global__ void k_leaf_reduce(const int32_t *valid, int nslots, int tiles, int A,
                              const float *leafpart, float *value, float *qroot) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nslots || !valid[c]) return;
  float best = -INFINITY;
  for (int a = 0; a < A; ++a) {
    float s = 0.f;
    for (int t = 0; t < tiles; ++t) s += leafpart[((size_t)c * tiles + t) * A + a];
    if (qroot) qroot[a] = s;
    best = fmaxf(best, s);
  }
  value[c] = best;
}

// ---------------------------------------------------------------------------
// k_backup: bottom-up expectimax (Alg. 6/7), one workgroup
// ---------------------------------------------------------------------------
struct BackupArgs {
  int D, n, K, A;
  float gamma;
  long long first[QV_MAX_DEPTH + 2];
  long long slots[QV_MAX_DEPTH + 1];
  const int32_t *valid, *count;
  float *value, *qvalue;
  const float *reward;
  int32_t *action_out;
  float *rootQ_out;
};

__global__ __launch_bounds__(1024) void k_backup(BackupArgs g) {
  for (int d = g.D - 1; d >= 0; --d) {
    const long long f = g.first[d], fc = g.first[d + 1];
    const long long npair = g.slots[d] * g.A;
    for (long long i = threadIdx.x; i < npair; i += blockDim.x) {
      const long long s = i / g.A;
      const int a = (int)(i - s * g.A);
      if (!g.valid[f + s]) continue;
      float q = g.reward[(f + s) * g.A + a];
      const long long cb = fc + s * g.K + (long long)a * g.n;
      for (int r = 0; r < g.n; ++r) {
        if (!g.valid[cb + r]) break;
        q += g.gamma * ((float)g.count[cb + r] / (float)g.n) * g.value[cb + r];
      }
      g.qvalue[(f + s) * g.A + a] = q;
    }
    __syncthreads();
    for (long long s = threadIdx.x; s < g.slots[d]; s += blockDim.x) {
      if (!g.valid[f + s]) continue;
      float best = -INFINITY;
      for (int a = 0; a < g.A; ++a) best = fmaxf(best, g.qvalue[(f + s) * g.A + a]);
      g.value[f + s] = best;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    float best = -INFINITY;
    for (int a = 0; a < g.A; ++a) best = fmaxf(best, g.qvalue[a]);
    int act = 0;
    for (int a = 0; a < g.A; ++a)
      if (g.qvalue[a] >= best - 1e-9f) {
        act = a;
        break;
      }
    g.action_out[0] = act;
    for (int a = 0; a < g.A; ++a) g.rootQ_out[a] = g.qvalue[a];
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static size_t band_bytes(int W, int TH) { return (size_t)(TH + 2) * (W + 2) * sizeof(float); }

hipError_t launch_plan(const qv_model *mm, const float *Q, const float *b0, int D, int n,
                       uint64_t seed, uint32_t qid, int flags, int32_t *action_out,
                       float *rootQ_out, char *ws, const PlanLayout &L, hipStream_t st) {
  const DevModel m = make_dev_model(mm);
  const qv_tree_layout &T = L.pub;
  const int A = m.A, K = A * n, S = m.S;
  const int TH = T.tile_rows, tiles = T.tiles;
  const bool store_leaves = (flags & QV_PLAN_STORE_LEAVES) != 0;
  int32_t *valid = (int32_t *)(ws + T.valid);
  int32_t *zrec = (int32_t *)(ws + T.z);
  int32_t *cnt = (int32_t *)(ws + T.count);
  float *pz = (float *)(ws + T.pz);
  float *value = (float *)(ws + T.value);
  float *qvalue = (float *)(ws + T.qvalue);
  float *reward = (float *)(ws + T.reward);
  uint32_t *sig = (uint32_t *)(ws + L.sig);
  float *staytab = (float *)(ws + L.staytab);
  float *part = (float *)(ws + L.part);
  float *lmv = (float *)(ws + L.lmv);
  float *leafpart = (float *)(ws + L.leafpart);
  int32_t *err = (int32_t *)(ws + L.err);

  {
    const int nthr = std::max(S, A * 256);
    const RootRecords root = {valid, zrec, cnt, pz};
    QV_LAUNCH(k_prep_sig, dim3((nthr + 255) / 256), dim3(256), 0, st, m, sig, staytab,
                       err, root);
    if (m.L > 0)
      QV_LAUNCH(k_prep_landmarks, dim3((m.L + 255) / 256), dim3(256), 0, st, m, sig,
                         err);
  }
  const size_t lds_band = band_bytes(m.W, TH);
  const size_t lds_stats = lds_band + 16 * kBlock * sizeof(float) + 4 * QV_MAX_ACTIONS * sizeof(float);
  const size_t lds_leaf = lds_band + 4 * kLeafGroup * QV_MAX_ACTIONS * sizeof(float);
  for (int d = 0; d < D; ++d) {
    LevelArgs lv;
    lv.d = d;
    lv.nslots = (int)T.level_slots[d];
    lv.tiles = tiles;
    lv.TH = TH;
    lv.n = n;
    lv.K = K;
    lv.key0 = (uint32_t)seed;
    lv.key1 = (uint32_t)(seed >> 32);
    lv.qid = qid;
    lv.pbel = d == 0 ? b0 : (const float *)(ws + T.belief_offset[d]);
    lv.pvalid = valid + T.level_first[d];
    lv.part = part;
    lv.lmv = lmv;
    lv.cvalid = valid + T.level_first[d + 1];
    lv.cz = zrec + T.level_first[d + 1];
    lv.ccount = cnt + T.level_first[d + 1];
    lv.cpz = pz + T.level_first[d + 1];
    lv.reward = reward + T.level_first[d] * A;
    const bool last = (d == D - 1);
    lv.cbel = (!last || store_leaves) ? (float *)(ws + T.belief_offset[d + 1]) : nullptr;
    lv.leafpart = leafpart;
    lv.Q = Q;
    lv.sig = sig;
    lv.staytab = staytab;
    const unsigned nblk = (unsigned)(lv.nslots * tiles);
    QV_LAUNCH(k_stats, dim3(nblk), dim3(kBlock), lds_stats, st, m, lv);
    const unsigned nsamp = (unsigned)((lv.nslots * A + 3) / 4);
    QV_LAUNCH(k_sample, dim3(nsamp), dim3(256), 0, st, m, lv);
    if (!last || store_leaves)
      QV_LAUNCH(k_update, dim3(nblk), dim3(kBlock), lds_band, st, m, lv);
    else
      QV_LAUNCH(k_leaf, dim3(nblk), dim3(kBlock), lds_leaf, st, m, lv);
  }
  const long long nleaf = T.level_slots[D];
  const int32_t *lvalid = valid + T.level_first[D];
  if (store_leaves || D == 0) {
    const float *lb = D == 0 ? b0 : (const float *)(ws + T.belief_offset[D]);
    QV_LAUNCH(k_leaf_score, dim3((unsigned)(nleaf * tiles)), dim3(kBlock), 0, st, m, lb,
                       lvalid, tiles, TH, Q, leafpart);
  }
  QV_LAUNCH(k_leaf_reduce, dim3((unsigned)((nleaf + 255) / 256)), dim3(256), 0, st,
                     lvalid, (int)nleaf, tiles, A, leafpart, value + T.level_first[D],
                     D == 0 ? qvalue : (float *)nullptr);
  BackupArgs g;
  g.D = D;
  g.n = n;
  g.K = K;
  g.A = A;
  g.gamma = m.gamma;
  for (int d = 0; d <= D + 1 && d < QV_MAX_DEPTH + 2; ++d) g.first[d] = T.level_first[d];
  for (int d = 0; d <= D; ++d) g.slots[d] = T.level_slots[d];
  g.valid = valid;
  g.count = cnt;
  g.value = value;
  g.qvalue = qvalue;
  g.reward = reward;
  g.action_out = action_out;
  g.rootQ_out = rootQ_out;
  QV_LAUNCH(k_backup, dim3(1), dim3(1024), 0, st, g);
  return hipGetLastError();
}

}  // namespace qv
