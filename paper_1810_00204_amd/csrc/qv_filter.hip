// qv_filter.hip -- batched Bayes filter step on gfx950 (Sec. III, posterior
// belief update): prediction through the slip stencil, the likelihood of
// the given observation, and normalisation.  Two passes over bands of rows:
// the first reduces P(z|b,a) per (belief, band) into the workspace, the
// second sums those partials in band order and writes the posterior.
#include <algorithm>
#include <mutex>

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

int32_t belief_update_args(const qv_model *m, int batch, const float *b, const int32_t *a,
                           const int32_t *z, const float *b_out, const float *p_out) {
  const int32_t st = check_model(m);
  if (st != QV_OK) return st;
  if (batch < 0) return QV_ERR_INVALID_ARG;
  if (batch > 0 && (!b || !a || !z || !b_out || !p_out)) return QV_ERR_INVALID_ARG;
  const size_t S = (size_t)m->W * m->H;
  if (batch > 0 && (const void *)b < (const void *)(b_out + (size_t)batch * S) &&
      (const void *)b_out < (const void *)(b + (size_t)batch * S))
    return QV_ERR_INVALID_ARG;
  return QV_OK;
}

int32_t belief_update_run(const qv_model *m, int batch, const float *b, const int32_t *a,
                          const int32_t *z, float *b_out, float *p_out, int check, char *ws,
                          hipStream_t hs) {
  const DevModel dm = make_dev_model(m);
  int32_t st = hip_status(launch_belief_update(dm, batch, b, a, z, b_out, p_out, ws, hs));
  if (st != QV_OK || !check) return st;
  const size_t S = (size_t)m->W * m->H;
  const size_t TH = tile_rows(m->W, m->H);
  const size_t tiles = (m->H + TH - 1) / TH;
  const size_t off = align_up(S * 4, 256) + align_up((size_t)m->A * 256 * 4, 256) +
                     align_up((size_t)batch * tiles * 4, 256);
  int32_t herr = 0;
  st = hip_status(hipMemcpyAsync(&herr, ws + off, 4, hipMemcpyDeviceToHost, hs));
  if (st != QV_OK) return st;
  st = hip_status(hipStreamSynchronize(hs));
  if (st != QV_OK) return st;
  if (herr & (4 | 8)) return QV_ERR_ZERO_LIKELIHOOD;
  if (herr) return QV_ERR_INVALID_ARG;
  return QV_OK;
}

// ---------------------------------------------------------------------------
// Belief update without allocation: the same kernels on a scratch region in
// the library's own device memory instead of a caller workspace.  Each GPU
// holds its own copy of `scratch` for the life of the process; host code
// uses the device address that hipGetSymbolAddress returns for the current
// device, never the array's name (a host-side stand-in).
// ---------------------------------------------------------------------------
constexpr int kBuMaxCells = 1 << 20;     // S = W*H at most
constexpr int kBuMaxParts = 1 << 14;     // batch * bands at most
constexpr size_t kBuScratchBytes =
    ((size_t)kBuMaxCells * 4) + ((size_t)QV_MAX_ACTIONS * 256 * 4 + 256) +
    ((size_t)kBuMaxParts * 4) + 256;
static __device__ __align__(256) char scratch[kBuScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch[kMaxDevices];

// The current device's copy of `scratch` (looked up once per device).
static hipError_t scratch_ptr(char **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *out = (char *)g_scratch[dev];
  return hipSuccess;
}

}  // namespace qv

extern "C" int32_t qv_belief_update_noalloc(const qv_model *m, int32_t batch, const float *b,
                                            const int32_t *a, const int32_t *z, float *b_out,
                                            float *p_out, int32_t check, void *stream) {
  using namespace qv;
  const int32_t st = belief_update_args(m, batch, b, a, z, b_out, p_out);
  if (st != QV_OK) return st;
  const long long S = (long long)m->W * m->H;
  const long long TH = tile_rows(m->W, m->H);
  const long long tiles = (m->H + TH - 1) / TH;
  if (S > kBuMaxCells || (long long)batch * tiles > kBuMaxParts) return QV_ERR_UNSUPPORTED;
  if (belief_update_ws(m, batch) > kBuScratchBytes) return QV_ERR_UNSUPPORTED;
  char *ws = nullptr;
  const int32_t hs = hip_status(scratch_ptr(&ws));
  if (hs != QV_OK) return hs;
  return belief_update_run(m, batch, b, a, z, b_out, p_out, check, ws, (hipStream_t)stream);
}

namespace qv {

// ===========================================================================
// Differentiable filter: negative log-likelihood of logged observations under
// the filter above and its adjoint with respect to the slip logits theta
// (T'(a,.) = softmax(theta[a,.])) and the wall-bit flip logits phi
// (f_j = logistic(phi_j)).  For each trajectory
//   c_t = T_{a_t}^T b_{t-1},  u_t = O(z_t|.) c_t,  eta_t = sum u_t,
//   b_t = u_t / eta_t,  NLL = -sum_t log eta_t,
// and in reverse
//   ubar_t = (lambda_t - <lambda_t, b_t> - 1) / eta_t,  cbar_t = O(z_t|.) ubar_t,
//   lambda_{t-1}(s) = sum_k T'(a_t,k) cbar_t(dest(s,k)),
//   dNLL/dT'(a_t,k) += sum_s b_{t-1}(s) cbar_t(dest(s,k)),
//   dNLL/df_j += sum_s c_t(s) ubar_t(s) dO(z_t|s)/df_j.
// One persistent 1024-thread workgroup per trajectory at a time.  Both bands
// (the belief being propagated and the adjoint source cbar) sit in LDS; each
// thread keeps its cells' b, lambda and c in registers.  Beliefs are stored
// every `k` steps; the reverse sweep recomputes each segment from its stored
// belief into a per-workgroup buffer.  Every sum runs in a fixed order.
// ===========================================================================
constexpr int kFBlock = 1024;
constexpr int kFWaves = kFBlock / kWave;
constexpr int kFGrad = 85;   // 81 slip entries (A*9 used) + 4 flip entries

struct FilterArgs {
  int ntraj, T, k, nseg, G;
  const float *theta, *phi;
  const float *b0;
  int b0_per_traj;
  const int32_t *acts, *obs;
  float *nll;         // [ntraj]
  double *gpart;      // [ntraj][kFGrad]
  float *ckpt;        // [G][nseg][S]   (entry 0 unused: the start belief)
  float *seg;         // [G][k+1][S]
  float *eta;         // [G][T+1]
  const uint32_t *sig;
  int32_t *err;
  int want_grad;
};

// Totals of N per-thread values over the 1024-thread workgroup, in a fixed
// order (DPP within each wavefront, then wavefronts 0..15).  Result i lands in
// out[i] (LDS) for all threads after the call.
template <int N>
__device__ __forceinline__ void fblock_sum(float (&v)[N], float *red /* [16][16] */,
                                           float *out /* [N] */) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = wave_total_lane63(v[i]);
  if (lane == kWave - 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) red[wave * 16 + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x < N) {
    float s = 0.f;
    for (int w = 0; w < kFWaves; ++w) s += red[w * 16 + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kFBlock) void k_filter(DevModel m, FilterArgs fa) {
  extern __shared__ float smem[];
  __shared__ float s_slip[81], s_flip[4];
  __shared__ float s_red[kFWaves * 16];
  __shared__ float s_out[16];
  __shared__ double s_g[kFGrad];
  __shared__ double s_nll;
  __shared__ float s_bgoal;            // own mass of the goal cell (its band entry is 0)
  const int W = m.W, H = m.H, S = m.S, A = m.A, BW = W + 2;
  const int BAND = (H + 2) * BW;
  float *band = smem;                  // forward: belief b_{t-1}; reverse: cbar_t
  float *cell = smem + BAND;           // [S] forward: u_t; reverse: lambda_t
  float *stay = smem + BAND + S;       // [A][256] stay probability of T'
  const int tid = threadIdx.x;
  // T' = softmax(theta), f = logistic(phi), and the stay table of T'
  if (tid < A) {
    float mx = -INFINITY;
    for (int k = 0; k < 9; ++k) mx = fmaxf(mx, fa.theta[tid * 9 + k]);
    float e[9], sum = 0.f;
    for (int k = 0; k < 9; ++k) {
      e[k] = expf(fa.theta[tid * 9 + k] - mx);
      sum += e[k];
    }
    for (int k = 0; k < 9; ++k) s_slip[tid * 9 + k] = e[k] / sum;
  }
  if (tid < 4) s_flip[tid] = 1.f / (1.f + expf(-fa.phi[tid]));
  if (tid == 0) s_bgoal = 0.f;
  __syncthreads();
  for (int i = tid; i < A * 256; i += kFBlock) {
    const int a = i >> 8, pat = i & 255;
    float st = s_slip[a * 9 + 4];
    int bit = 0;
    for (int k = 0; k < 9; ++k) {
      if (k == 4) continue;
      if (!((pat >> bit) & 1)) st += s_slip[a * 9 + k];
      ++bit;
    }
    stay[i] = st;
  }
  for (int i = tid; i < BAND; i += kFBlock) band[i] = 0.f;   // halo stays zero
  __syncthreads();
  const float rW = 1.0f / (float)W;
  auto bidx = [&](int t) {
    const int ly = fdiv(t, W, rW);
    return (ly + 1) * BW + (t - ly * W) + 1;
  };
  float *ckpt = fa.ckpt + (size_t)blockIdx.x * fa.nseg * S;
  float *segb = fa.seg + (size_t)blockIdx.x * (fa.k + 2) * S;   // k+1 beliefs, then lambda
  float *lsave = segb + (size_t)(fa.k + 1) * S;
  float *eta = fa.eta + (size_t)blockIdx.x * (fa.T + 1);

  // belief src -> band (blocked cells carry no mass; the goal's own mass goes
  // to s_bgoal, its band entry stays 0)
  auto load = [&](const float *src) {
    for (int t = tid; t < S; t += kFBlock) {
      const uint32_t sg = fa.sig[t];
      const float v = (sg & kSigFree) ? src[t] : 0.f;
      if (sg & kSigGoal) s_bgoal = v;
      band[bidx(t)] = (sg & kSigGoal) ? 0.f : v;
    }
  };
  auto store = [&](float *dst) {
    for (int t = tid; t < S; t += kFBlock) {
      const uint32_t sg = fa.sig[t];
      dst[t] = (sg & kSigGoal) ? s_bgoal : band[bidx(t)];
    }
  };
  // one filter step: band holds b_{t-1} on entry and b_t on exit; returns eta_t
  auto fstep = [&](int a, int z) -> float {
    const float *sl = s_slip + a * 9;
    const float *sa = stay + a * 256;
    const uint32_t zw = (uint32_t)(z & 15), zl = (uint32_t)(z >> 4);
    float loc[1] = {0.f};
    for (int t = tid; t < S; t += kFBlock) {
      const uint32_t sg = fa.sig[t];
      float c = 0.f;
      if (sg & kSigFree) {
        const float *cp = band + bidx(t);
        c = (sg & kSigGoal) ? stencil(cp, BW, sl, 1.f, s_bgoal)
                            : stencil(cp, BW, sl, sa[sig_out8(sg)], cp[0]);
      }
      const float u = wall_lik(s_flip, zw, sig_wall(sg)) * lm_lik(m.lm_p, zl, sig_lm(sg)) * c;
      cell[t] = u;
      loc[0] += u;
    }
    fblock_sum<1>(loc, s_red, s_out);   // ends with a barrier: band reads are done
    const float e = s_out[0];
    for (int t = tid; t < S; t += kFBlock) {
      const uint32_t sg = fa.sig[t];
      const float b = cell[t] / e;
      if (sg & kSigGoal) s_bgoal = b;
      band[bidx(t)] = (sg & kSigGoal) ? 0.f : b;
    }
    __syncthreads();
    return e;
  };

  for (int tr = blockIdx.x; tr < fa.ntraj; tr += fa.G) {
    const int32_t *at = fa.acts + (size_t)tr * fa.T;
    const int32_t *zt = fa.obs + (size_t)tr * fa.T;
    const float *b0 = fa.b0 + (fa.b0_per_traj ? (size_t)tr * S : 0);
    // ---- forward pass
    __syncthreads();
    if (tid == 0) s_nll = 0.0;
    load(b0);
    __syncthreads();
    bool bad = false;
    for (int t = 1; t <= fa.T; ++t) {
      const int a = at[t - 1], z = zt[t - 1];
      if (a < 0 || a >= A || z < 0 || z >= 16 * (m.L + 1)) {
        bad = true;
        break;
      }
      const float e = fstep(a, z);
      if (tid == 0) {
        s_nll -= log((double)e);
        eta[t] = e;
      }
      if (t % fa.k == 0 && t < fa.T) store(ckpt + (size_t)(t / fa.k) * S);
    }
    __syncthreads();
    if (bad) {
      if (tid == 0) {
        atomicOr(fa.err, 4);
        fa.nll[tr] = NAN;
      }
      if (fa.want_grad && tid < kFGrad) fa.gpart[(size_t)tr * kFGrad + tid] = 0.0;
      continue;
    }
    if (tid == 0) {
      fa.nll[tr] = (float)s_nll;
      if (!(s_nll < INFINITY)) atomicOr(fa.err, 8);
    }
    if (!fa.want_grad) continue;

    // ---- reverse sweep, one stored segment at a time; lambda_T = 0
    if (tid < kFGrad) s_g[tid] = 0.0;
    for (int t = tid; t < S; t += kFBlock) lsave[t] = 0.f;
    for (int sgi = fa.nseg - 1; sgi >= 0; --sgi) {
      const int t0 = sgi * fa.k, t1 = min(fa.T, t0 + fa.k);
      // recompute b_{t0..t1} into the segment buffer (cell is the u scratch)
      __syncthreads();
      load(sgi == 0 ? b0 : ckpt + (size_t)sgi * S);
      __syncthreads();
      store(segb);
      for (int t = t0 + 1; t <= t1; ++t) {
        fstep(at[t - 1], zt[t - 1]);
        store(segb + (size_t)(t - t0) * S);
      }
      __syncthreads();
      for (int t = tid; t < S; t += kFBlock) cell[t] = lsave[t];   // lambda_{t1}
      __syncthreads();
      for (int t = t1; t > t0; --t) {
        const int a = at[t - 1], z = zt[t - 1];
        const uint32_t zw = (uint32_t)(z & 15), zl = (uint32_t)(z >> 4);
        const float *sl = s_slip + a * 9;
        const float *bt = segb + (size_t)(t - t0) * S;
        const float *bp = segb + (size_t)(t - 1 - t0) * S;
        const float e = eta[t];
        float lb[1] = {0.f};
        for (int t2 = tid; t2 < S; t2 += kFBlock) lb[0] = fmaf(cell[t2], bt[t2], lb[0]);
        fblock_sum<1>(lb, s_red, s_out);
        const float lbt = s_out[0];
        float gs[13];
#pragma unroll
        for (int i = 0; i < 13; ++i) gs[i] = 0.f;
        // cbar_t = O(z_t|.) ubar_t into the band; flip partials with
        // c_t = eta_t b_t / O (where O = 0 the partials vanish)
        for (int t2 = tid; t2 < S; t2 += kFBlock) {
          const uint32_t sg = fa.sig[t2];
          const float ub = (cell[t2] - lbt - 1.f) / e;
          const uint32_t w = sig_wall(sg);
          const float lmf = lm_lik(m.lm_p, zl, sig_lm(sg));
          const float o = wall_lik(s_flip, zw, w) * lmf;
          band[bidx(t2)] = o * ub;
          if (o > 0.f) {
            const float go = (e * bt[t2] / o) * ub;
            const uint32_t mis = zw ^ w;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              // dO/df_i: landmark factor times the other bits, + if bit i misread
              float rest = lmf;
#pragma unroll
              for (int i2 = 0; i2 < 4; ++i2)
                if (i2 != i) rest *= ((mis >> i2) & 1u) ? s_flip[i2] : 1.f - s_flip[i2];
              gs[i] = fmaf(go, ((mis >> i) & 1u) ? rest : -rest, gs[i]);
            }
          }
        }
        __syncthreads();
        // lambda_{t-1}(s) = sum_k T'(a,k) cbar(dest(s,k)); slip partials
        for (int t2 = tid; t2 < S; t2 += kFBlock) {
          const uint32_t sg = fa.sig[t2];
          const float *cp = band + bidx(t2);
          if ((sg & kSigFree) && !(sg & kSigGoal)) {
            const uint32_t out8 = sig_out8(sg);
            const float bprev = bp[t2];
            float acc = 0.f;
            int bit = 0;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
              float cd;
              if (k == 4) {
                cd = cp[0];
              } else {
                cd = ((out8 >> bit) & 1u) ? cp[(k / 3 - 1) * BW + (k % 3 - 1)] : cp[0];
                ++bit;
              }
              acc = fmaf(sl[k], cd, acc);
              gs[4 + k] = fmaf(bprev, cd, gs[4 + k]);
            }
            cell[t2] = acc;
          } else {
            // the goal keeps its own mass; a blocked cell never receives any,
            // so its adjoint is 0
            cell[t2] = (sg & kSigGoal) ? cp[0] : 0.f;
          }
        }
        fblock_sum<13>(gs, s_red, s_out);
        if (tid < 4) s_g[81 + tid] += (double)s_out[tid];
        if (tid >= 4 && tid < 13) s_g[a * 9 + tid - 4] += (double)s_out[tid];
      }
      __syncthreads();
      for (int t = tid; t < S; t += kFBlock) lsave[t] = cell[t];   // lambda_{t0}
    }
    __syncthreads();
    if (tid < kFGrad) fa.gpart[(size_t)tr * kFGrad + tid] = s_g[tid];
  }
}

// Sum of the per-trajectory partials in trajectory order (FP64), then the
// chain rule through the softmax and the logistic.
__global__ void k_filter_grad(int ntraj, int A, const float *theta, const float *phi,
                              const double *gpart, float *g_slip, float *g_flip) {
  __shared__ double g[kFGrad];
  __shared__ double sl[81];
  const int tid = threadIdx.x;
  if (tid < kFGrad) {
    double s = 0.0;
    for (int i = 0; i < ntraj; ++i) s += gpart[(size_t)i * kFGrad + tid];
    g[tid] = s;
  }
  if (tid < A) {
    double mx = -INFINITY, sum = 0.0;
    for (int k = 0; k < 9; ++k) mx = fmax(mx, (double)theta[tid * 9 + k]);
    for (int k = 0; k < 9; ++k) sum += exp((double)theta[tid * 9 + k] - mx);
    for (int k = 0; k < 9; ++k) sl[tid * 9 + k] = exp((double)theta[tid * 9 + k] - mx) / sum;
  }
  __syncthreads();
  if (tid < A * 9) {
    const int a = tid / 9, j = tid - a * 9;
    double s = 0.0;
    for (int k = 0; k < 9; ++k)
      s += g[a * 9 + k] * sl[a * 9 + k] * ((k == j ? 1.0 : 0.0) - sl[a * 9 + j]);
    g_slip[tid] = (float)s;
  }
  if (tid < 4) {
    const double f = 1.0 / (1.0 + exp(-(double)phi[tid]));
    g_flip[tid] = (float)(g[81 + tid] * f * (1.0 - f));
  }
}

size_t filter_lds_bytes(const qv_model *m) {
  return ((size_t)(m->H + 2) * (m->W + 2) + (size_t)m->W * m->H + (size_t)m->A * 256) *
         sizeof(float);
}

bool filter_supported(const qv_model *m) { return filter_lds_bytes(m) <= 150 * 1024; }

int filter_groups(int ntraj) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return std::max(1, std::min(ntraj, cus));
}

size_t filter_ws(const qv_model *m, int ntraj, int T, int k, int G) {
  const size_t S = (size_t)m->W * m->H;
  const int nseg = (T + k - 1) / k;
  size_t off = 0;
  off += align_up(S * 4, 256);                                   // sig
  off += align_up((size_t)m->A * 256 * 4, 256);                  // staytab (prep)
  off += align_up((size_t)G * nseg * S * 4, 256);                // stored beliefs
  off += align_up((size_t)G * (k + 2) * S * 4, 256);             // segment buffers + lambda
  off += align_up((size_t)G * (T + 1) * 4, 256);                 // eta
  off += align_up((size_t)ntraj * kFGrad * 8, 256);              // per-trajectory partials
  off += 256;                                                    // err
  return off;
}

hipError_t launch_filter(const DevModel &m, const float *theta, const float *phi, int ntraj,
                         int T, const float *b0, int b0_per_traj, const int32_t *acts,
                         const int32_t *obs, int k, float *nll, float *g_slip, float *g_flip,
                         char *ws, int G, hipStream_t st) {
  const size_t S = (size_t)m.S;
  const int nseg = (T + k - 1) / k;
  size_t off = 0;
  uint32_t *sig = (uint32_t *)(ws + off);
  off += align_up(S * 4, 256);
  float *staytab = (float *)(ws + off);
  off += align_up((size_t)m.A * 256 * 4, 256);
  float *ckpt = (float *)(ws + off);
  off += align_up((size_t)G * nseg * S * 4, 256);
  float *segb = (float *)(ws + off);
  off += align_up((size_t)G * (k + 2) * S * 4, 256);
  float *eta = (float *)(ws + off);
  off += align_up((size_t)G * (T + 1) * 4, 256);
  double *gpart = (double *)(ws + off);
  off += align_up((size_t)ntraj * kFGrad * 8, 256);
  int32_t *err = (int32_t *)(ws + off);
  hipError_t e = launch_prep(m, sig, staytab, err, st);
  if (e != hipSuccess) return e;
  FilterArgs fa;
  fa.ntraj = ntraj;
  fa.T = T;
  fa.k = k;
  fa.nseg = nseg;
  fa.G = G;
  fa.theta = theta;
  fa.phi = phi;
  fa.b0 = b0;
  fa.b0_per_traj = b0_per_traj;
  fa.acts = acts;
  fa.obs = obs;
  fa.nll = nll;
  fa.gpart = gpart;
  fa.ckpt = ckpt;
  fa.seg = segb;
  fa.eta = eta;
  fa.sig = sig;
  fa.err = err;
  fa.want_grad = (g_slip && g_flip) ? 1 : 0;
  const size_t lds =
      ((size_t)(m.H + 2) * (m.W + 2) + (size_t)m.W * m.H + (size_t)m.A * 256) * sizeof(float);
  e = hipFuncSetAttribute((const void *)k_filter, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds);
  if (e != hipSuccess) return e;
  if (ntraj > 0) QV_LAUNCH(k_filter, dim3(G), dim3(kFBlock), lds, st, m, fa);
  // with no trajectories the gradient kernel writes zeros
  if (fa.want_grad)
    QV_LAUNCH(k_filter_grad, dim3(1), dim3(128), 0, st, ntraj, m.A, theta, phi, gpart, g_slip,
              g_flip);
  return hipGetLastError();
}

}  // namespace qv
