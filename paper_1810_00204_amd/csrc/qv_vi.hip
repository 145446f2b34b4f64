// qv_vi.hip -- offline value bounds on gfx950 that score the leaves of the
// QV-tree:
//   * Q-MDP value iteration: the MDP value iteration of Sec. V-B, which is
//     the alpha-vector recursion of Sec. IV-A with a perfect sensor;
//   * the fast informed bound (FIB), the alpha-vector equation of Sec. IV-A:
//       alpha^a(x) = R(x,a) + gamma sum_z max_a' sum_x' O(z|x') T(x,a,x') alpha^a'(x').
// Both are Jacobi sweeps in FP32.  The residual of sweep k, max |x_k - x_{k-1}|
// over free cells (and actions), is formed in FP64 (exact for a difference
// of two FP32 values) and max-reduced with an integer atomic on its bit
// pattern, which is order independent.
//
// On small and medium grids all sweeps of a solve run in one cooperative
// launch: every workgroup is resident, and after each sweep the workgroups
// meet at a grid barrier, read the sweep's residual and max |value| and so
// all stop after the same sweep (the stopping rule sees the same numbers
// everywhere); the host waits once, at the end.  On large grids (and where a
// cooperative launch is not possible) the sweeps are launched one by one,
// each doing nothing once the rule has fired, and the host reads the
// residuals every kViChunk sweeps.  Both forms do the same arithmetic per
// cell, so their results are bitwise equal.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "qv_internal.h"

namespace qv {

constexpr int kViChunk = 32;
constexpr int kMaxCoopGrid = 4096;   // workgroups of a one-launch solve at most

// ---------------------------------------------------------------------------
// grid barrier and the shared stopping rule
// ---------------------------------------------------------------------------

// Values that other workgroups of the same launch read (V_k, alpha_k) are
// stored with agent-scope atomic stores and loaded with agent-scope atomic
// loads.  In the AMDGPU memory model such accesses are performed at the
// device's coherence point (past the per-XCD L2, which is not coherent
// across XCDs), so no cache-wide fence is needed; read-only tables (map
// signature, stay table, rewards) keep their L2 copies across sweeps.
template <bool COH>
__device__ __forceinline__ float ld_val(const float *p) {
  if constexpr (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return *p;
}
template <bool COH>
__device__ __forceinline__ void st_val(float *p, float v) {
  if constexpr (COH)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}

// Grid barrier of a cooperative launch, round r = 1, 2, ...: the counter
// *bar reaches r * gridDim.x once every workgroup has arrived.  Every
// thread first waits until its own stores (and the workgroup's residual
// atomics) have completed at the coherence point (s_waitcnt 0); after the
// workgroup barrier lane 0 arrives with an agent-scope atomic add and polls
// the counter.  A workgroup that sees the full count therefore reads, with
// its agent-scope loads, everything every workgroup wrote before arriving.
// The wait is bounded: after kSpinLimit polls (seconds, far beyond any
// sweep) lane 0 raises *abort and leaves, and every other waiting workgroup
// leaves as soon as it sees the flag, so the launch always ends; the
// caller then stops.
constexpr long long kSpinLimit = 1ll << 22;

__device__ __forceinline__ void grid_sync(unsigned long long *bar, unsigned long long target,
                                          unsigned int *abort) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long long polls = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
      if (++polls > kSpinLimit) {
        __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
}

// Control block of one solve in the workspace.
struct SweepCtl {
  unsigned long long *res, *vmax;   // [max_sweeps + 2]: bit patterns of r_k, max |x_k|
  unsigned long long *bar;          // grid barrier counter
  double *out_res;                  // residual of the last sweep
  int *out_k;                       // number of sweeps run
  unsigned int *abort;              // set when a barrier wait gave up
  double *part;                     // [2][2][grid]: per-workgroup r, max |x| of a sweep
  int max_sweeps;
  double tol;
};

__device__ __forceinline__ double load_bits(const unsigned long long *p) {
  return __longlong_as_double(
      (long long)__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// One-launch form: workgroup g's (r, max |x|) of sweep k go to slot g of the
// sweep's parity buffer (plain coherent stores, no atomic on a shared word);
// after the grid barrier wavefront 0 of every workgroup takes the maxima
// over all slots (the same values everywhere: max is order independent),
// and workgroup 0 records them as sweep k's residual.  Returns whether the
// rule fires (in lane 0 of wavefront 0).
__device__ __forceinline__ void sweep_part_store(const SweepCtl &c, int k, double r, double v,
                                                 double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    r = fmax(r, __shfl_xor(r, o, kWave));
    v = fmax(v, __shfl_xor(v, o, kWave));
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) {
    red[wave] = r;
    red[kBlock / kWave + wave] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) {
      r = fmax(r, red[w]);
      v = fmax(v, red[kBlock / kWave + w]);
    }
    double *p = c.part + (size_t)(k & 1) * 2 * gridDim.x;
    __hip_atomic_store(p + blockIdx.x, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + gridDim.x + blockIdx.x, v, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ int sweep_part_decide(const SweepCtl &c, int k) {
  const int lane = threadIdx.x & (kWave - 1);
  const double *p = c.part + (size_t)(k & 1) * 2 * gridDim.x;
  double r = 0.0, v = 0.0;
  for (int g = lane; g < (int)gridDim.x; g += kWave) {
    r = fmax(r, __hip_atomic_load(p + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    v = fmax(v, __hip_atomic_load(p + gridDim.x + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    r = fmax(r, __shfl_xor(r, o, kWave));
    v = fmax(v, __shfl_xor(v, o, kWave));
  }
  if (blockIdx.x == 0 && lane == 0) {
    c.res[k] = (unsigned long long)__double_as_longlong(r);
    c.vmax[k] = (unsigned long long)__double_as_longlong(v);
  }
  return (r == 0.0 || r <= c.tol * fmax(1.0, v)) ? 1 : 0;
}

// Stop after sweep k: r_k = 0 or r_k <= tol * max(1, max |x_k|).
__device__ __forceinline__ bool sweep_converged(const SweepCtl &c, int k) {
  const double r = load_bits(c.res + k), vm = load_bits(c.vmax + k);
  return r == 0.0 || r <= c.tol * fmax(1.0, vm);
}

// Workgroup max of (r, v); thread 0 folds the result into sweep k's records
// (non-negative doubles order like their bit patterns).  Ends with a barrier.
__device__ __forceinline__ void sweep_report(double r, double v, unsigned long long *res,
                                             unsigned long long *vmax, int k, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    r = fmax(r, __shfl_xor(r, o, kWave));
    v = fmax(v, __shfl_xor(v, o, kWave));
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) {
    red[wave] = r;
    red[kBlock / kWave + wave] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) {
      r = fmax(r, red[w]);
      v = fmax(v, red[kBlock / kWave + w]);
    }
    atomicMax(&res[k], (unsigned long long)__double_as_longlong(r));
    atomicMax(&vmax[k], (unsigned long long)__double_as_longlong(v));
  }
  __syncthreads();
}

__global__ void k_sweep_fill(unsigned long long *res, unsigned long long *vmax, int n,
                             unsigned long long *bar, float *x0, long long nx) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    res[i] = 0ull;
    vmax[i] = 0ull;
  }
  if (i == 0) {
    bar[0] = 0ull;   // barrier counter
    bar[2] = 0ull;   // sweep count and abort flag
  }
  if (i < nx) x0[i] = 0.f;
}

// ---------------------------------------------------------------------------
// Q-MDP value iteration
// ---------------------------------------------------------------------------

// V band: off-grid and blocked cells read as zero (their value is 0), the
// goal keeps its value.
template <bool COH>
__device__ __forceinline__ void load_vband(const DevModel &m, const uint32_t *sig,
                                           const float *V, int y0, int th, float *band,
                                           int BW) {
  constexpr int kBatch = 8;   // band entries whose loads a thread issues together
  const int n = (th + 2) * BW;
  const float rBW = 1.0f / (float)BW;
  for (int i0 = threadIdx.x; i0 < n; i0 += kBatch * kBlock) {
    int cell[kBatch];
    uint32_t sg[kBatch];
    float v[kBatch];
    // every lane loads (cell 0 for halo and padding lanes) and masks after,
    // so the batch's loads go out together
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int i = i0 + j * kBlock;
      const int r = fdiv(i, BW, rBW);
      const int gy = y0 - 1 + r, gx = i - r * BW - 1;
      const bool in = i < n && gy >= 0 && gy < m.H && gx >= 0 && gx < m.W;
      cell[j] = in ? gy * m.W + gx : -1;
      sg[j] = sig[in ? cell[j] : 0];
      v[j] = ld_val<COH>(V + (in ? cell[j] : 0));
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int i = i0 + j * kBlock;
      if (i < n) band[i] = (cell[j] >= 0 && (sg[j] & kSigFree)) ? v[j] : 0.f;
    }
  }
}

// Q(s,a) = R(s,a) + gamma * (sum_k T'(a,k) V(s + d_k) + stay(s,a) V(s)):
// the expectation over T(s,a,.) of Sec. V, with the band zero where a move
// fails (its mass is in `stay`).
__device__ __forceinline__ float q_backup(const DevModel &m, const float *c, int BW,
                                          const float *sl, float stay, float r) {
  float v = sl[0] * c[-BW - 1];
  v = fmaf(sl[1], c[-BW], v);
  v = fmaf(sl[2], c[-BW + 1], v);
  v = fmaf(sl[3], c[-1], v);
  v = fmaf(sl[5], c[1], v);
  v = fmaf(sl[6], c[BW - 1], v);
  v = fmaf(sl[7], c[BW], v);
  v = fmaf(sl[8], c[BW + 1], v);
  v = fmaf(stay, c[0], v);
  return fmaf(m.gamma, v, r);
}

__device__ __forceinline__ float cell_q(const DevModel &m, const float *band, int BW, int ly,
                                        int lx, uint32_t sg, const float *staytab, int a,
                                        int t) {
  const float *c = band + (ly + 1) * BW + lx + 1;
  const float r = m.R[(size_t)t * m.A + a];
  if (sg & kSigGoal) return fmaf(m.gamma, c[0], r);
  return q_backup(m, c, BW, &m.slip[a * 9], staytab[a * 256 + sig_out8(sg)], r);
}

// One band of sweep k: V_k from V_{k-1} (in the LDS band); the band's
// largest |V_k - V_{k-1}| and |V_k| (free cells) are folded into r, vm.
template <bool COH>
__device__ __forceinline__ void vi_band(const DevModel &m, const uint32_t *sig,
                                        const float *staytab, int TH, int tile,
                                        const float *Vin, float *Vout, float *band, double &r,
                                        double &vm) {
  const int W = m.W, BW = W + 2;
  const int y0 = tile * TH;
  const int th = min(TH, m.H - y0);
  load_vband<COH>(m, sig, Vin, y0, th, band, BW);
  __syncthreads();
  const float rW = 1.0f / (float)W;
  for (int i = threadIdx.x; i < th * W; i += kBlock) {
    const int ly = fdiv(i, W, rW), lx = i - ly * W;
    const int t = (y0 + ly) * W + lx;
    const uint32_t sg = sig[t];
    float best = 0.f;
    if (sg & kSigFree) {
      best = -INFINITY;
      for (int a = 0; a < m.A; ++a)
        best = fmaxf(best, cell_q(m, band, BW, ly, lx, sg, staytab, a, t));
      const double d = fabs((double)best - (double)band[(ly + 1) * BW + lx + 1]);
      r = fmax(r, d);
      vm = fmax(vm, fabs((double)best));
    }
    st_val<COH>(Vout + t, best);
  }
  __syncthreads();   // the band is reused by the next tile
}

// Q(t, .) of one band from V (the Q-values of a sweep from its input V).
template <bool COH>
__device__ __forceinline__ void vi_q_band(const DevModel &m, const uint32_t *sig,
                                          const float *staytab, int TH, int tile, const float *V,
                                          float *Q, float *band) {
  const int W = m.W, BW = W + 2;
  const int y0 = tile * TH;
  const int th = min(TH, m.H - y0);
  load_vband<COH>(m, sig, V, y0, th, band, BW);
  __syncthreads();
  const float rW = 1.0f / (float)W;
  for (int i = threadIdx.x; i < th * W; i += kBlock) {
    const int ly = fdiv(i, W, rW), lx = i - ly * W;
    const int t = (y0 + ly) * W + lx;
    const uint32_t sg = sig[t];
    for (int a = 0; a < m.A; ++a)
      Q[(size_t)t * m.A + a] =
          (sg & kSigFree) ? cell_q(m, band, BW, ly, lx, sg, staytab, a, t) : 0.f;
  }
  __syncthreads();
}

// Every sweep in one launch (cooperative: all workgroups resident).  V[0]
// holds V_0 = 0; sweep k writes V_k into V[k & 1].  After the last sweep kc
// the workgroups write Q_kc (from V_{kc-1}) into Q.
__global__ __launch_bounds__(kBlock) void k_vi_coop(DevModel m, const uint32_t *sig,
                                                    const float *staytab, int TH, int tiles,
                                                    float *V0, float *V1, float *Q,
                                                    SweepCtl c) {
  extern __shared__ float smem[];
  __shared__ double red[2 * kBlock / kWave];
  __shared__ int s_stop;
  if (threadIdx.x == 0) s_stop = 0;
  int kend = c.max_sweeps;
  for (int k = 1; k <= c.max_sweeps; ++k) {
    const float *Vin = (k & 1) ? V0 : V1;
    float *Vout = (k & 1) ? V1 : V0;
    double r = 0.0, vm = 0.0;
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x)
      vi_band<true>(m, sig, staytab, TH, tile, Vin, Vout, smem, r, vm);
    sweep_part_store(c, k, r, vm, red);
    grid_sync(c.bar, (unsigned long long)k * gridDim.x, c.abort);
    if (threadIdx.x < kWave) {
      const int conv = sweep_part_decide(c, k);
      if (threadIdx.x == 0)
        s_stop = __hip_atomic_load(c.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 2
                                                                                        : conv;
    }
    __syncthreads();
    if (s_stop) {   // the same decision in every workgroup (unless aborted)
      kend = k;
      break;
    }
  }
  if (s_stop == 2) return;
  const float *Vprev = (kend & 1) ? V0 : V1;
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x)
    vi_q_band<true>(m, sig, staytab, TH, tile, Vprev, Q, smem);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *c.out_k = kend;
    *c.out_res = load_bits(c.res + kend);
  }
}

// Per-sweep form: sweep k >= 1, V_k from V_{k-1}; does nothing once the
// rule has fired at an earlier sweep.
__global__ __launch_bounds__(kBlock) void k_vi_sweep(DevModel m, const uint32_t *sig,
                                                     const float *staytab, int TH,
                                                     const float *Vin, float *Vout, int k,
                                                     SweepCtl c) {
  if (k > 1 && sweep_converged(c, k - 1)) return;
  extern __shared__ float smem[];
  __shared__ double red[2 * kBlock / kWave];
  double r = 0.0, vm = 0.0;
  vi_band<false>(m, sig, staytab, TH, blockIdx.x, Vin, Vout, smem, r, vm);
  sweep_report(r, vm, c.res, c.vmax, k, red);
}

// Q_k(s,.) from V_{k-1}, the Q-values of the last sweep (same arithmetic).
__global__ __launch_bounds__(kBlock) void k_vi_q(DevModel m, const uint32_t *sig,
                                                 const float *staytab, int TH, const float *V,
                                                 float *Q) {
  extern __shared__ float smem[];
  vi_q_band<false>(m, sig, staytab, TH, blockIdx.x, V, Q, smem);
}

// ---------------------------------------------------------------------------
// fast informed bound
// ---------------------------------------------------------------------------

// The FIB right-hand side at free cell x for every action (AM >= A columns,
// rows of the alpha tables have A entries).  The successors of x are its
// neighbours k != 4 that a move enters (sig bits) and x itself, which takes
// the stay mass: T(x,a,x + d_k) = T'(a,k), T(x,a,x) = stay(x,a).  With
// C[zw][w] the wall-reading likelihood (ctab) and lambda(x') = 1 - rho on a
// landmark cell, else 1, the sum over z splits into
//   zl = 0:  sum_zw max_a' sum_k C[zw][w(x_k)] lambda(x_k) T_k(a) alpha^a'(x_k),
//   zl = l:  rho T_k(a) max_a' alpha^a'(x_k) for the successor x_k that is
//            landmark l (only it can report l, and sum_zw C[zw][w] = 1).
// The goal is absorbing: its right-hand side is R + gamma max_a' alpha^a'(goal).
template <int AM, bool COH>
__device__ __forceinline__ void fib_cell(const DevModel &m, const uint32_t *sig,
                                         const float *staytab, const float *al,
                                         const float *ctab, int x, uint32_t sg,
                                         float (&out)[AM]) {
  const int A = m.A, W = m.W, L = m.L;
  const float rho = m.lm_p;
  if (sg & kSigGoal) {
    float best = -INFINITY;
#pragma unroll
    for (int ap = 0; ap < AM; ++ap)
      if (ap < A) best = fmaxf(best, ld_val<COH>(al + (size_t)x * A + ap));
#pragma unroll
    for (int a = 0; a < AM; ++a)
      out[a] = a < A ? fmaf(m.gamma, best, m.R[(size_t)x * A + a]) : 0.f;
    return;
  }
  // the successors' alpha rows (zero where the move fails), wall readings
  // and landmark factors; loads go out together at valid addresses
  float v[9][AM];
  uint32_t wk[9];
  float lam[9];
  bool lmk[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const bool ok = (k == 4) || ((sg >> (k < 4 ? k : k - 1)) & 1u);
    const int t = ok ? x + (k / 3 - 1) * W + (k % 3 - 1) : x;
    const uint32_t st = sig[t];
    const uint32_t lm = sig_lm(st);
    wk[k] = sig_wall(st);
    lmk[k] = ok && lm != 0u && lm <= (uint32_t)L;
    lam[k] = lmk[k] ? 1.f - rho : 1.f;
#pragma unroll
    for (int ap = 0; ap < AM; ++ap) {
      const float av = ld_val<COH>(al + (size_t)t * A + (ap < A ? ap : 0));
      v[k][ap] = (ok && ap < A) ? av : 0.f;
    }
  }
  float acc[AM], stay[AM];
  const int pat = (int)sig_out8(sg);
#pragma unroll
  for (int a = 0; a < AM; ++a) {
    acc[a] = 0.f;
    stay[a] = staytab[(a < A ? a : 0) * 256 + pat];
  }
  for (int zw = 0; zw < 16; ++zw) {
    float cw[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) cw[k] = ctab[zw * 16 + wk[k]] * lam[k];
#pragma unroll
    for (int a = 0; a < AM; ++a) {
      if (a >= A) continue;
      float g[9];
#pragma unroll
      for (int k = 0; k < 9; ++k)
        g[k] = cw[k] * (k == 4 ? stay[a] : m.slip[a * 9 + k]);
      float best = -INFINITY;
#pragma unroll
      for (int ap = 0; ap < AM; ++ap) {
        if (ap >= A) continue;
        float s = g[0] * v[0][ap];
#pragma unroll
        for (int k = 1; k < 9; ++k) s = fmaf(g[k], v[k][ap], s);
        best = fmaxf(best, s);
      }
      acc[a] += best;
    }
  }
  // landmark observations of the successors
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (!lmk[k]) continue;
    float mk = -INFINITY;
#pragma unroll
    for (int ap = 0; ap < AM; ++ap)
      if (ap < A) mk = fmaxf(mk, v[k][ap]);
#pragma unroll
    for (int a = 0; a < AM; ++a) {
      if (a >= A) continue;
      const float tk = k == 4 ? stay[a] : m.slip[a * 9 + k];
      acc[a] = fmaf(rho * tk, mk, acc[a]);
    }
  }
#pragma unroll
  for (int a = 0; a < AM; ++a)
    out[a] = a < A ? fmaf(m.gamma, acc[a], m.R[(size_t)x * A + a]) : 0.f;
}

// The blind-policy right-hand side at free cell x for every action: each
// action's own vector, alpha^a(x) = R(x,a) + gamma sum_x' T(x,a,x') alpha^a(x')
// (no max over actions: the value of taking a forever, a lower bound).
template <int AM, bool COH>
__device__ __forceinline__ void blind_cell(const DevModel &m, const uint32_t *sig,
                                           const float *staytab, const float *al, int x,
                                           uint32_t sg, float (&out)[AM]) {
  const int A = m.A, W = m.W;
  if (sg & kSigGoal) {
#pragma unroll
    for (int a = 0; a < AM; ++a)
      out[a] = a < A ? fmaf(m.gamma, ld_val<COH>(al + (size_t)x * A + a),
                            m.R[(size_t)x * A + a])
                     : 0.f;
    return;
  }
  const int pat = (int)sig_out8(sg);
  float acc[AM];
#pragma unroll
  for (int a = 0; a < AM; ++a) acc[a] = 0.f;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const bool ok = (k == 4) || ((sg >> (k < 4 ? k : k - 1)) & 1u);
    const int t = ok ? x + (k / 3 - 1) * W + (k % 3 - 1) : x;
#pragma unroll
    for (int a = 0; a < AM; ++a) {
      if (a >= A) continue;
      const float av = ld_val<COH>(al + (size_t)t * A + a);
      const float tk = k == 4 ? staytab[a * 256 + pat] : m.slip[a * 9 + k];
      acc[a] = fmaf(tk, ok ? av : 0.f, acc[a]);
    }
  }
#pragma unroll
  for (int a = 0; a < AM; ++a)
    out[a] = a < A ? fmaf(m.gamma, acc[a], m.R[(size_t)x * A + a]) : 0.f;
}

// C[zw][w] = prod_j (bit j of zw ^ w set ? f_j : 1 - f_j) into LDS.
__device__ __forceinline__ void fib_ctab(const DevModel &m, float *ctab) {
  if (threadIdx.x < 256) ctab[threadIdx.x] = wall_lik(m.flip, threadIdx.x >> 4, threadIdx.x & 15u);
  __syncthreads();
}

// One sweep over the cells i = blockIdx.x * kBlock + threadIdx.x + j * stride.
template <int AM, bool COH, int OP>
__device__ __forceinline__ void fib_pass(const DevModel &m, const uint32_t *sig,
                                         const float *staytab, const float *ain, float *aout,
                                         const float *ctab, long long stride, double &r,
                                         double &vm) {
  const int A = m.A;
  for (long long x = (long long)blockIdx.x * kBlock + threadIdx.x; x < m.S; x += stride) {
    const uint32_t sg = sig[x];
    float o[AM];
    if (sg & kSigFree) {
      if constexpr (OP == 0)
        fib_cell<AM, COH>(m, sig, staytab, ain, ctab, (int)x, sg, o);
      else
        blind_cell<AM, COH>(m, sig, staytab, ain, (int)x, sg, o);
#pragma unroll
      for (int a = 0; a < AM; ++a) {
        if (a >= A) continue;
        r = fmax(r, fabs((double)o[a] - (double)ld_val<COH>(ain + x * A + a)));
        vm = fmax(vm, fabs((double)o[a]));
      }
    } else {
#pragma unroll
      for (int a = 0; a < AM; ++a) o[a] = 0.f;
    }
#pragma unroll
    for (int a = 0; a < AM; ++a)
      if (a < A) st_val<COH>(aout + x * A + a, o[a]);
  }
}

// Every FIB sweep in one launch (cooperative).  al[0] holds alpha_0 = 0;
// sweep k writes alpha_k into al[k & 1]; the last one is copied to out.
template <int AM, int OP>
__global__ __launch_bounds__(kBlock) void k_fib_coop(DevModel m, const uint32_t *sig,
                                                     const float *staytab, float *al0,
                                                     float *al1, float *out, SweepCtl c) {
  __shared__ float ctab[256];
  __shared__ double red[2 * kBlock / kWave];
  __shared__ int s_stop;
  if (threadIdx.x == 0) s_stop = 0;
  fib_ctab(m, ctab);
  const long long stride = (long long)gridDim.x * kBlock;
  int kend = c.max_sweeps;
  for (int k = 1; k <= c.max_sweeps; ++k) {
    const float *ain = (k & 1) ? al0 : al1;
    float *aout = (k & 1) ? al1 : al0;
    double r = 0.0, vm = 0.0;
    fib_pass<AM, true, OP>(m, sig, staytab, ain, aout, ctab, stride, r, vm);
    sweep_part_store(c, k, r, vm, red);
    grid_sync(c.bar, (unsigned long long)k * gridDim.x, c.abort);
    if (threadIdx.x < kWave) {
      const int conv = sweep_part_decide(c, k);
      if (threadIdx.x == 0)
        s_stop = __hip_atomic_load(c.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 2
                                                                                        : conv;
    }
    __syncthreads();
    if (s_stop) {
      kend = k;
      break;
    }
  }
  if (s_stop == 2) return;
  const float *last = (kend & 1) ? al1 : al0;
  const long long n = (long long)m.S * m.A;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
    out[i] = ld_val<true>(last + i);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *c.out_k = kend;
    *c.out_res = load_bits(c.res + kend);
  }
}

// Per-sweep form of FIB sweep k (nothing once the rule has fired).
template <int AM, int OP>
__global__ __launch_bounds__(kBlock) void k_fib_sweep(DevModel m, const uint32_t *sig,
                                                      const float *staytab, const float *ain,
                                                      float *aout, int k, SweepCtl c) {
  if (k > 1 && sweep_converged(c, k - 1)) return;
  __shared__ float ctab[256];
  __shared__ double red[2 * kBlock / kWave];
  fib_ctab(m, ctab);
  double r = 0.0, vm = 0.0;
  fib_pass<AM, false, OP>(m, sig, staytab, ain, aout, ctab, (long long)gridDim.x * kBlock, r,
                          vm);
  sweep_report(r, vm, c.res, c.vmax, k, red);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// Workspace: sig [S], staytab [A][256], two value buffers of `vals` floats,
// res and vmax [max_sweeps + 2], then barrier counter, residual and sweep
// count, error word.
static size_t sweep_ws(const qv_model *m, long long vals, int max_sweeps) {
  const size_t S = (size_t)m->W * m->H;
  size_t off = 0;
  off += align_up(S * 4, 256);
  off += align_up((size_t)m->A * 256 * 4, 256);
  off += 2 * align_up((size_t)vals * 4, 256);
  off += 2 * align_up((size_t)(max_sweeps + 2) * 8, 256);
  off += 256;   // barrier counter, residual, sweep count
  off += 256;   // error word
  off += align_up((size_t)4 * kMaxCoopGrid * 8, 256);   // per-workgroup residual partials
  return off;
}

size_t vi_ws(const qv_model *m, int max_sweeps) {
  return sweep_ws(m, (long long)m->W * m->H, max_sweeps);
}

size_t fib_ws(const qv_model *m, int max_sweeps) {
  return sweep_ws(m, (long long)m->W * m->H * m->A, max_sweeps);
}

struct SweepWs {
  uint32_t *sig;
  float *staytab;
  float *x[2];
  int32_t *err;
  SweepCtl c;
};

static SweepWs carve(const DevModel &m, long long vals, int max_sweeps, float tol, char *ws) {
  SweepWs w;
  size_t off = 0;
  w.sig = (uint32_t *)(ws + off);
  off += align_up((size_t)m.S * 4, 256);
  w.staytab = (float *)(ws + off);
  off += align_up((size_t)m.A * 256 * 4, 256);
  for (int i = 0; i < 2; ++i) {
    w.x[i] = (float *)(ws + off);
    off += align_up((size_t)vals * 4, 256);
  }
  w.c.res = (unsigned long long *)(ws + off);
  off += align_up((size_t)(max_sweeps + 2) * 8, 256);
  w.c.vmax = (unsigned long long *)(ws + off);
  off += align_up((size_t)(max_sweeps + 2) * 8, 256);
  w.c.bar = (unsigned long long *)(ws + off);
  w.c.out_res = (double *)(ws + off + 8);
  w.c.out_k = (int *)(ws + off + 16);
  w.c.abort = (unsigned int *)(ws + off + 20);
  off += 256;
  w.err = (int32_t *)(ws + off);
  off += 256;
  w.c.part = (double *)(ws + off);
  w.c.max_sweeps = max_sweeps;
  w.c.tol = (double)tol;
  return w;
}

// Map signature, stay table, cleared records and x_0 = 0.
static hipError_t sweep_setup(const DevModel &m, const SweepWs &w, long long vals,
                              hipStream_t st) {
  hipError_t e = launch_prep(m, w.sig, w.staytab, w.err, st);
  if (e != hipSuccess) return e;
  const long long n = std::max<long long>(w.c.max_sweeps + 2, vals);
  QV_LAUNCH(k_sweep_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w.c.res,
            w.c.vmax, w.c.max_sweeps + 2, w.c.bar, w.x[0], vals);
  return hipGetLastError();
}

// Grids up to this many cells take the one-launch form; larger ones the
// per-sweep launches.  Measured on MI355X (a sweep, one-launch vs
// per-sweep): 4096 cells, value iteration 12.3 vs 15.3 us, FIB 44.7 vs 46.4;
// 262144 cells, value iteration 20.4 vs 16.4, FIB 138 vs 123, blind bound
// 162 vs 46 -- at that size the coherent loads of the gathered values (past
// the L2) cost more than the launches they save.
constexpr long long kCoopMaxCells = 16384;

// Workgroups of a cooperative launch of `kernel`: at most `want`, and no
// more than can be resident at once; 0 for the per-sweep form: a grid of
// more than kCoopMaxCells cells, no cooperative launch on this device, or
// QVTS_SWEEP_LAUNCHES=1.  QVTS_SWEEP_COOP=1 takes the one-launch form at
// any size.
static int coop_grid(const void *kernel, size_t lds, int want, long long cells) {
  const char *e = std::getenv("QVTS_SWEEP_LAUNCHES");
  if (e && std::atoi(e) == 1) return 0;
  const char *f = std::getenv("QVTS_SWEEP_COOP");
  if (!(f && std::atoi(f) == 1) && cells > kCoopMaxCells) return 0;
  int dev = 0, coop = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
      !coop)
    return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, lds) != hipSuccess ||
      per < 1)
    return 0;
  return std::max(1, std::min(std::min(want, per * cus), kMaxCoopGrid));
}

// Residual and sweep count of a cooperative solve (one wait); a barrier
// wait that gave up is reported as a launch time-out.
static hipError_t read_result(const SweepWs &w, double *residual, int *sweeps,
                              hipStream_t st) {
  unsigned char buf[16];
  hipError_t e = hipMemcpyAsync(buf, w.c.out_res, 16, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  unsigned int aborted;
  memcpy(residual, buf, 8);
  memcpy(sweeps, buf + 8, 4);
  memcpy(&aborted, buf + 12, 4);
  return aborted ? hipErrorLaunchTimeOut : hipSuccess;
}

// Per-sweep form: `launch(k, in, out)` enqueues sweep k; every kViChunk
// sweeps the host reads the chunk's residuals and stops at the first sweep
// that meets the rule.  Returns the last sweep in *sweeps.
template <class F>
static hipError_t sweep_chunks(const SweepWs &w, F launch, double *residual, int *sweeps,
                               hipStream_t st) {
  std::vector<unsigned long long> hres(kViChunk), hvm(kViChunk);
  const int max_sweeps = w.c.max_sweeps;
  int done = 0;
  hipError_t e;
  for (int k0 = 1; k0 <= max_sweeps && !done; k0 += kViChunk) {
    const int k1 = std::min(max_sweeps, k0 + kViChunk - 1);
    for (int k = k0; k <= k1; ++k) launch(k, w.x[(k - 1) & 1], w.x[k & 1]);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int cnt = k1 - k0 + 1;
    e = hipMemcpyAsync(hres.data(), w.c.res + k0, cnt * 8, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(hvm.data(), w.c.vmax + k0, cnt * 8, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    for (int i = 0; i < cnt; ++i) {
      double r, vm;
      memcpy(&r, &hres[i], 8);
      memcpy(&vm, &hvm[i], 8);
      *residual = r;
      *sweeps = k0 + i;
      if (r == 0.0 || r <= w.c.tol * std::max(1.0, vm)) {
        done = 1;
        break;
      }
    }
  }
  return hipSuccess;
}

hipError_t run_value_iteration(const DevModel &m, float tol, int max_sweeps, float *Q,
                               double *residual, int *sweeps, char *ws, hipStream_t st) {
  const SweepWs w = carve(m, m.S, max_sweeps, tol, ws);
  hipError_t e = sweep_setup(m, w, m.S, st);
  if (e != hipSuccess) return e;
  const int TH = tile_rows(m.W, m.H);
  const int tiles = (m.H + TH - 1) / TH;
  const size_t lds = (size_t)(TH + 2) * (m.W + 2) * sizeof(float);
  const int G = coop_grid(reinterpret_cast<const void *>(&k_vi_coop), lds, tiles, m.S);
  if (G > 0) {
    DevModel mm = m;
    const uint32_t *sig = w.sig;
    const float *stay = w.staytab;
    int th = TH, nt = tiles;
    float *v0 = w.x[0], *v1 = w.x[1];
    SweepCtl c = w.c;
    void *args[] = {&mm, &sig, &stay, &th, &nt, &v0, &v1, &Q, &c};
    {
      TimingScope ts("k_vi_coop", st);
      e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_vi_coop), dim3(G),
                                     dim3(kBlock), args, (unsigned)lds, st);
    }
    if (e != hipSuccess) return e;
    return read_result(w, residual, sweeps, st);
  }
  e = sweep_chunks(
      w,
      [&](int k, float *in, float *out) {
        QV_LAUNCH(k_vi_sweep, dim3(tiles), dim3(kBlock), lds, st, m, w.sig, w.staytab, TH, in,
                  out, k, w.c);
      },
      residual, sweeps, st);
  if (e != hipSuccess) return e;
  const int kc = *sweeps;
  QV_LAUNCH(k_vi_q, dim3(tiles), dim3(kBlock), lds, st, m, w.sig, w.staytab, TH,
            w.x[(kc - 1) & 1], Q);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

template <int AM, int OP>
static hipError_t run_fib_am(const DevModel &m, const SweepWs &w, float *alpha,
                             double *residual, int *sweeps, hipStream_t st) {
  const long long vals = (long long)m.S * m.A;
  const int want = (int)std::min<long long>((m.S + kBlock - 1) / kBlock, 1 << 20);
  const int G = coop_grid(reinterpret_cast<const void *>(&k_fib_coop<AM, OP>), 0, want, m.S);
  hipError_t e;
  if (G > 0) {
    DevModel mm = m;
    const uint32_t *sig = w.sig;
    const float *stay = w.staytab;
    float *a0 = w.x[0], *a1 = w.x[1];
    SweepCtl c = w.c;
    void *args[] = {&mm, &sig, &stay, &a0, &a1, &alpha, &c};
    {
      TimingScope ts(OP == 0 ? "k_fib_coop" : "k_blind_coop", st);
      e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_fib_coop<AM, OP>),
                                     dim3(G), dim3(kBlock), args, 0u, st);
    }
    if (e != hipSuccess) return e;
    return read_result(w, residual, sweeps, st);
  }
  e = sweep_chunks(
      w,
      [&](int k, float *in, float *out) {
        QV_LAUNCH((k_fib_sweep<AM, OP>), dim3(want), dim3(kBlock), 0, st, m, w.sig, w.staytab,
                  in, out, k, w.c);
      },
      residual, sweeps, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(alpha, w.x[*sweeps & 1], (size_t)vals * 4, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

// op 0: the FIB equation; op 1: the blind-policy equation.
hipError_t run_fib(const DevModel &m, float tol, int max_sweeps, float *alpha,
                   double *residual, int *sweeps, char *ws, hipStream_t st, int op) {
  const long long vals = (long long)m.S * m.A;
  const SweepWs w = carve(m, vals, max_sweeps, tol, ws);
  hipError_t e = sweep_setup(m, w, vals, st);
  if (e != hipSuccess) return e;
  if (op == 1) {
    if (m.A <= 4) return run_fib_am<4, 1>(m, w, alpha, residual, sweeps, st);
    if (m.A <= 8) return run_fib_am<8, 1>(m, w, alpha, residual, sweeps, st);
    return run_fib_am<9, 1>(m, w, alpha, residual, sweeps, st);
  }
  if (m.A <= 4) return run_fib_am<4, 0>(m, w, alpha, residual, sweeps, st);
  if (m.A <= 8) return run_fib_am<8, 0>(m, w, alpha, residual, sweeps, st);
  return run_fib_am<9, 0>(m, w, alpha, residual, sweeps, st);
}

}  // namespace qv
