// qv_vi.hip -- Q-MDP value iteration on gfx950 (the MDP value iteration of
// Sec. V-B; equivalently the FIB alpha-vector recursion of Sec. IV-A with a
// perfect sensor).  Jacobi sweeps in FP32 over bands of rows with a
// one-cell halo; the sweep residual max_s |V_{k+1}(s) - V_k(s)| is formed in
// FP64 (exact for a difference of two FP32 values) and max-reduced with an
// integer atomic on the bit pattern, which is order independent.  Sweeps
// are enqueued in chunks; each sweep first reads the previous residual and
// does nothing once the stopping rule has fired, so the host only
// synchronises once per chunk.
#include <algorithm>
#include <cstring>
#include <vector>

#include "qv_internal.h"

namespace qv {

constexpr int kViChunk = 32;

// V band: off-grid and blocked cells read as zero (their value is 0), the
// goal keeps its value.
__device__ __forceinline__ void load_vband(const DevModel &m, const uint32_t *sig,
                                           const float *V, int y0, int th, float *band,
                                           int BW) {
  const int n = (th + 2) * BW;
  const float rBW = 1.0f / (float)BW;
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const int r = fdiv(i, BW, rBW);
    const int gy = y0 - 1 + r, gx = i - r * BW - 1;
    float v = 0.f;
    if (gy >= 0 && gy < m.H && gx >= 0 && gx < m.W) {
      const int s = gy * m.W + gx;
      if (sig[s] & kSigFree) v = V[s];
    }
    band[i] = v;
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

__device__ __forceinline__ bool vi_converged(const unsigned long long *res,
                                             const unsigned long long *vmax, int k,
                                             double tol) {
  const double r = __longlong_as_double((long long)res[k]);
  const double vm = __longlong_as_double((long long)vmax[k]);
  return r == 0.0 || r <= tol * fmax(1.0, vm);
}

__global__ void k_vi_fill(unsigned long long *res, unsigned long long *vmax, int n, float *V0,
                          int S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    res[i] = 0ull;
    vmax[i] = 0ull;
  }
  if (i < S) V0[i] = 0.f;
}

// sweep k >= 1: V_k from V_{k-1}
__global__ __launch_bounds__(kBlock) void k_vi_sweep(DevModel m, const uint32_t *sig,
                                                     const float *staytab, int TH,
                                                     const float *Vin, float *Vout, int k,
                                                     double tol, unsigned long long *res,
                                                     unsigned long long *vmax) {
  if (k > 1 && vi_converged(res, vmax, k - 1, tol)) return;
  extern __shared__ float smem[];
  __shared__ double red[2][kBlock / kWave];
  const int W = m.W, BW = W + 2;
  const int y0 = blockIdx.x * TH;
  const int th = min(TH, m.H - y0);
  float *band = smem;
  load_vband(m, sig, Vin, y0, th, band, BW);
  __syncthreads();
  const float rW = 1.0f / (float)W;
  double rmax = 0.0, vm = 0.0;
  for (int i = threadIdx.x; i < th * W; i += kBlock) {
    const int ly = fdiv(i, W, rW), lx = i - ly * W;
    const int t = (y0 + ly) * W + lx;
    const uint32_t sg = sig[t];
    float best = 0.f;
    if (sg & kSigFree) {
      best = -INFINITY;
      for (int a = 0; a < m.A; ++a) best = fmaxf(best, cell_q(m, band, BW, ly, lx, sg, staytab, a, t));
      const double d = fabs((double)best - (double)band[(ly + 1) * BW + lx + 1]);
      rmax = fmax(rmax, d);
      vm = fmax(vm, fabs((double)best));
    }
    Vout[t] = best;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    rmax = fmax(rmax, __shfl_xor(rmax, o, kWave));
    vm = fmax(vm, __shfl_xor(vm, o, kWave));
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) {
    red[0][wave] = rmax;
    red[1][wave] = vm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) {
      rmax = fmax(rmax, red[0][w]);
      vm = fmax(vm, red[1][w]);
    }
    // non-negative doubles order like their bit patterns
    atomicMax(&res[k], (unsigned long long)__double_as_longlong(rmax));
    atomicMax(&vmax[k], (unsigned long long)__double_as_longlong(vm));
  }
}

// Q_k(s,.) from V_{k-1}, the Q-values of the last sweep (same arithmetic).
__global__ __launch_bounds__(kBlock) void k_vi_q(DevModel m, const uint32_t *sig,
                                                 const float *staytab, int TH, const float *V,
                                                 float *Q) {
  extern __shared__ float smem[];
  const int W = m.W, BW = W + 2;
  const int y0 = blockIdx.x * TH;
  const int th = min(TH, m.H - y0);
  float *band = smem;
  load_vband(m, sig, V, y0, th, band, BW);
  __syncthreads();
  const float rW = 1.0f / (float)W;
  for (int i = threadIdx.x; i < th * W; i += kBlock) {
    const int ly = fdiv(i, W, rW), lx = i - ly * W;
    const int t = (y0 + ly) * W + lx;
    const uint32_t sg = sig[t];
    for (int a = 0; a < m.A; ++a)
      Q[(size_t)t * m.A + a] = (sg & kSigFree) ? cell_q(m, band, BW, ly, lx, sg, staytab, a, t) : 0.f;
  }
}

size_t vi_ws(const qv_model *m, int max_sweeps) {
  const size_t S = (size_t)m->W * m->H;
  size_t off = 0;
  off += align_up(S * 4, 256);                       // sig
  off += align_up((size_t)m->A * 256 * 4, 256);      // staytab
  off += 2 * align_up(S * 4, 256);                   // V ping-pong
  off += 2 * align_up((size_t)(max_sweeps + 2) * 8, 256);  // res, vmax
  off += 256;                                        // err
  return off;
}

hipError_t run_value_iteration(const DevModel &m, float tol, int max_sweeps, float *Q,
                               double *residual, int *sweeps, char *ws, hipStream_t st) {
  const size_t S = (size_t)m.S;
  size_t off = 0;
  uint32_t *sig = (uint32_t *)(ws + off);
  off += align_up(S * 4, 256);
  float *staytab = (float *)(ws + off);
  off += align_up((size_t)m.A * 256 * 4, 256);
  float *V[2];
  V[0] = (float *)(ws + off);
  off += align_up(S * 4, 256);
  V[1] = (float *)(ws + off);
  off += align_up(S * 4, 256);
  unsigned long long *res = (unsigned long long *)(ws + off);
  off += align_up((size_t)(max_sweeps + 2) * 8, 256);
  unsigned long long *vmax = (unsigned long long *)(ws + off);
  off += align_up((size_t)(max_sweeps + 2) * 8, 256);
  int32_t *err = (int32_t *)(ws + off);

  hipError_t e = launch_prep(m, sig, staytab, err, st);
  if (e != hipSuccess) return e;
  const int nfill = std::max<int>(max_sweeps + 2, m.S);
  QV_LAUNCH(k_vi_fill, dim3((nfill + 255) / 256), dim3(256), 0, st, res, vmax,
                     max_sweeps + 2, V[0], m.S);
  const int TH = tile_rows(m.W, m.H);
  const int tiles = (m.H + TH - 1) / TH;
  const size_t lds = (size_t)(TH + 2) * (m.W + 2) * sizeof(float);
  const double dtol = (double)tol;
  std::vector<unsigned long long> hres(kViChunk), hvm(kViChunk);
  int done = 0;
  for (int k0 = 1; k0 <= max_sweeps && !done; k0 += kViChunk) {
    const int k1 = std::min(max_sweeps, k0 + kViChunk - 1);
    for (int k = k0; k <= k1; ++k)
      QV_LAUNCH(k_vi_sweep, dim3(tiles), dim3(kBlock), lds, st, m, sig, staytab, TH,
                         V[(k - 1) & 1], V[k & 1], k, dtol, res, vmax);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int cnt = k1 - k0 + 1;
    e = hipMemcpyAsync(hres.data(), res + k0, cnt * 8, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(hvm.data(), vmax + k0, cnt * 8, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    for (int i = 0; i < cnt; ++i) {
      double r, vm;
      memcpy(&r, &hres[i], 8);
      memcpy(&vm, &hvm[i], 8);
      *residual = r;
      *sweeps = k0 + i;
      if (r == 0.0 || r <= dtol * std::max(1.0, vm)) {
        done = 1;
        break;
      }
    }
  }
  const int kc = *sweeps;
  QV_LAUNCH(k_vi_q, dim3(tiles), dim3(kBlock), lds, st, m, sig, staytab, TH,
                     V[(kc - 1) & 1], Q);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

}  // namespace qv
