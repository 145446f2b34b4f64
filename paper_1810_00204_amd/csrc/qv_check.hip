// qv_check.hip -- device validation of a problem statement (the tuple of
// Sec. II on the grid world of Sec. V): the start belief must be a
// distribution over the free cells (b0 in B(X), finite, non-negative, zero
// on blocked cells, summing to 1), the reward table finite, and every
// landmark on a free cell of the grid.  One grid-stride pass writes error
// bits and the belief's total (FP64) into a small check record; the host
// reads it back and turns it into a status.
#include <cmath>
#include <cstring>

#include "qv_internal.h"

namespace qv {

constexpr int kCheckBelief = 1;     // an entry of b0 is negative, not finite, or on a blocked cell
constexpr int kCheckReward = 2;     // an entry of R is not finite
constexpr int kCheckLandmark = 4;   // a landmark is off the grid or on a blocked cell

// Record: err bits (int32) at +0, the belief total (double) at +8.
__global__ __launch_bounds__(kBlock) void k_check(DevModel m, const float *b0, int check_r,
                                                  int32_t *err, double *total) {
  __shared__ double red[kBlock / kWave];
  const long long S = m.S;
  const long long stride = (long long)gridDim.x * kBlock;
  const long long i0 = (long long)blockIdx.x * kBlock + threadIdx.x;
  int bits = 0;
  double sum = 0.0;
  for (long long s = i0; s < S; s += stride) {
    const bool blocked = m.occ[s] != 0;
    if (b0) {
      const float v = b0[s];
      if (!(v >= 0.f) || !isfinite(v) || (blocked && v != 0.f)) bits |= kCheckBelief;
      sum += (double)v;
    }
    if (check_r)
      for (int a = 0; a < m.A; ++a)
        if (!isfinite(m.R[s * m.A + a])) bits |= kCheckReward;
  }
  for (long long l = i0; l < m.L; l += stride) {
    const int c = m.lm_cell[l];
    if (c < 0 || c >= m.S || m.occ[c] != 0) bits |= kCheckLandmark;
  }
  if (bits) atomicOr(err, bits);
  if (!b0) return;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, kWave);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) red[wave] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += red[w];
    atomicAdd(total, t);
  }
}

__global__ void k_check_clear(int32_t *err, double *total) {
  *err = 0;
  *total = 0.0;
}

// Runs the checks (b0 may be null; check_r: also the reward table) with the
// 16-byte record at rec, waits, and returns a status.
int32_t run_model_check(const DevModel &m, const float *b0, bool check_r, char *rec,
                        hipStream_t st) {
  int32_t *err = (int32_t *)rec;
  double *total = (double *)(rec + 8);
  QV_LAUNCH(k_check_clear, dim3(1), dim3(1), 0, st, err, total);
  long long need = (long long)m.S > m.L ? (long long)m.S : (long long)m.L;
  int blocks = (int)((need + kBlock - 1) / kBlock);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  QV_LAUNCH(k_check, dim3(blocks), dim3(kBlock), 0, st, m, b0, check_r ? 1 : 0, err, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e);
  unsigned char host[16];
  e = hipMemcpyAsync(host, rec, 16, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_status(e);
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_status(e);
  int32_t bits;
  double tot;
  memcpy(&bits, host, 4);
  memcpy(&tot, host + 8, 8);
  if (bits & (kCheckReward | kCheckLandmark)) return QV_ERR_INVALID_ARG;
  if (bits & kCheckBelief) return QV_ERR_BELIEF_INVALID;
  if (b0 && !(std::fabs(tot - 1.0) <= 1e-5)) return QV_ERR_BELIEF_INVALID;
  return QV_OK;
}

}  // namespace qv
