// qv_device.h -- device-side building blocks shared by the gfx950 kernels of
// libqvts: the per-cell map signature, the slip stencil in gather form, the
// wall-bit/landmark sensor, Philox4x32-10, and wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qv {

constexpr int kBlock = 256;   // threads per workgroup for the tiled kernels
constexpr int kWave = 64;     // CDNA wavefront width
// ints per sorted leaf band: kBlock chunk ranges, the first chunk of each
// wall reading (17), the first sorted position of each wall reading (17)
constexpr int kSortChunkInts = 2 * kBlock + 34;

// Model as passed to kernels by value (small tables live in the kernarg
// segment, so uniform indexing lands them in scalar registers).
struct DevModel {
  int W, H, S, A, L, goal;
  float gamma, lm_p;
  float slip[81];
  float flip[4];
  const uint8_t *occ;
  const int32_t *lm_cell;
  const float *R;
};

// ---------------------------------------------------------------------------
// Per-cell map signature, built once per call from the occupancy grid.
//   bits 0..7  : neighbour k (k = 0,1,2,3,5,6,7,8 in that order) is inside the
//                grid and free, i.e. a move towards it succeeds (Sec. V)
//   bit  8     : the cell is free
//   bit  9     : the cell is the absorbing goal
//   bits 10..13: true wall reading (bit 0 up, 1 left, 2 right, 3 down;
//                1 = occupied or off-grid), the noiseless sensor output
//   bits 14..22: landmark id (0 = none)
// ---------------------------------------------------------------------------
constexpr uint32_t kSigFree = 1u << 8;
constexpr uint32_t kSigGoal = 1u << 9;
__device__ __forceinline__ uint32_t sig_out8(uint32_t s) { return s & 0xFFu; }
__device__ __forceinline__ uint32_t sig_wall(uint32_t s) { return (s >> 10) & 0xFu; }
__device__ __forceinline__ uint32_t sig_lm(uint32_t s) { return (s >> 14) & 0x1FFu; }

// Predicted mass at cell t under action a, gathered from the 3x3 band
// neighbourhood `c` (row pitch BW) of the parent belief:
//   b'(t) = sum_{j != 4} T'(a, 8-j) b(t + d_j) + stay(t,a) b(t),
// where the band holds zeros off-grid, on blocked cells and on the goal (so
// those never act as sources), stay(t,a) = T'(a,4) plus the slip mass aimed
// at blocked/off-grid neighbours (or 1 at the goal), and `self` is b(t).
__device__ __forceinline__ float stencil(const float *c, int BW, const float *sl,
                                         float stay, float self) {
  float v = sl[8] * c[-BW - 1];
  v = fmaf(sl[7], c[-BW], v);
  v = fmaf(sl[6], c[-BW + 1], v);
  v = fmaf(sl[5], c[-1], v);
  v = fmaf(sl[3], c[1], v);
  v = fmaf(sl[2], c[BW - 1], v);
  v = fmaf(sl[1], c[BW], v);
  v = fmaf(sl[0], c[BW + 1], v);
  return fmaf(stay, self, v);
}

// Wall-bit likelihood O_w(zw | w) = prod_j (bit j misread ? f_j : 1 - f_j).
__device__ __forceinline__ float wall_lik(const float *f, uint32_t zw, uint32_t w) {
  uint32_t mis = zw ^ w;
  float o = (mis & 1u) ? f[0] : 1.f - f[0];
  o *= (mis & 2u) ? f[1] : 1.f - f[1];
  o *= (mis & 4u) ? f[2] : 1.f - f[2];
  o *= (mis & 8u) ? f[3] : 1.f - f[3];
  return o;
}

// Landmark factor O_l(zl | cell with landmark id lm).
__device__ __forceinline__ float lm_lik(float rho, uint32_t zl, uint32_t lm) {
  if (zl == 0u) return lm ? 1.f - rho : 1.f;
  return (lm == zl) ? rho : 0.f;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC 2011): ten rounds of the 4x32 S-box with
// multipliers 0xD2511F53 / 0xCD9E8D57 and key increments 0x9E3779B9 /
// 0xBB67AE85.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

__device__ __forceinline__ float u24(uint32_t r) {
  return (float)(r >> 8) * (1.0f / 16777216.0f);
}

// ---------------------------------------------------------------------------
// reductions (fixed order, hence bitwise reproducible)
// ---------------------------------------------------------------------------
// One step of a wavefront reduction on the DPP network: v plus the value of
// the lane selected by CTRL, for the rows enabled in ROW_MASK (others add 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
  const int s = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false);
  return v + __int_as_float(s);
}

// The value of the neighbouring lane (lane ^ 1), on the DPP network.
__device__ __forceinline__ float dpp_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// Sum over each row of 16 lanes, returned to every lane of the row (pairs,
// quads, half rows, then rows; every lane adds the same operands, so all
// hold the same bits).
__device__ __forceinline__ float row16_sum(float v) {
  v = dpp_add<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xF>(v);   // row_half_mirror
  v = dpp_add<0x140, 0xF>(v);   // row_mirror
  return v;
}

// Sum over aligned groups of TPB = 16, 32 or 64 lanes on the DPP network; the
// group's total is valid in its last lane.
template <int TPB>
__device__ __forceinline__ float group_sum(float v);

// Sum over the 64 lanes in a fixed order; the total lands in lane 63
// (pairs, quads, half rows, rows, then rows broadcast into rows 1/3 and 2/3).
__device__ __forceinline__ float wave_total_lane63(float v) {
  v = dpp_add<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xF>(v);   // row_half_mirror
  v = dpp_add<0x140, 0xF>(v);   // row_mirror
  v = dpp_add<0x142, 0xA>(v);   // row_bcast:15
  v = dpp_add<0x143, 0xC>(v);   // row_bcast:31
  return v;
}

template <int TPB>
__device__ __forceinline__ float group_sum(float v) {
  static_assert(TPB == 16 || TPB == 32 || TPB == 64, "groups of 16, 32 or 64 lanes");
  if constexpr (TPB == 64) return wave_total_lane63(v);
  v = row16_sum(v);
  if constexpr (TPB == 32) v = dpp_add<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  return v;
}

// Inclusive prefix sum of integers over the 64 lanes on the DPP network
// (within rows of 16 by shifts of 1, 2, 4, 8, then rows 0 -> 1 and 2 -> 3,
// then rows 0-1 -> 2-3).
__device__ __forceinline__ int wave_scan_incl(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);   // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);   // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);   // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);   // row_bcast:31
  return v;
}

// As wave_scan_incl, on unsigned integers (sums modulo 2^32).
__device__ __forceinline__ uint32_t wave_scan_incl_u32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);   // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);   // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);   // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);   // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);   // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);   // row_bcast:31
  return v;
}

// Wavefront total, returned to every lane.
__device__ __forceinline__ float wave_sum(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_total_lane63(v)), 63));
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
  return v;
}

// Floor division for 0 <= i < 2^23 and 1 <= d < 2^14 through an FP32
// reciprocal, corrected to the exact quotient.
__device__ __forceinline__ int fdiv(int i, int d, float rd) {
  int q = (int)((float)i * rd);
  q -= (q * d > i);
  q += ((q + 1) * d <= i);
  return q;
}

}  // namespace qv
