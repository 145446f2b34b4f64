// qv_plan.hip -- level-synchronous QV-tree expansion on gfx950.
//
// One planning step builds the depth-D tree of Alg. 1-7 (Sec. IV-C) one
// frontier at a time.  Work items are (parent slot, band of rows, action):
// every Q-node of the level is spread over many workgroups.  For each level
// d < D:
//   k_stats   predicted belief b' = T_a^T b (slip stencil, Sec. V) reduced to
//             a 16-bin histogram by true wall reading, the predicted mass on
//             each landmark cell, and R(b,a) (Sec. III).  The last band of a
//             Q-node to finish then forms P(z|b,a) over all z and draws the n
//             observations (Alg. 3/4), keeping each distinct z with its
//             frequency;
//   k_update  (d < D-1) writes the child beliefs Phi(b,a,z) (posterior belief
//             update, Sec. III) for the next level, or
//   k_leaf    (d = D-1) forms the same posterior values and scores them on the
//             fly against the Q-MDP vectors, sum_s b(s) Q(s,a') (Alg. 5),
//             without storing them.  The last workgroup to finish a node
//             completes its backup (Alg. 6/7) and, as the last child of its
//             parent, the parent's, up to the root.
// Beliefs stream through LDS in bands of whole rows with a one-cell halo;
// all cross-workgroup sums run in a fixed order, so results are bitwise
// reproducible.
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "qv_internal.h"

namespace qv {

// ---------------------------------------------------------------------------
// map signature, stay table, counters
// ---------------------------------------------------------------------------
// Signature of cell s without its landmark id: the 8-neighbour move pattern
// (bit set = the move is possible), free and goal bits, and the true wall
// reading in bits 10..13.
// The nine occupancy reads go out together: an off-grid neighbour reads the
// cell itself and is masked (bitwise conditions, so no branch guards a load).
__device__ __forceinline__ uint32_t cell_bits(const DevModel &m, int s) {
  const int y = s / m.W, x0 = s - y * m.W;
  uint32_t o[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int ny = y + k / 3 - 1, nx = x0 + k % 3 - 1;
    const uint32_t in = (uint32_t)(ny >= 0) & (uint32_t)(ny < m.H) & (uint32_t)(nx >= 0) &
                        (uint32_t)(nx < m.W);
    const uint32_t oc = m.occ[in ? ny * m.W + nx : s];
    o[k] = in & (uint32_t)(oc == 0);   // 1: the move to neighbour k is possible
  }
  uint32_t v = 0;
  int bit = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (k == 4) continue;
    v |= o[k] << bit;
    ++bit;
  }
  if (o[4]) v |= kSigFree;
  if (s == m.goal) v |= kSigGoal;
  // wall bits up/left/right/down are neighbours k = 1, 3, 5, 7 -> bits 1, 3, 4, 6
  const uint32_t w = (((v >> 1) & 1u) ^ 1u) | ((((v >> 3) & 1u) ^ 1u) << 1) |
                     ((((v >> 4) & 1u) ^ 1u) << 2) | ((((v >> 6) & 1u) ^ 1u) << 3);
  return v | (w << 10);
}

// stay(a, pattern) from the slip row of a: T'(a,4) plus the slip mass of
// every move whose target is blocked or off-grid (bit clear in the
// 8-neighbour pattern).
__device__ __forceinline__ float stay_value(const float (&sl)[9], int pat) {
  float st = sl[4];
  int bit = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (k == 4) continue;
    st += ((pat >> bit) & 1) ? 0.f : sl[k];
    ++bit;
  }
  return st;
}

// Thread g of the prep pass of one query: clears the error word, writes the
// root records and the counters and the stay table (everything but the
// signatures).
__device__ void prep_misc_one(const DevModel &m, float *staytab, int32_t *err,
                              const PrepExtra &x, long long g) {
  const int s = (int)g;
  if (g == 0) {
    err[0] = 0;
    if (x.valid) {
      x.valid[0] = 1;
      x.z[0] = -1;
      x.count[0] = 0;
      x.pz[0] = 0.f;
    }
  }
  if (g < x.nzero) x.zero[g] = 0;
  if (g < m.A * 256) {
    float sl[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) sl[k] = m.slip[(s >> 8) * 9 + k];
    staytab[s] = stay_value(sl, s & 255);
  }
}

// As prep_misc_one, plus the signature of cell g (without landmark ids).
__device__ void prep_sig_one(const DevModel &m, uint32_t *sig, float *staytab, int32_t *err,
                             const PrepExtra &x, long long g) {
  prep_misc_one(m, staytab, err, x, g);
  if (g < m.S) sig[g] = cell_bits(m, (int)g);
}

__global__ void k_prep_sig(DevModel m, uint32_t *sig, float *staytab, int32_t *err,
                           PrepExtra x) {
  prep_sig_one(m, sig, staytab, err, x, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// Landmark l of one query: its id goes into the signature of its cell.
__device__ void prep_landmark_one(const DevModel &m, uint32_t *sig, int32_t *err,
                                  uint32_t *lm_wall, int l) {
  if (l >= m.L) return;
  const int c = m.lm_cell[l];
  if (c < 0 || c >= m.S) {
    if (lm_wall) lm_wall[l] = 0xFFFFFFFFu;   // never observed
    atomicOr(err, 1);
    return;
  }
  if (lm_wall) lm_wall[l] = sig_wall(sig[c]);
  // a cell carries at most one landmark id: a second one is refused and flagged
  uint32_t cur = sig[c];
  while (sig_lm(cur) == 0u) {
    const uint32_t prev = atomicCAS(&sig[c], cur, cur | ((uint32_t)(l + 1) << 14));
    if (prev == cur) return;
    cur = prev;
  }
  atomicOr(err, 2);
}

__global__ void k_prep_landmarks(DevModel m, uint32_t *sig, int32_t *err, uint32_t *lm_wall) {
  prep_landmark_one(m, sig, err, lm_wall, blockIdx.x * blockDim.x + threadIdx.x);
}

// The prep pass of a plan in one launch: as k_prep_sig, with each cell's
// landmark id found by a scan of the landmark list (staged in LDS; the
// lowest id wins if two share a cell) instead of a second launch that
// inserts the ids.  Every landmark on a cell takes the cell's wall reading;
// a landmark off the grid reads all ones.  The occupancy loads of a cell's
// bits go out together with the landmark list's, so the pass costs one
// round trip to memory.  Landmark errors are not flagged here (a plan does
// not read the error word).
__global__ __launch_bounds__(256) void k_prep_plan(DevModel m, uint32_t *sig, float *staytab,
                                                   int32_t *err, PrepExtra x) {
  static_assert(QV_MAX_LANDMARKS <= 2 * 256, "two landmarks per thread");
  __shared__ int s_lm[QV_MAX_LANDMARKS];
  __shared__ uint32_t s_v[256];   // this workgroup's cells' signatures
  __shared__ int s_id[256];       // the smallest landmark id on each of them
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = (int)g;
  // every load first, at valid addresses (masked afterwards), so that one
  // wait covers them all
  int lmc[2] = {0, 0};
  if (m.L > 0) {   // lm_cell may be null without landmarks
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int l = threadIdx.x + k * 256;
      lmc[k] = m.lm_cell[l < m.L ? l : 0];
    }
  }
  const int sc = g < m.S ? s : 0;
  const uint32_t v = cell_bits(m, sc);
  const int sa = g < m.A * 256 ? s >> 8 : 0;
  float sl[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) sl[k] = m.slip[sa * 9 + k];
#pragma unroll
  for (int k = 0; k < 2; ++k)
    if (threadIdx.x + k * 256 < m.L) s_lm[threadIdx.x + k * 256] = lmc[k];
  s_v[threadIdx.x] = v;
  s_id[threadIdx.x] = 0x7fffffff;
  if (g < m.A * 256) staytab[s] = stay_value(sl, s & 255);
  if (g == 0) {
    err[0] = 0;
    if (x.valid) {
      x.valid[0] = 1;
      x.z[0] = -1;
      x.count[0] = 0;
      x.pz[0] = 0.f;
    }
  }
  if (g < x.nzero) x.zero[g] = 0;
  __syncthreads();
  // landmarks on this workgroup's cells: the cell takes the smallest id of
  // those on it; every such landmark records the cell's wall reading
  const long long base = (long long)blockIdx.x * blockDim.x;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int l = threadIdx.x + k * 256;
    if (l < m.L) {
      const long long c = lmc[k];
      if (c >= base && c < base + 256 && c < m.S) {
        atomicMin(&s_id[c - base], l + 1);
        x.lm_wall[l] = sig_wall(s_v[c - base]);
      }
    }
  }
  __syncthreads();
  if (g < m.S) {
    const int id = s_id[threadIdx.x];
    sig[s] = id != 0x7fffffff ? v | ((uint32_t)id << 14) : v;
  }
  if (g < m.L) {
    const int c = s_lm[g];
    if (c < 0 || c >= m.S) x.lm_wall[g] = 0xFFFFFFFFu;
  }
}

// Sorted cell entries: bits 0..21 the cell index (S <= 2048 * 2048 = 2^22),
// bits 22..29 the cell's 8-neighbour move pattern (signature bits 0..7),
// bit 30 goal, bit 31 landmark.
constexpr uint32_t kSortCell = 0x3FFFFFu;
constexpr int kSortOutShift = 22;
constexpr uint32_t kSortGoal = 1u << 30;
constexpr uint32_t kSortLandmark = 1u << 31;

// Free cells of one band of rows grouped by their true wall reading w
// (stable: ascending cell index within a reading), for the leaf-level
// wall-reading histograms.  The band's cells are [c_lo, c_hi); its ordered
// list takes the same positions of `cells`, cut into at most kBlock chunks
// of at most C cells, each holding one reading only: with
// C = ceil(Sf / (kBlock - 16)) for the band's Sf free cells, the 16
// readings need sum_w ceil(n_w / C) <= Sf / C + 16 <= kBlock chunks.
//   cells[c_lo + k]             ordered free cells (packed entries, see above)
//   chunk[2k], chunk[2k+1]      first and one-past-last position of chunk k
//                               (equal for unused k)
//   chunk[2 kBlock + w]         first chunk of reading w, w = 0..16
//   chunk[2 kBlock + 17 + w]    first position of reading w, w = 0..16
// One workgroup per band; thread i first counts cells c_lo + [i R, (i+1) R).
constexpr int kSortMaxCells = 16384;   // cells of one sorted band (leaf bands <= 8192)
// per-cell summary kept in LDS while sorting: bits 0..7 move pattern, 8..11
// wall reading, 12 free, 13 goal, 14 landmark
// DYN: the tables live in the caller's LDS at `lds` (sort_band_lds_bytes of
// the band's cells) instead of static arrays sized for kSortMaxCells, so a
// kernel that sorts in a few of its workgroups keeps its other workgroups
// small.
template <int NT>
__host__ __device__ inline size_t sort_band_lds_bytes(int cells) {
  return (size_t)(17 * NT + NT / kWave + 17 + 17 + 1) * 4 + (size_t)(cells + NT + 2) * 2;
}
template <int NT = kBlock, bool DYN = false>
__device__ void sort_band(int c_lo, int c_hi, int L, const uint32_t *sig, int32_t *cells,
                          int32_t *chunk, void *lds = nullptr) {
  // [w][thread], then exclusive offsets; entry e at e + e / 16 (one pad word
  // per 16), so a thread's 16 consecutive entries and its neighbours' fall in
  // different LDS banks
  int *cnt, *wtot, *s_start, *s_pchunk, *s_Cp;
  uint16_t *cs;
  if constexpr (DYN) {
    cnt = (int *)lds;
    wtot = cnt + 17 * NT;
    s_start = wtot + NT / kWave;
    s_pchunk = s_start + 17;
    s_Cp = s_pchunk + 17;
    cs = (uint16_t *)(s_Cp + 1);
  } else {
    __shared__ int cnt_s[17 * NT];
    __shared__ uint16_t cs_s[kSortMaxCells + NT + 2];
    __shared__ int wtot_s[NT / kWave];
    __shared__ int start_s[17], pchunk_s[17], c_s;
    cnt = cnt_s;
    cs = cs_s;
    wtot = wtot_s;
    s_start = start_s;
    s_pchunk = pchunk_s;
    s_Cp = &c_s;
  }
  auto cx = [](int e) { return e + (e >> 4); };
  const int tid = threadIdx.x;
  const int S = c_hi - c_lo;
  // thread i counts and scatters cells [i R, (i+1) R); cell c sits at
  // c + c / R in cs, so each thread's cells are R + 1 entries apart from its
  // neighbour's (an odd stride in 16-bit words: two lanes per LDS bank
  // instead of R)
  static_assert(kSortMaxCells / NT < 256, "a thread's counts fit 8-bit fields");
  const int R = (S + NT - 1) / NT;
  const float rR = 1.0f / (float)R;
  // the band's signatures, coalesced, all of a thread's loads in flight
  // together for a band of 8192 cells
  constexpr int LB = 8192 / NT;
  for (int i0 = tid; i0 < S; i0 += LB * NT) {
    uint32_t sg[LB];
#pragma unroll
    for (int k = 0; k < LB; ++k) {
      const int i = i0 + k * NT;
      const uint32_t sv = sig[c_lo + (i < S ? i : 0)];   // every lane loads, then masks
      sg[k] = i < S ? sv : 0u;
    }
#pragma unroll
    for (int k = 0; k < LB; ++k) {
      const int i = i0 + k * NT;
      if (i < S) {
        const uint32_t lm = sig_lm(sg[k]);
        cs[i + fdiv(i, R, rR)] = (uint16_t)(sig_out8(sg[k]) | (sig_wall(sg[k]) << 8) |
                           ((sg[k] & kSigFree) ? 1u << 12 : 0u) |
                           ((sg[k] & kSigGoal) ? 1u << 13 : 0u) |
                           ((lm && lm <= (uint32_t)L) ? 1u << 14 : 0u));
      }
    }
  }
  __syncthreads();
  const int c0 = min(S, tid * R), c1 = min(S, c0 + R);   // band-relative
  const uint16_t *mine = cs + tid;                        // cell t at mine[t]
  // free cells per wall reading, as 8-bit fields (a thread has <= 64 cells):
  // readings 0..7 in lo, 8..15 in hi; eight LDS reads in flight at a time
  uint64_t nlo = 0, nhi = 0;
  for (int t0 = c0; t0 < c1; t0 += 8) {
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = t0 + k < c1 ? (uint32_t)mine[t0 + k] : 0u;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t w = (v[k] >> 8) & 15u;
      const uint64_t one = (v[k] & (1u << 12)) ? 1ull << (8 * (w & 7u)) : 0ull;
      nlo += w < 8u ? one : 0ull;
      nhi += w < 8u ? 0ull : one;
    }
  }
#pragma unroll
  for (int w = 0; w < 16; ++w)
    cnt[cx(w * NT + tid)] = (int)(((w < 8 ? nlo : nhi) >> (8 * (w & 7))) & 255u);
  __syncthreads();
  // exclusive scan of cnt in (w, thread) order: thread i owns entries
  // [16 i, 16 i + 16), then the NT owner totals are scanned
  int loc[16], sum = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    loc[k] = sum;
    sum += cnt[cx(16 * tid + k)];
  }
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  const int inc = wave_scan_incl(sum);
  if (lane == kWave - 1) wtot[wave] = inc;
  __syncthreads();
  int base = inc - sum;
  for (int v = 0; v < wave; ++v) base += wtot[v];
#pragma unroll
  for (int k = 0; k < 16; ++k) cnt[cx(16 * tid + k)] = base + loc[k];
  __syncthreads();
  if (tid == 0) {
    int Sf = 0;
    for (int v = 0; v < NT / kWave; ++v) Sf += wtot[v];
    const int C = max(1, (Sf + (kBlock - 16) - 1) / (kBlock - 16));
    int pc = 0;
    for (int w = 0; w < 16; ++w) {
      s_start[w] = cnt[cx(w * NT)];
      s_pchunk[w] = pc;
      const int nw = (w < 15 ? cnt[cx((w + 1) * NT)] : Sf) - cnt[cx(w * NT)];
      pc += (nw + C - 1) / C;
    }
    s_start[16] = Sf;
    s_pchunk[16] = pc;
    *s_Cp = C;
  }
  // scatter: each thread walks its cells again in order; a cell's position
  // is its reading's offset for this thread (cnt, read from LDS) plus the
  // thread's earlier cells of that reading (the same 8-bit fields)
  uint64_t rlo = 0, rhi = 0;
  for (int t0 = c0; t0 < c1; t0 += 8) {
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = t0 + k < c1 ? (uint32_t)mine[t0 + k] : 0u;
    int base[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) base[k] = cnt[cx((int)((v[k] >> 8) & 15u) * NT + tid)];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t c = v[k];
      if (!(c & (1u << 12))) continue;   // blocked, or past the thread's cells
      const uint32_t w = (c >> 8) & 15u, sh8 = 8 * (w & 7u);
      const int pos = base[k] + (int)(((w < 8u ? rlo : rhi) >> sh8) & 255u);
      if (w < 8u)
        rlo += 1ull << sh8;
      else
        rhi += 1ull << sh8;
      cells[c_lo + pos] = (int32_t)((uint32_t)(c_lo + t0 + k) | ((c & 0xFFu) << kSortOutShift) |
                                    ((c & (1u << 13)) ? kSortGoal : 0u) |
                                    ((c & (1u << 14)) ? kSortLandmark : 0u));
    }
  }
  __syncthreads();
  // chunk k (one per thread of the leaf kernel, kBlock of them) belongs to
  // the reading w with pchunk[w] <= k < pchunk[w+1]
  if (tid < kBlock) {
    int w = 0;
    while (w < 16 && s_pchunk[w + 1] <= tid) ++w;
    int j0 = 0, j1 = 0;
    if (w < 16) {
      j0 = s_start[w] + (tid - s_pchunk[w]) * *s_Cp;
      j1 = min(j0 + *s_Cp, s_start[w + 1]);
    }
    chunk[2 * tid] = c_lo + j0;
    chunk[2 * tid + 1] = c_lo + j1;
  }
  if (tid <= 16) {
    chunk[2 * kBlock + tid] = s_pchunk[tid];
    chunk[2 * kBlock + 17 + tid] = c_lo + s_start[tid];
  }
}

// band = blockIdx.x: cells [band * TC, min(S, (band + 1) * TC))
__global__ __launch_bounds__(kBlock) void k_prep_sort(int S, int TC, int L, const uint32_t *sig,
                                                       int32_t *cells, int32_t *chunk) {
  const int c_lo = blockIdx.x * TC;
  sort_band(c_lo, min(S, c_lo + TC), L, sig, cells, chunk + (size_t)blockIdx.x * kSortChunkInts);
}

static void prep_launch(const DevModel &dm, uint32_t *sig, float *staytab, int32_t *err,
                        const PrepExtra &x, hipStream_t st) {
  const long long n = std::max<long long>(std::max(dm.S, dm.A * 256), x.nzero);
  QV_LAUNCH(k_prep_sig, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dm, sig, staytab,
            err, x);
  if (dm.L > 0)
    QV_LAUNCH(k_prep_landmarks, dim3((dm.L + 255) / 256), dim3(256), 0, st, dm, sig, err,
              x.lm_wall);
}

static void prep_plan_launch(const DevModel &dm, uint32_t *sig, float *staytab, int32_t *err,
                             const PrepExtra &x, hipStream_t st) {
  const long long n =
      std::max<long long>(std::max<long long>(std::max(dm.S, dm.A * 256), x.nzero), dm.L);
  QV_LAUNCH(k_prep_plan, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dm, sig, staytab,
            err, x);
}

hipError_t launch_prep(const DevModel &dm, uint32_t *sig, float *staytab, int32_t *err,
                       hipStream_t st) {
  const PrepExtra none = {nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr};
  prep_launch(dm, sig, staytab, err, none, st);
  return hipGetLastError();
}

hipError_t launch_prep_lm(const DevModel &dm, uint32_t *sig, float *staytab, int32_t *err,
                          uint32_t *lm_wall, hipStream_t st) {
  const PrepExtra x = {nullptr, nullptr, nullptr, nullptr, nullptr, 0, lm_wall};
  prep_launch(dm, sig, staytab, err, x, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// shared pieces of the tiled kernels
// ---------------------------------------------------------------------------

// Rows y0-1 .. y0+th of belief b, columns -1 .. W, into LDS (pitch BW=W+2).
// Off-grid cells and the goal read as zero: neither is a source of moving
// mass (the goal is absorbing and keeps its own mass).  Blocked cells hold
// zero mass in every belief the library forms; with `mask` (the caller's
// start belief) they are zeroed here as well.  Loads are issued in batches
// so that each thread has several in flight.
constexpr int kBandBatch = 8;
template <int BATCH = kBandBatch, int NT = kBlock>
__device__ __forceinline__ void load_band(const DevModel &m, const uint32_t *sig,
                                          const float *b, int y0, int th, float *band,
                                          int BW, bool mask) {
  const int n = (th + 2) * BW;
  const float rBW = 1.0f / (float)BW;
  for (int i0 = threadIdx.x; i0 < n; i0 += BATCH * NT) {
    int cell[BATCH];
    float v[BATCH];
#pragma unroll
    for (int j = 0; j < BATCH; ++j) {
      const int i = i0 + j * NT;
      const int r = fdiv(i, BW, rBW);
      const int gy = y0 - 1 + r, gx = i - r * BW - 1;
      const bool in = i < n && gy >= 0 && gy < m.H && gx >= 0 && gx < m.W;
      cell[j] = in ? gy * m.W + gx : -1;
      // every lane loads (cell 0 for halo and padding lanes), so the loads of
      // the batch go out together without a branch around each
      // (bitwise conditions: a short-circuit one lets the compiler move the
      // load under a branch)
      const float bv = b[in ? cell[j] : 0];
      v[j] = ((uint32_t)in & (uint32_t)(cell[j] != m.goal)) ? bv : 0.f;
    }
    if (mask) {
#pragma unroll
      for (int j = 0; j < BATCH; ++j) {
        const uint32_t sv = sig[cell[j] >= 0 ? cell[j] : 0];
        v[j] = ((uint32_t)(cell[j] >= 0) & (sv ^ kSigFree) & kSigFree) ? 0.f : v[j];
      }
    }
#pragma unroll
    for (int j = 0; j < BATCH; ++j) {
      const int i = i0 + j * NT;
      if (i < n) band[i] = v[j];
    }
  }
}

// b'(t) for cell t = (y0+ly)*W + lx of the band.
__device__ __forceinline__ float predict_cell(const float *band, int BW, int ly, int lx,
                                              uint32_t sg, const float *sl,
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

// As predict_cell with b(t) already loaded (bt).
__device__ __forceinline__ float predict_cell_v(const float *band, int BW, int ly, int lx,
                                                uint32_t sg, const float *sl,
                                                const float *stay_a, float bt) {
  if (!(sg & kSigFree)) return 0.f;
  const float *c = band + (ly + 1) * BW + lx + 1;
  if (sg & kSigGoal) return stencil(c, BW, sl, 1.f, bt);
  return stencil(c, BW, sl, stay_a[sig_out8(sg)], c[0]);
}

constexpr int kCellBatch = 4;   // cells whose loads a thread issues together
constexpr int kLeafBatch = 2;
constexpr int kNodeBatch = 16;  // the same in k_node (bound by LDS, not registers)
constexpr int kNodeBlock = 512;  // threads of an inner-level k_node workgroup

// Sum of the per-wavefront partials r[0..NW) in a fixed pairwise order.
template <int NW>
__device__ __forceinline__ float sum_waves(const float *r) {
  static_assert(NW == 4 || NW == 8, "4 or 8 wavefronts");
  if constexpr (NW == 4) return (r[0] + r[1]) + (r[2] + r[3]);
  return ((r[0] + r[1]) + (r[2] + r[3])) + ((r[4] + r[5]) + (r[6] + r[7]));
}
constexpr int kSortBatch = 8;   // cells of a leaf-histogram chunk loaded together

// k_node's dynamic LDS: b' [S], then X (the band; then chunk partials or the
// landmark terms of the draws; then the backup scratch) of this many floats,
// then (inner levels) 16 histogram bins per thread.
__host__ __device__ inline size_t small_x_floats(int W, int H, int A, int n, int L) {
  size_t x = (size_t)(H + 2) * (W + 2);
  const size_t c[4] = {(size_t)(16 + 1) * kBlock,   // leaf chunk partials, A <= 16
                       (size_t)A * n + A, (size_t)2 * L + 32, (size_t)16};
  for (int i = 0; i < 4; ++i) x = x > c[i] ? x : c[i];
  return x;
}

// Q(t, .) padded to APAD entries; float4 loads when rows are APAD wide.
// QV: 1 rows are read as float4 (A = APAD, 16-byte aligned), 0 element by
// element, -1 as lv.q_vec says.
template <int APAD, int QV = -1>
__device__ __forceinline__ void load_q_row(const LevelArgs &lv, int A, int t, float (&q)[APAD]) {
  if (APAD <= 8 && (QV == 1 || (QV == -1 && lv.q_vec))) {
    const float4 *q4 = (const float4 *)(lv.Q + (size_t)t * APAD);
#pragma unroll
    for (int c4 = 0; c4 < APAD / 4; ++c4) {
      const float4 v4 = q4[c4];
      q[4 * c4 + 0] = v4.x;
      q[4 * c4 + 1] = v4.y;
      q[4 * c4 + 2] = v4.z;
      q[4 * c4 + 3] = v4.w;
    }
  } else {
    const float *Qr = lv.Q + (size_t)t * A;
#pragma unroll
    for (int c = 0; c < APAD; ++c) q[c] = (c < A) ? Qr[c] : 0.f;
  }
}

// Sum of x[k * stride] over lo <= k < hi in a fixed order: eight running
// sums over k - lo mod 8, then added pairwise.  The last partial group loads
// all eight slots (x[0] in place of those past hi) and masks them, so its
// loads go out together.
__device__ __forceinline__ float range_sum(const float *x, int stride, int lo, int hi) {
  float s[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) s[u] = 0.f;
  int k = lo;
  for (; k + 8 <= hi; k += 8)
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += x[(k + u) * stride];
  float t[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) t[u] = x[(k + u < hi ? k + u : 0) * stride];
#pragma unroll
  for (int u = 0; u < 8; ++u) s[u] += (k + u < hi) ? t[u] : 0.f;
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// Hand-off between workgroups of one launch.  Values another workgroup will
// read are written with device-scope atomic stores (written through to the
// device-coherent level, past this XCD's L2), the writer waits until its
// stores have completed and only then bumps a counter; the workgroup that
// sees the final count reads with device-scope atomic loads.  This orders
// the hand-off without a device-scope fence, which on this GPU writes back
// and invalidates the whole L2 of the XCD.
__device__ __forceinline__ float ld_coherent(const float *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(float *p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// wait until all memory operations this thread issued have completed
__device__ __forceinline__ void wait_mem() { __builtin_amdgcn_s_waitcnt(0); }
// wait until this wavefront's LDS operations have completed (lgkmcnt(0); the
// vector memory and export counters at their maxima, so no store is waited for)
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(0xC07F); }
__device__ __forceinline__ int count_arrival(int32_t *ctr) {
  return __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup totals of 32 per-thread values: each wavefront reduces every
// value on the DPP network (total in lane 63), lane 63 stores its 32 totals,
// and thread i < 32 adds the four wavefronts' totals of value i in order.
// red: [4][32] floats.  Ends with a barrier.
template <int NT = kBlock>
__device__ __forceinline__ float block_sum32(float (&v)[32], float *red) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < 32; ++i) v[i] = wave_total_lane63(v[i]);
  if (lane == kWave - 1) {
#pragma unroll
    for (int i = 0; i < 32; ++i) red[wave * 32 + i] = v[i];
  }
  __syncthreads();
  float out = 0.f;
  if (threadIdx.x < 32) {
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) out += red[w * 32 + threadIdx.x];
  }
  __syncthreads();
  return out;
}

// ---------------------------------------------------------------------------
// observation draws of one Q-node, by one wavefront
// ---------------------------------------------------------------------------
// Copy of the drawn children kept in LDS for the rest of a workgroup.
struct DrawOut {
  int z[QV_MAX_SAMPLES], count[QV_MAX_SAMPLES];
  float inv[QV_MAX_SAMPLES];
  int U;
};

// The observations z = zw + 16 zl come in blocks of 16 (one block per zl, the
// wall reading zw inside it).  Block 0 is "no landmark seen": P(zw, 0) from
// the LDS table p0.  Block l >= 1 is landmark l: O_w(zw | w_l) rho b'(x_l),
// zero when landmark l sits on a blocked cell (w_l > 15).  O_w(zw | w)
// depends on the misread pattern zw ^ w only: otab (LDS) holds its 16 values.
// Every lane reads at valid addresses and selects, with no branch.
__device__ __forceinline__ void obs_block(int blk, int L, const float *otab, float lmp,
                                          const float *p0, const uint32_t *lw,
                                          const float *lvv, float (&v)[16]) {
  const bool lmk = blk >= 1 && blk <= L;
  const int li = lmk ? blk - 1 : 0;
  const uint32_t wl = lw[li];
  const float ml = lvv[li];
  const uint32_t w = lmk ? wl : 16u;
  const float mass = lmk ? ml : 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const float o = otab[(uint32_t)i ^ (w & 15u)];
    const float pl = w > 15u ? 0.f : o * lmp * mass;
    const float pz = p0[i];
    v[i] = blk == 0 ? pz : pl;
  }
}

// The inverse-CDF search runs on integer masses: each P(z|b,a) times a
// power of two 2^e, rounded to an integer, with e chosen from the total so
// that the integer total lies in [2^30, 2^31) (each mass keeps a resolution
// of about 2^-30 of the total).  Integer running totals are exact and their
// order of addition does not matter, so the lanes' totals are prefixed on the
// DPP network, and a z is drawn only where its integer mass is positive.
constexpr int kObsPages = (QV_MAX_LANDMARKS + 1 + kWave - 1) / kWave;   // pages of 64 blocks

// Integer masses of the 16 entries of one block and their total.
__device__ __forceinline__ uint32_t block_masses(const float (&v)[16], int e, uint32_t (&q)[16]) {
  uint32_t t = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    q[i] = (uint32_t)rintf(ldexpf(v[i], e));
    t += q[i];
  }
  return t;
}

// Observation draws of Q-node (slot p, action a) of level lv.d from its
// statistics: lane w < 16 holds H[w], the predicted mass with true wall
// reading w (landmark cells weighted by their "no landmark" factor); lw/lvv
// (LDS) hold each landmark's wall reading and predicted mass.  Forms P(z|b,a)
// over all z in ascending order, draws n observations by inverse CDF with
// Philox uniforms (the first z whose running total exceeds u times the total,
// on the integer masses above), and writes one child record per distinct z
// (ascending) with its frequency (Alg. 3/4).  One full wavefront; out (LDS)
// optional; p0tab: 32 floats of LDS (P(zw, no landmark), then the
// wall-likelihood table).
// cbase >= 0 places the child records at cbase + a*n instead of the
// capacity slots p*K + a*n (p still keys the draws).
__device__ int sample_draws(const DevModel &m, const LevelArgs &lv, int p, int a, float hs,
                             const uint32_t *lw, const float *lvv, float *p0tab, DrawOut *out,
                             int cbase = -1) {
  const int lane = threadIdx.x & (kWave - 1);
  const int n = lv.n;
  const int cb = (cbase >= 0 ? cbase : p * lv.K) + a * n;
  // the model's sensor scalars, once, as uniform registers
  float fl[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
    fl[j] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(m.flip[j])));
  const float lmp = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(m.lm_p)));
  const int L = __builtin_amdgcn_readfirstlane(m.L);
  // O_w(zw | w) by misread pattern zw ^ w, once, into the LDS table otab
  float *otab = p0tab + 16;
  if (lane < 16) otab[lane] = wall_lik(fl, (uint32_t)lane, 0u);
  wait_lds();
  __builtin_amdgcn_wave_barrier();
  // P(zw, no landmark) = sum_w O_w(zw|w) H[w] (landmark cells entered H with
  // their "no landmark" factor already), published in the LDS table p0tab
  float p0 = 0.f;
#pragma unroll
  for (int w = 0; w < 16; ++w) {
    const float hw = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hs), w));
    p0 = fmaf(otab[(uint32_t)(lane & 15) ^ (uint32_t)w], hw, p0);
  }
  if (lane < 16) p0tab[lane] = p0;
  wait_lds();
  __builtin_amdgcn_wave_barrier();
  const int npg = (L + 1 + kWave - 1) / kWave;
  // the total mass, for the scale only: the no-landmark entries sum to that
  // of H (O_w sums to 1 over readings), landmark l's block to rho b'(x_l)
  float pa = lane < 16 ? p0 : 0.f;
  for (int l = lane; l < L; l += kWave) pa += lw[l] > 15u ? 0.f : lmp * lvv[l];
  pa = wave_sum(pa);
  int ex = 0;
  (void)frexpf(pa, &ex);   // pa = f 2^ex with f in [0.5, 1)
  const int e = 31 - ex;   // pa 2^e in [2^30, 2^31)
  // integer running totals: incl[g] = total up to the end of the lane's
  // block of page g; pbase[g] = total before page g (uniform)
  uint32_t incl[kObsPages], pbase[kObsPages];
  uint32_t base = 0;
#pragma unroll
  for (int g = 0; g < kObsPages; ++g) {
    incl[g] = base;
    pbase[g] = base;
    if (g < npg) {
      float v[16];
      uint32_t q[16];
      obs_block(g * kWave + lane, L, otab, lmp, p0tab, lw, lvv, v);
      const uint32_t t = block_masses(v, e, q);
      const uint32_t c = wave_scan_incl_u32(t);
      incl[g] = base + c;
      base += (uint32_t)__builtin_amdgcn_readlane((int)c, kWave - 1);
    }
  }
  const uint32_t total = base;   // < 2^32: at most 2^31 plus rounding
  // lane k < n: its uniform from the Philox counter (a*ceil(n/4) + k/4, slot,
  // level, query), word k%4, and its integer target floor(u total), u the
  // word's top 24 bits over 2^24 (so target < total)
  uint32_t tgt = 0u;
  if (lane < n) {
    const int ng = (n + 3) / 4;
    const uint4 r = philox4x32_10(
        make_uint4((uint32_t)(a * ng + (lane >> 2)), (uint32_t)p, (uint32_t)lv.d, lv.qid),
        lv.key0, lv.key1);
    const int q = lane & 3;
    const uint32_t w = q == 0 ? r.x : q == 1 ? r.y : q == 2 ? r.z : r.w;
    tgt = (uint32_t)(((unsigned long long)(w >> 8) * total) >> 24);
  }
  // draw k: the block holding it is the first whose running total exceeds the
  // target (totals only grow in page and lane order); lane k keeps the block
  // and the target's offset into it
  constexpr int kNone = 0x7fffffff;
  int zsel = kNone, dblk = 0;
  uint32_t doff = 0u;
  if (total > 0u) {
    for (int k = 0; k < n; ++k) {
      const uint32_t tk = (uint32_t)__builtin_amdgcn_readlane((int)tgt, k);
      bool done = false;
#pragma unroll
      for (int g = 0; g < kObsPages; ++g) {
        if (done || g >= npg) continue;
        const unsigned long long hit = __ballot(incl[g] > tk);
        if (hit == 0ull) continue;
        const int js = __ffsll((long long)hit) - 1;
        const uint32_t before =
            js > 0 ? (uint32_t)__builtin_amdgcn_readlane((int)incl[g], js - 1) : pbase[g];
        if (lane == k) {
          dblk = g * kWave + js;
          doff = tk - before;
        }
        done = true;
      }
    }
    // lane k < n: the first entry of its block whose running total within the
    // block exceeds the offset (an entry of positive integer mass)
    if (lane < n) {
      float v[16];
      uint32_t q[16];
      obs_block(dblk, L, otab, lmp, p0tab, lw, lvv, v);
      (void)block_masses(v, e, q);
      uint32_t run = 0u;
      int c = 16;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        run += q[i];
        if (c == 16 && run > doff) c = i;
      }
      if (c < 16) zsel = dblk * 16 + c;
    }
  }
  if (zsel == kNone) zsel = -1;   // no mass at all: no draw
  // lane k < n: P(z_k) of its draw
  float pk = 0.f;
  if (lane < n && zsel >= 0) {
    const int zw = zsel & 15, zl = zsel >> 4;
    if (zl == 0) {
      pk = p0tab[zw];
    } else {
      const uint32_t w = lw[zl - 1];
      pk = w > 15u ? 0.f : otab[(uint32_t)zw ^ (w & 15u)] * lmp * lvv[zl - 1];
    }
  }
  // one child per distinct z in ascending z order, with its frequency: lane k
  // compares its draw with every other one
  uint32_t eq = 0u, lt = 0u;
  for (int j = 0; j < n; ++j) {
    const int zj = __builtin_amdgcn_readlane(zsel, j);
    eq |= (uint32_t)(zj == zsel) << j;
    lt |= (uint32_t)(zj < zsel) << j;
  }
  const bool first = lane < n && (eq & ((1u << lane) - 1u)) == 0u;
  const bool ok = lane < n && zsel >= 0 && pk > 0.f;
  const uint32_t heads = (uint32_t)__ballot(first && ok);
  const int U = __popc(heads);
  if (first && ok) {
    const int r = __popc(lt & heads);
    lv.cvalid[cb + r] = 1;
    lv.cz[cb + r] = zsel;
    lv.ccount[cb + r] = __popc(eq);
    lv.cpz[cb + r] = pk;
    if (out) {
      out->z[r] = zsel;
      out->count[r] = __popc(eq);
      out->inv[r] = 1.0f / pk;
    }
  }
  if (lane >= U && lane < n) {
    lv.cvalid[cb + lane] = 0;
    lv.cz[cb + lane] = -1;
    lv.ccount[cb + lane] = 0;
    lv.cpz[cb + lane] = 0.f;
  }
  if (out && lane == 0) out->U = U;
  return U;
}

// The next level's visiting order: a Q-node's children cb .. cb+n-1, the U
// present ones (packed first) appended at the front of lv.slot_list, the
// absent ones at the back.  Two steps, so that a caller can issue the
// atomics early and write the entries once their positions have arrived:
// list_take on thread 0 (positions returned), list_put on wavefront 0.
struct ListPos {
  int live0, dead0;
};
__device__ __forceinline__ ListPos list_take(const LevelArgs &lv, int U) {
  ListPos lp = {0, 0};
  if (U > 0) lp.live0 = atomicAdd(&lv.slot_n[0], U);
  if (lv.n > U) lp.dead0 = atomicAdd(&lv.slot_n[1], lv.n - U);
  return lp;
}
__device__ __forceinline__ void list_put(const LevelArgs &lv, int cb, int U, ListPos lp) {
  const int lane = threadIdx.x & (kWave - 1);
  const int live0 = __shfl(lp.live0, 0, kWave), dead0 = __shfl(lp.dead0, 0, kWave);
  if (lane < U)
    lv.slot_list[live0 + lane] = cb + lane;
  else if (lane < lv.n)
    lv.slot_list[lv.slot_cap - 1 - (dead0 + lane - U)] = cb + lane;
}

// The n children of a Q-node whose parent is absent; all of wavefront 0.
__device__ __forceinline__ void list_absent_children(const LevelArgs &lv, int cb) {
  if (!lv.slot_list || threadIdx.x >= kWave) return;
  ListPos lp = {0, 0};
  if (threadIdx.x == 0) lp = list_take(lv, 0);
  list_put(lv, cb, 0, lp);
}

// Tiled path: the statistics of the Q-node are spread over per-band partials
// written by other workgroups of this launch; sum them in band order, stage
// the landmark terms in LDS (lds: 2*L words), then draw.
__device__ void sample_qnode(const DevModel &m, const LevelArgs &lv, int p, int a, float *lds) {
  const int lane = threadIdx.x & (kWave - 1);
  const int idx = p * m.A + a;
  // the 17 band sums: lane j adds bands j, j+64, ... (loads issued together),
  // then each value is reduced across the wavefront in a fixed order
  const float *pp = lv.part + (size_t)idx * lv.tiles * 17;
  float v[17];
#pragma unroll
  for (int k = 0; k < 17; ++k) v[k] = 0.f;
  for (int t = lane; t < lv.tiles; t += kWave) {
    float x[17];
#pragma unroll
    for (int k = 0; k < 17; ++k) x[k] = ld_coherent(pp + (size_t)t * 17 + k);
#pragma unroll
    for (int k = 0; k < 17; ++k) v[k] += x[k];
  }
  float hs = 0.f;
#pragma unroll
  for (int k = 0; k < 17; ++k) {
    const float tot = __int_as_float(
        __builtin_amdgcn_readlane(__float_as_int(wave_total_lane63(v[k])), 63));
    if (lane == k) hs = tot;
  }
  uint32_t *lw = (uint32_t *)lds;
  float *lvv = lds + m.L;
  for (int l = lane; l < m.L; l += kWave) {
    lw[l] = lv.lm_wall[l];
    lvv[l] = ld_coherent(lv.lmv + (size_t)idx * m.L + l);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  const int U = sample_draws(m, lv, p, a, hs, lw, lvv, lds + 2 * m.L, nullptr);
  // (after the draws: the wait before them need not cover this store)
  if (lane == 16) lv.reward[idx] = hs;
  if (lv.slot_list) {
    ListPos lp = {0, 0};
    if (lane == 0) lp = list_take(lv, U);
    list_put(lv, p * lv.K + a * lv.n, U, lp);
  }
}

// Workgroups go to the 8 XCDs in turn (workgroup id mod 8), each XCD with
// its own L2.  This renumbering gives every XCD a contiguous range of
// logical ids, so neighbouring items -- the actions of one parent, which
// read the same parent belief -- meet in one L2.  A bijection on [0, n).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_local_id(int i, int n) {
  const int q = n / kXcds, r = n - q * kXcds, x = i % kXcds;
  return x * q + min(x, r) + i / kXcds;
}

// Work item idx = (p * tiles + tile) * A + a of a level.
struct Item {
  int p, tile, a;
};
__device__ __forceinline__ Item decode_item(int idx, int tiles, int A) {
  Item it;
  const int pt = idx / A;
  it.a = idx - pt * A;
  it.p = pt / tiles;
  it.tile = pt - it.p * tiles;
  return it;
}

// As decode_item, with the parents taken in the level's visiting order.
__device__ __forceinline__ Item decode_item(int idx, const LevelArgs &lv, int A) {
  Item it = decode_item(idx, lv.tiles, A);
  if (lv.porder) it.p = lv.porder[it.p];
  return it;
}

// Static LDS of the banded item functions.
struct BandShared {
  float stay[256];            // stay probability of action a by neighbour pattern
  float red[kBlock / kWave];
  int last;
};

// The slip row of action a and the flip probabilities, copied to registers.
struct ActTables {
  float sl[9];
  float fl[4];
};
__device__ __forceinline__ ActTables act_tables(const DevModel &m, int a) {
  ActTables t;
#pragma unroll
  for (int k = 0; k < 9; ++k) t.sl[k] = m.slip[a * 9 + k];
#pragma unroll
  for (int j = 0; j < 4; ++j) t.fl[j] = m.flip[j];
  return t;
}

// ---------------------------------------------------------------------------
// k_stats: per (parent slot, band, action)
// ---------------------------------------------------------------------------
__device__ void stats_item(const DevModel &m, const LevelArgs &lv, Item it, float *smem,
                           BandShared &sh) {
  float *s_stay = sh.stay;
  float *red = sh.red;
  int &s_last = sh.last;
  const int p = it.p, tile = it.tile, a = it.a;
  // children of an invalid parent are marked absent by its first band
  if (!lv.pvalid[p]) {
    if (tile == 0 && threadIdx.x < lv.n) {
      const int c = p * lv.K + a * lv.n + threadIdx.x;
      lv.cvalid[c] = 0;
      lv.cz[c] = -1;
      lv.ccount[c] = 0;
      lv.cpz[c] = 0.f;
    }
    if (tile == 0) list_absent_children(lv, p * lv.K + a * lv.n);
    return;
  }
  const int W = m.W, BW = W + 2, A = m.A;
  const int y0 = tile * lv.TH;
  const int th = min(lv.TH, m.H - y0);
  float *band = smem;
  float *hist = band + (lv.TH + 2) * BW;   // [16][kBlock] per-thread bins
  const float *b = lv.pbel + (size_t)p * m.S;
  s_stay[threadIdx.x] = lv.staytab[a * 256 + threadIdx.x];
  load_band(m, lv.sig, b, y0, th, band, BW, lv.d == 0);
  const int tid = threadIdx.x;
#pragma unroll
  for (int w = 1; w < 16; ++w) hist[w * kBlock + tid] = 0.f;
  __syncthreads();
  const int ncell = th * W;
  const float rW = 1.0f / (float)W;
  const ActTables at = act_tables(m, a);
  const float *sl = at.sl;
  const float *stay_a = s_stay;
  const float rho = m.lm_p;
  const int L = m.L;
  const float *Rt = m.R;
  float h0 = 0.f, racc = 0.f;
  const int t00 = y0 * W;
  for (int i0 = tid; i0 < ncell; i0 += kCellBatch * kBlock) {
    uint32_t sg[kCellBatch];
    float bt[kCellBatch], rr[kCellBatch];
#pragma unroll
    for (int j = 0; j < kCellBatch; ++j) {
      const int i = i0 + j * kBlock;
      const bool ok = i < ncell;
      const int t = t00 + (ok ? i : 0);
      const uint32_t sv = lv.sig[t];   // loaded by every lane, then masked
      const float bv = b[t], rv = Rt[(size_t)t * A + a];
      sg[j] = ok ? sv : 0u;
      bt[j] = ok ? bv : 0.f;
      rr[j] = ok ? rv : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kCellBatch; ++j) {
      const int i = i0 + j * kBlock;
      if (i >= ncell) break;
      // R(b,a) = sum_x R(x,a) b(x) (Sec. III)
      racc = fmaf(bt[j], rr[j], racc);
      const int ly = fdiv(i, W, rW), lx = i - ly * W;
      const float bp = predict_cell_v(band, BW, ly, lx, sg[j], sl, stay_a, bt[j]);
      const uint32_t lm = sig_lm(sg[j]);
      float contrib = bp;
      if (lm && lm <= (uint32_t)L) {
        contrib = bp * (1.f - rho);
        st_coherent(lv.lmv + ((size_t)p * A + a) * L + lm - 1, bp);
      }
      const uint32_t w = sig_wall(sg[j]);
      if (w == 0u)
        h0 += contrib;
      else
        hist[w * kBlock + tid] += contrib;
    }
  }
  hist[tid] = h0;
  racc = wave_sum(racc);
  if ((tid & (kWave - 1)) == 0) red[tid / kWave] = racc;
  __syncthreads();
  float *part = lv.part + (((size_t)p * A + a) * lv.tiles + tile) * 17;
  // bin = tid/16: lane k of the bin's 16 adds entries k, k + 16, ... (the 16
  // lanes read consecutive words; the four bins of a wavefront start their
  // walks one step apart, so no two lanes share an LDS bank), then the 16
  // lanes combine
  {
    const int k = tid & 15, rot = (tid >> 4) & 3;
    const float *hb = hist + (tid >> 4) * kBlock;
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += hb[k + 16 * ((i + rot) & 15)];
    s = group_sum<16>(s);
    if ((tid & 15) == 15) st_coherent(part + (tid >> 4), s);
    if (tid == 0) st_coherent(part + 16, (red[0] + red[1]) + (red[2] + red[3]));
  }
  // the last band of this Q-node to finish draws its observations
  wait_mem();
  __syncthreads();
  if (tid == 0) {
    const int prev = count_arrival(&lv.ctr[p * A + a]);
    s_last = (prev == lv.tiles - 1);
  }
  __syncthreads();
  if (!s_last) return;
  if (tid < kWave) sample_qnode(m, lv, p, a, hist);
  if (tid == 0) lv.ctr[p * A + a] = 0;
}

__global__ __launch_bounds__(kBlock) void k_stats(DevModel m, LevelArgs lv) {
  extern __shared__ float smem[];
  __shared__ BandShared sh;
  stats_item(m, lv, decode_item(xcd_local_id(blockIdx.x, gridDim.x), lv, m.A), smem, sh);
}

// ---------------------------------------------------------------------------
// k_update: per (parent slot, band, action); writes Phi(b,a,z) per child
// ---------------------------------------------------------------------------
__device__ void update_item(const DevModel &m, const LevelArgs &lv, Item it, float *smem,
                            BandShared &sh) {
  float *s_stay = sh.stay;
  const int p = it.p, tile = it.tile, a = it.a;
  if (!lv.pvalid[p]) return;
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
  if (U == 0) return;
  const int W = m.W, BW = W + 2, S = m.S;
  const int y0 = tile * lv.TH;
  const int th = min(lv.TH, m.H - y0);
  float *band = smem;
  const float *b = lv.pbel + (size_t)p * S;
  s_stay[threadIdx.x] = lv.staytab[a * 256 + threadIdx.x];
  load_band(m, lv.sig, b, y0, th, band, BW, lv.d == 0);
  __syncthreads();
  const int ncell = th * W;
  const float rW = 1.0f / (float)W;
  const ActTables at = act_tables(m, a);
  const float *sl = at.sl;
  const float rho = m.lm_p;
  const float *stay_a = s_stay;
  const int t00 = y0 * W;
  for (int i0 = threadIdx.x; i0 < ncell; i0 += kCellBatch * kBlock) {
    uint32_t sg[kCellBatch];
    float bt[kCellBatch];
#pragma unroll
    for (int j = 0; j < kCellBatch; ++j) {
      const int i = i0 + j * kBlock;
      const bool ok = i < ncell;
      const int t = t00 + (ok ? i : 0);
      const uint32_t sv = lv.sig[t];   // loaded by every lane, then masked
      const float bv = b[t];
      sg[j] = ok ? sv : 0u;
      bt[j] = ok ? bv : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kCellBatch; ++j) {
      const int i = i0 + j * kBlock;
      if (i >= ncell) break;
      const int ly = fdiv(i, W, rW), lx = i - ly * W;
      const int t = t00 + i;
      const float bp = predict_cell_v(band, BW, ly, lx, sg[j], sl, stay_a, bt[j]);
      const uint32_t w = sig_wall(sg[j]), lm = sig_lm(sg[j]);
#pragma unroll
      for (int r = 0; r < QV_MAX_SAMPLES; ++r) {
        if (r < U) {
          const float o = wall_lik(at.fl, (uint32_t)(zr[r] & 15), w) *
                          lm_lik(rho, (uint32_t)(zr[r] >> 4), lm);
          lv.cbel[(size_t)(cb + r) * S + t] = o * bp * inv[r];
        }
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_update(DevModel m, LevelArgs lv) {
  extern __shared__ float smem[];
  __shared__ BandShared sh;
  update_item(m, lv, decode_item(xcd_local_id(blockIdx.x, gridDim.x), lv, m.A), smem, sh);
}

// ---------------------------------------------------------------------------
// Banded inner levels with every action of a parent in one item: a
// workgroup per (parent slot, band) loads the parent's band once and serves
// all |A| Q-nodes from it, instead of one item per (parent, band, action)
// that each load the band.  The per-action arithmetic is that of stats_item
// and update_item, in the same order, so results are bitwise the same.
// ---------------------------------------------------------------------------
constexpr int kParentCells = 8;   // cells per thread of a band: at most 2048 / kBlock

struct ParentShared {
  float stay[QV_MAX_ACTIONS * 256];   // stay probability by neighbour pattern, per action
  float red[QV_MAX_ACTIONS][kBlock / kWave];
  int zr[QV_MAX_ACTIONS * QV_MAX_SAMPLES];
  float inv[QV_MAX_ACTIONS * QV_MAX_SAMPLES];
  int U[QV_MAX_ACTIONS];
  int last;
};

// Dynamic LDS floats of k_stats_parent: the band and the per-thread bins,
// or the four wavefronts' sampler tables.
__host__ __device__ inline size_t stats_parent_lds_floats(int W, int TH, int L) {
  const size_t a = (size_t)(TH + 2) * (W + 2) + 16 * kBlock;
  const size_t b = (size_t)(kBlock / kWave) * (2 * (size_t)L + 32);
  return a > b ? a : b;
}

__device__ void stats_parent_item(const DevModel &m, const LevelArgs &lv, int p, int tile,
                                  float *smem, ParentShared &sh) {
  const int A = m.A, tid = threadIdx.x;
  if (!lv.pvalid[p]) {
    // children of an absent parent are marked absent by its first band
    if (tile == 0) {
      for (int i = tid; i < lv.K; i += kBlock) {
        const int c = p * lv.K + i;
        lv.cvalid[c] = 0;
        lv.cz[c] = -1;
        lv.ccount[c] = 0;
        lv.cpz[c] = 0.f;
      }
      for (int a = 0; a < A; ++a) list_absent_children(lv, p * lv.K + a * lv.n);
    }
    return;
  }
  const int W = m.W, BW = W + 2;
  const int y0 = tile * lv.TH;
  const int th = min(lv.TH, m.H - y0);
  float *band = smem;
  float *hist = band + (lv.TH + 2) * BW;   // [16][kBlock] per-thread bins
  const float *b = lv.pbel + (size_t)p * m.S;
  for (int i = tid; i < A * 256; i += kBlock) sh.stay[i] = lv.staytab[i];
  load_band(m, lv.sig, b, y0, th, band, BW, lv.d == 0);
  const int ncell = th * W;
  const float rW = 1.0f / (float)W;
  const int t00 = y0 * W;
  // the thread's cells (the same ones, in the same order, as stats_item's)
  // with their rows of R: all loads go out before any is used
  const int jn = (ncell + kBlock - 1) / kBlock;   // uniform
  uint32_t sg[kParentCells];
  float bt[kParentCells];
  float racc[QV_MAX_ACTIONS];
#pragma unroll
  for (int a = 0; a < QV_MAX_ACTIONS; ++a) racc[a] = 0.f;
#pragma unroll
  for (int j = 0; j < kParentCells; ++j) {
    if (j >= jn) break;
    const int i = tid + j * kBlock;
    const bool ok = i < ncell;
    const int t = t00 + (ok ? i : 0);
    const uint32_t sv = lv.sig[t];
    const float bv = b[t];
    sg[j] = ok ? sv : 0u;
    bt[j] = ok ? bv : 0.f;
  }
  // R(b,a) = sum_x R(x,a) b(x) for every action (Sec. III), cells in order
#pragma unroll
  for (int j = 0; j < kParentCells; ++j) {
    if (j >= jn) break;
    const int i = tid + j * kBlock;
    const float *row = m.R + (size_t)(t00 + (i < ncell ? i : 0)) * A;
    float rv[QV_MAX_ACTIONS];
#pragma unroll
    for (int a = 0; a < QV_MAX_ACTIONS; ++a) rv[a] = row[a < A ? a : 0];
    if (i < ncell) {
#pragma unroll
      for (int a = 0; a < QV_MAX_ACTIONS; ++a)
        if (a < A) racc[a] = fmaf(bt[j], rv[a], racc[a]);
    }
  }
#pragma unroll
  for (int a = 0; a < QV_MAX_ACTIONS; ++a) {
    if (a >= A) break;
    const float r = wave_sum(racc[a]);
    if ((tid & (kWave - 1)) == 0) sh.red[a][tid / kWave] = r;
  }
  __syncthreads();
  const float rho = m.lm_p;
  const int L = m.L;
  for (int a = 0; a < A; ++a) {
    const float *sl = &m.slip[a * 9];
    const float *stay_a = sh.stay + a * 256;
#pragma unroll
    for (int w = 1; w < 16; ++w) hist[w * kBlock + tid] = 0.f;
    float h0 = 0.f;
#pragma unroll
    for (int j = 0; j < kParentCells; ++j) {
      const int i = tid + j * kBlock;
      if (j >= jn || i >= ncell) break;
      const int ly = fdiv(i, W, rW), lx = i - ly * W;
      const float bp = predict_cell_v(band, BW, ly, lx, sg[j], sl, stay_a, bt[j]);
      const uint32_t lm = sig_lm(sg[j]);
      float contrib = bp;
      if (lm && lm <= (uint32_t)L) {
        contrib = bp * (1.f - rho);
        st_coherent(lv.lmv + ((size_t)p * A + a) * L + lm - 1, bp);
      }
      const uint32_t w = sig_wall(sg[j]);
      if (w == 0u)
        h0 += contrib;
      else
        hist[w * kBlock + tid] += contrib;
    }
    hist[tid] = h0;
    __syncthreads();
    float *part = lv.part + (((size_t)p * A + a) * lv.tiles + tile) * 17;
    {
      const int k = tid & 15, rot = (tid >> 4) & 3;
      const float *hb = hist + (tid >> 4) * kBlock;
      float sum = 0.f;
#pragma unroll
      for (int i = 0; i < 16; ++i) sum += hb[k + 16 * ((i + rot) & 15)];
      sum = group_sum<16>(sum);
      if ((tid & 15) == 15) st_coherent(part + (tid >> 4), sum);
      if (tid == 0)
        st_coherent(part + 16, (sh.red[a][0] + sh.red[a][1]) + (sh.red[a][2] + sh.red[a][3]));
    }
    __syncthreads();   // the bins are reused by the next action
  }
  // k_stats_draws draws for every action after the launch; else the last
  // band of this parent to finish does
  if (lv.draws_apart) return;
  wait_mem();
  __syncthreads();
  if (tid == 0) sh.last = (count_arrival(&lv.ctr[p * A]) == lv.tiles - 1);
  __syncthreads();
  if (!sh.last) return;
  const int wave = tid / kWave;
  float *scratch = smem + (size_t)wave * (2 * L + 32);
  for (int a = wave; a < A; a += kBlock / kWave) sample_qnode(m, lv, p, a, scratch);
  if (tid == 0) lv.ctr[p * A] = 0;
}

// Workgroup i takes band i mod tiles of parent i / tiles: consecutive bands of
// a parent go to different XCDs (workgroups are dealt to the XCDs in turn),
// so every XCD gets an equal share of every present parent's bands (a band
// is read by one workgroup only, for all actions; the same bands recur on an
// XCD, whose L2 then holds their rows of R).  SORT: lv.sort_bands extra
// workgroups ahead of the items sort the last level's bands (as
// k_prep_sort); the level-0 launch, one item per CU, has room for them.
template <bool SORT>
__global__ __launch_bounds__(kBlock) void k_stats_parent(DevModel m, LevelArgs lv) {
  extern __shared__ float smem[];
  __shared__ ParentShared sh;
  int i = blockIdx.x;
  if constexpr (SORT) {
    if (i < lv.sort_bands) {   // the launch's dynamic LDS holds the sort's tables
      const int c_lo = i * lv.sort_tc;
      sort_band<kBlock, true>(c_lo, min(m.S, c_lo + lv.sort_tc), m.L, lv.sig,
                              (int32_t *)lv.sort_cells,
                              (int32_t *)lv.sort_chunk + (size_t)i * kSortChunkInts, smem);
      return;
    }
    i -= lv.sort_bands;
  }
  const int p = i / lv.tiles;
  stats_parent_item(m, lv, p, i - p * lv.tiles, smem, sh);
}

// The draws of the Q-nodes of a banded level once every band has written its
// partial sums: one wavefront per (parent, action).  Run apart from the band
// items, the draws neither wait for the last band of each parent nor pile up
// on the XCD whose bands arrive last.  Absent parents were handled by their
// first band.  LDS: 2 L + 32 floats.
__global__ __launch_bounds__(kWave) void k_stats_draws(DevModel m, LevelArgs lv) {
  extern __shared__ float smem[];
  const int p = blockIdx.x / m.A, a = blockIdx.x - p * m.A;
  if (!lv.pvalid[p]) return;
  sample_qnode(m, lv, p, a, smem);
}

__device__ void update_parent_item(const DevModel &m, const LevelArgs &lv, int p, int tile,
                                   int a_lo, int a_hi, float *smem, ParentShared &sh) {
  if (!lv.pvalid[p]) return;
  const int A = m.A, n = lv.n, K = lv.K, tid = threadIdx.x;
  // the drawn children of every action (valid ones are packed first)
  for (int i = tid; i < K; i += kBlock) {
    const int c = p * K + i;
    const int v = lv.cvalid[c];
    sh.zr[i] = v ? lv.cz[c] : 0;
    sh.inv[i] = v ? 1.0f / lv.cpz[c] : 0.f;
  }
  if (tid < A) {
    int U = 0;
    for (int r = 0; r < n; ++r) U += lv.cvalid[p * K + tid * n + r] ? 1 : 0;
    sh.U[tid] = U;
  }
  for (int i = tid; i < A * 256; i += kBlock) sh.stay[i] = lv.staytab[i];
  const int W = m.W, BW = W + 2, S = m.S;
  const int y0 = tile * lv.TH;
  const int th = min(lv.TH, m.H - y0);
  float *band = smem;
  const float *b = lv.pbel + (size_t)p * S;
  load_band(m, lv.sig, b, y0, th, band, BW, lv.d == 0);
  __syncthreads();
  const int ncell = th * W;
  const float rW = 1.0f / (float)W;
  const float rho = m.lm_p;
  const int t00 = y0 * W;
  for (int i0 = tid; i0 < ncell; i0 += kCellBatch * kBlock) {
    uint32_t sg[kCellBatch];
    float bt[kCellBatch];
#pragma unroll
    for (int j = 0; j < kCellBatch; ++j) {
      const int i = i0 + j * kBlock;
      const bool ok = i < ncell;
      const int t = t00 + (ok ? i : 0);
      const uint32_t sv = lv.sig[t];
      const float bv = b[t];
      sg[j] = ok ? sv : 0u;
      bt[j] = ok ? bv : 0.f;
    }
    for (int a = a_lo; a < a_hi; ++a) {
      const int U = sh.U[a];
      if (U == 0) continue;
      const float *sl = &m.slip[a * 9];
      const float *stay_a = sh.stay + a * 256;
      const int cb = p * K + a * n;
      float bp[kCellBatch];
#pragma unroll
      for (int j = 0; j < kCellBatch; ++j) {
        const int i = i0 + j * kBlock;
        const int ly = fdiv(i, W, rW), lx = i - ly * W;
        bp[j] = i < ncell ? predict_cell_v(band, BW, ly, lx, sg[j], sl, stay_a, bt[j]) : 0.f;
      }
      // child by child, so each child's rows of the band go out together
      for (int r = 0; r < U; ++r) {
        const int zz = sh.zr[a * n + r];
        const float inv = sh.inv[a * n + r];
        float *out = lv.cbel + (size_t)(cb + r) * S + t00;
#pragma unroll
        for (int j = 0; j < kCellBatch; ++j) {
          const int i = i0 + j * kBlock;
          if (i >= ncell) break;
          const float o = wall_lik(m.flip, (uint32_t)(zz & 15), sig_wall(sg[j])) *
                          lm_lik(rho, (uint32_t)(zz >> 4), sig_lm(sg[j]));
          __builtin_nontemporal_store(o * bp[j] * inv, out + i);   // streamed: read back much later
        }
      }
    }
  }
}

// Workgroup i takes band i mod tiles of parent i / (tiles G), actions of
// group (i / tiles) mod G (see k_stats_parent for the band order).
__global__ __launch_bounds__(kBlock) void k_update_parent(DevModel m, LevelArgs lv) {
  extern __shared__ float smem[];
  __shared__ ParentShared sh;
  const int i = blockIdx.x;
  // item i: parent i / (tiles G), action group (i / tiles) mod G, band i mod
  // tiles (G = lv.agroups: a level with few items splits each band's
  // actions over G workgroups)
  const int G = lv.agroups > 1 ? lv.agroups : 1;
  const int per = lv.tiles * G;
  const int p = i / per, rem = i - p * per;
  const int g = rem / lv.tiles, tile = rem - g * lv.tiles;
  const int apg = (m.A + G - 1) / G;
  update_parent_item(m, lv, p, tile, g * apg, min(m.A, (g + 1) * apg), smem, sh);
}

// ---------------------------------------------------------------------------
// expectimax backup of one node, by one thread (Alg. 6/7)
// ---------------------------------------------------------------------------

// V(v) = max_a Q(v,a) from the node's Q-values q[0..A); at the root also the
// action (lowest a within 1e-9 of the best) and the root Q-values.  One thread.
__device__ void finish_node(const TreeArgs &t, int d, long long g, const float *q) {
  float best = -INFINITY;
  for (int a = 0; a < t.A; ++a) best = fmaxf(best, q[a]);
  st_coherent(t.value + g, best);
  if (d == 0) {
    int act = 0;
    for (int a = 0; a < t.A; ++a)
      if (q[a] >= best - 1e-9f) {
        act = a;
        break;
      }
    t.action_out[0] = act;
    for (int a = 0; a < t.A; ++a) t.rootQ_out[a] = q[a];
  }
}

// Backup of node (d, slot) by the whole workgroup (Alg. 6/7):
//   Q(v,a) = R(b_v,a) + gamma * sum_children (f/n) V(child),  V(v) = max_a Q(v,a);
// at the root also the action (lowest a within 1e-9 of the best).  sh holds
// the node's K child values (entries of absent children unused) and has room
// for A more.  Ends with a barrier.
__device__ void backup_node_wg(const TreeArgs &t, int d, long long slot, float *sh) {
  const long long g = t.first[d] + slot;
  if (threadIdx.x < t.A) {
    const int a = threadIdx.x;
    float q = t.reward[g * t.A + a];
    const long long cb = t.first[d + 1] + slot * t.K + (long long)a * t.n;
    for (int r = 0; r < t.n; ++r) {
      if (!t.valid[cb + r]) break;
      q += t.gamma * ((float)t.count[cb + r] / (float)t.n) * sh[a * t.n + r];
    }
    t.qvalue[g * t.A + a] = q;
    sh[t.K + a] = q;
  }
  __syncthreads();
  if (threadIdx.x == 0) finish_node(t, d, g, sh + t.K);
  __syncthreads();
}

// Node (d, slot) is complete: report to the parent; the workgroup holding
// the last child of a parent completes the parent, and so on to the root.
__device__ void climb_wg(const TreeArgs &t, int d, long long slot, float *sh, int *s_go) {
  while (d > 0) {
    const long long ps = slot / t.K;
    const long long c0 = t.first[d] + ps * t.K;
    wait_mem();
    __syncthreads();
    if (threadIdx.x == 0) {
      int expect = 0;
      for (int c = 0; c < t.K; ++c) expect += t.valid[c0 + c] ? 1 : 0;
      const int prev = count_arrival(&t.node_ctr[t.first[d - 1] + ps]);
      *s_go = (prev == expect - 1);
    }
    __syncthreads();
    if (!*s_go) return;
    for (int c = threadIdx.x; c < t.K; c += kBlock)
      sh[c] = t.valid[c0 + c] ? ld_coherent(t.value + c0 + c) : 0.f;
    __syncthreads();
    --d;
    slot = ps;
    backup_node_wg(t, d, slot, sh);
  }
}

// ---------------------------------------------------------------------------
// k_leaf: per (parent slot, band, action) at the last level; each child
// belief value is formed as in k_update and dotted with Q(.,a') at once
// ---------------------------------------------------------------------------
template <int APAD>
__device__ void leaf_item(const DevModel &m, const LevelArgs &lv, const TreeArgs &tr, Item it,
                          float *smem, BandShared &sh) {
  constexpr int G = 32 / APAD;            // children per accumulation group
  float *s_stay = sh.stay;
  int &s_last = sh.last;
  const int p = it.p, tile = it.tile, a = it.a;
  if (!lv.pvalid[p]) return;
  const int W = m.W, BW = W + 2, A = m.A, S = m.S;
  const int cb = p * lv.K + a * lv.n;
  float *red = smem + (lv.TH + 2) * BW;   // transpose / backup scratch
  int U = 0;
  for (int r = 0; r < lv.n; ++r) U += lv.cvalid[cb + r] ? 1 : 0;
  if (U > 0) {
    const int y0 = tile * lv.TH;
    const int th = min(lv.TH, m.H - y0);
    float *band = smem;
    const float *b = lv.pbel + (size_t)p * S;
    s_stay[threadIdx.x] = lv.staytab[a * 256 + threadIdx.x];
  load_band(m, lv.sig, b, y0, th, band, BW, lv.d == 0);
    __syncthreads();
    const int ncell = th * W;
    const float rW = 1.0f / (float)W;
    const ActTables at = act_tables(m, a);
    const float *sl = at.sl;
    const float rho = m.lm_p;
    const float *stay_a = s_stay;
    for (int r0 = 0; r0 < U; r0 += G) {
      int zr[G];
      float inv[G];
#pragma unroll
      for (int r = 0; r < G; ++r) {
        zr[r] = 0;
        inv[r] = 0.f;
        if (r0 + r < U) {
          zr[r] = lv.cz[cb + r0 + r];
          inv[r] = 1.0f / lv.cpz[cb + r0 + r];
        }
      }
      float acc[32];
#pragma unroll
      for (int i = 0; i < 32; ++i) acc[i] = 0.f;
      const int t00 = y0 * W;
      for (int i0 = threadIdx.x; i0 < ncell; i0 += kLeafBatch * kBlock) {
        uint32_t sg[kLeafBatch];
        float bt[kLeafBatch];
        float q[kLeafBatch][APAD];
#pragma unroll
        for (int j = 0; j < kLeafBatch; ++j) {
          const int i = i0 + j * kBlock;
          const bool ok = i < ncell;
          const int t = t00 + (ok ? i : 0);
          const uint32_t sv = lv.sig[t];   // loaded by every lane, then masked
          const float bv = b[t];
          sg[j] = ok ? sv : 0u;
          bt[j] = ok ? bv : 0.f;
          load_q_row<APAD>(lv, A, t, q[j]);
        }
#pragma unroll
        for (int j = 0; j < kLeafBatch; ++j) {
          const int i = i0 + j * kBlock;
          if (i >= ncell) break;
          const int ly = fdiv(i, W, rW), lx = i - ly * W;
          const float bp = predict_cell_v(band, BW, ly, lx, sg[j], sl, stay_a, bt[j]);
          const uint32_t w = sig_wall(sg[j]), lm = sig_lm(sg[j]);
#pragma unroll
          for (int r = 0; r < G; ++r) {
            if (r0 + r < U) {
              const float o = wall_lik(at.fl, (uint32_t)(zr[r] & 15), w) *
                              lm_lik(rho, (uint32_t)(zr[r] >> 4), lm);
              const float v = o * bp * inv[r];
#pragma unroll
              for (int c = 0; c < APAD; ++c)
                acc[r * APAD + c] = fmaf(v, q[j][c], acc[r * APAD + c]);
            }
          }
        }
      }
      const float tot = block_sum32(acc, red);
      const int r = threadIdx.x / APAD, c = threadIdx.x - r * APAD;
      if (threadIdx.x < 32 && r0 + r < U && c < A)
        st_coherent(lv.leafpart + ((size_t)(cb + r0 + r) * lv.tiles + tile) * A + c, tot);
    }
  }
  // every (band, action) of the node reports; the last one scores the node's
  // children and completes the node's backup
  wait_mem();
  __syncthreads();
  const long long g = tr.first[lv.d] + p;
  if (threadIdx.x == 0) {
    const int prev = count_arrival(&tr.node_ctr[g]);
    s_last = (prev == A * lv.tiles - 1);
  }
  __syncthreads();
  if (!s_last) return;
  // leaf values V(c) = max_a' sum over bands, K*A sums spread over the threads
  const int K = lv.K;
  const long long lf = tr.first[lv.d + 1] + (long long)p * K;
  float *sums = red + K + A;
  for (int i = threadIdx.x; i < K * A; i += kBlock) {
    const int c = i / A, ap = i - c * A;
    float s = 0.f;
    if (tr.valid[lf + c])
      for (int t = 0; t < lv.tiles; ++t)
        s += ld_coherent(lv.leafpart + ((size_t)(p * K + c) * lv.tiles + t) * A + ap);
    sums[i] = s;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < K; c += kBlock) {
    float best = 0.f;
    if (tr.valid[lf + c]) {
      best = -INFINITY;
      for (int ap = 0; ap < A; ++ap) best = fmaxf(best, sums[c * A + ap]);
      st_coherent(tr.value + lf + c, best);
    }
    red[c] = best;
  }
  __syncthreads();
  backup_node_wg(tr, lv.d, p, red);
  climb_wg(tr, lv.d, p, red, &s_last);
}

template <int APAD>
__global__ __launch_bounds__(kBlock) void k_leaf(DevModel m, LevelArgs lv, TreeArgs tr) {
  extern __shared__ float smem[];
  __shared__ BandShared sh;
  leaf_item<APAD>(m, lv, tr, decode_item(xcd_local_id(blockIdx.x, gridDim.x), lv, m.A), smem, sh);
}

// ---------------------------------------------------------------------------
// k_node: grids whose belief fits in LDS -- one workgroup per Q-node (parent
// slot, action).  The parent belief and its prediction b' stay in LDS; the
// workgroup forms the statistics, draws the observations, and then either
// writes the child beliefs (LEAF = false) or scores the leaf children and
// forms the Q-node value (LEAF = true; the last Q-node of a node completes
// the node and climbs towards the root).
// ---------------------------------------------------------------------------
// SORT: the launch carries lv.sort_bands extra workgroups, placed after the
// Q-node workgroups, that sort the leaf bands (as k_prep_sort) while the
// first level runs.
template <int APAD, bool LEAF, bool SORT = false>
__global__ __launch_bounds__(LEAF ? kBlock : kNodeBlock) void k_node(DevModel m, LevelArgs lv,
                                                                     TreeArgs tr) {
  // threads: kNodeBlock at inner levels; the leaf variant keeps kBlock (one
  // thread per sorted chunk)
  constexpr int NB = LEAF ? kBlock : kNodeBlock;
  constexpr int NBATCH = kNodeBatch * kBlock / NB;   // cells per thread and pass
  extern __shared__ float smem[];
  __shared__ float s_stay[256];
  __shared__ float s_red[NB / kWave * 32];
  __shared__ float s_H[17];
  __shared__ DrawOut s_draw;
  __shared__ float s_tab[QV_MAX_SAMPLES * 16];     // O_w(zw_r | w) / P(z_r)
  __shared__ float s_leaf[(QV_MAX_SAMPLES + 8) * 16];
  __shared__ float s_HQ[LEAF ? 16 * (APAD + 1) : 1];
  __shared__ int s_last;
  const int A = m.A, W = m.W, H = m.H, S = m.S, BW = W + 2;
  int nodes = gridDim.x;
  if constexpr (SORT) {
    nodes -= lv.sort_bands;
    if ((int)blockIdx.x >= nodes) {
      const int band = blockIdx.x - nodes, c_lo = band * lv.sort_tc;
      sort_band<NB>(c_lo, min(S, c_lo + lv.sort_tc), m.L, lv.sig, (int32_t *)lv.sort_cells,
                (int32_t *)lv.sort_chunk + (size_t)band * kSortChunkInts);
      return;
    }
  }
  const int bid = xcd_local_id(blockIdx.x, nodes);
  const int pj = bid / A, a = bid - pj * A;
  const int p = lv.porder ? lv.porder[pj] : pj;   // present parents first
  const int cb = p * lv.K + a * lv.n;
  const int tid = threadIdx.x;
  if (!lv.pvalid[p]) {
    if (tid < lv.n) {
      lv.cvalid[cb + tid] = 0;
      lv.cz[cb + tid] = -1;
      lv.ccount[cb + tid] = 0;
      lv.cpz[cb + tid] = 0.f;
    }
    list_absent_children(lv, cb);
    return;
  }
  float *bpl = smem;                      // [S] predicted belief b'
  float *X = smem + ((S + 3) & ~3);       // band, then scratch
  float *band = X;
  float *hist = X + small_x_floats(W, H, A, lv.n, m.L);   // [16][NB] bins (LEAF = false)
  const float *b = lv.pbel + (size_t)p * S;
  const float rW = 1.0f / (float)W;
  // per-cell inputs of a batch: signature and R(t,a) (b(t) comes from the
  // band); the first batch goes out before the band load.  Lanes past S load
  // cell 0 and are masked.
  uint32_t sg[NBATCH];
  float rr[NBATCH];
#pragma unroll
  for (int j = 0; j < NBATCH; ++j) {
    const int t = tid + j * NB;
    const int tc = t < S ? t : 0;
    const uint32_t sv = lv.sig[tc];
    const float rv = m.R[(size_t)tc * A + a];
    sg[j] = t < S ? sv : 0u;
    rr[j] = t < S ? rv : 0.f;
  }
  // the goal keeps its own mass (the band holds zero there)
  const float bgoal = m.goal >= 0 ? b[m.goal] : 0.f;
  if (tid < 256) s_stay[tid] = lv.staytab[a * 256 + tid];
  load_band<24 * kBlock / NB, NB>(m, lv.sig, b, 0, H, band, BW, lv.d == 0);
  if (!LEAF) {
#pragma unroll
    for (int w = 1; w < 16; ++w) hist[w * NB + tid] = 0.f;
  }
  __syncthreads();
  const float *sl = &m.slip[a * 9];
  const float rho = m.lm_p;
  // b'(x) for every cell (slip stencil), R(b,a) = sum_x R(x,a) b(x) and the
  // histogram of b' by true wall reading (per-thread bins; landmark cells
  // weighted by their "no landmark" factor)
  const bool one_pass = S <= NBATCH * NB;
  float racc = 0.f, h0 = 0.f;
  for (int t0 = tid; t0 < S; t0 += NBATCH * NB) {
    if (t0 != tid) {
#pragma unroll
      for (int j = 0; j < NBATCH; ++j) {
        const int t = t0 + j * NB;
        const int tc = t < S ? t : 0;
        const uint32_t sv = lv.sig[tc];
        const float rv = m.R[(size_t)tc * A + a];
        sg[j] = t < S ? sv : 0u;
        rr[j] = t < S ? rv : 0.f;
      }
    }
#pragma unroll
    for (int j = 0; j < NBATCH; ++j) {
      const int t = t0 + j * NB;
      if (t < S) {
        const int ly = fdiv(t, W, rW), lx = t - ly * W;
        // b(t): the band holds the belief (blocked cells hold no mass in any
        // belief the planner accepts or forms), except at the goal
        const float bt = t == m.goal ? bgoal : band[(ly + 1) * BW + lx + 1];
        racc = fmaf(bt, rr[j], racc);
        const float bp = predict_cell_v(band, BW, ly, lx, sg[j], sl, s_stay, bt);
        bpl[t] = bp;
        if (!LEAF) {
          const uint32_t lm = sig_lm(sg[j]);
          const float contrib = (lm && lm <= (uint32_t)m.L) ? bp * (1.f - rho) : bp;
          const uint32_t w = sig_wall(sg[j]);
          if (w == 0u)
            h0 += contrib;
          else
            hist[w * NB + tid] += contrib;
        }
      }
    }
  }
  if (!LEAF) hist[tid] = h0;
  racc = wave_sum(racc);
  if ((tid & (kWave - 1)) == 0) s_red[tid / kWave] = racc;
  __syncthreads();
  if (LEAF) {
    // Every leaf child's score comes from histograms by true wall reading w:
    //   HQ[w][c] = sum over free x with reading w of lambda(x) b'(x) Q(x,c),
    //   HQ[w][APAD] = sum of lambda(x) b'(x)  (the histogram behind P(z)),
    // lambda = 1 - rho on landmark cells, else 1.  Cells come in reading
    // order; thread k sums chunk k (one reading), then the chunk partials of
    // each reading are added in chunk order.
    constexpr int NV = APAD + 1;
    float *part = X;                      // [kBlock][NV]
    const int j0 = lv.sort_chunk[2 * tid], j1 = lv.sort_chunk[2 * tid + 1];
    float acc[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[c] = 0.f;
    for (int j = j0; j < j1; j += kSortBatch) {
      uint32_t e[kSortBatch];
      float q[kSortBatch][APAD];
#pragma unroll
      for (int k = 0; k < kSortBatch; ++k) e[k] = j + k < j1 ? (uint32_t)lv.sort_cells[j + k] : 0u;
#pragma unroll
      for (int k = 0; k < kSortBatch; ++k) load_q_row<APAD>(lv, A, (int)(e[k] & kSortCell), q[k]);
#pragma unroll
      for (int k = 0; k < kSortBatch; ++k) {
        if (j + k < j1) {
          const float bp = bpl[e[k] & kSortCell];
          const float v = (e[k] & kSortLandmark) ? bp * (1.f - rho) : bp;
#pragma unroll
          for (int c = 0; c < APAD; ++c) acc[c] = fmaf(v, q[k][c], acc[c]);
          acc[APAD] += v;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) part[tid * NV + c] = acc[c];
    __syncthreads();
    const int32_t *pch = lv.sort_chunk + 2 * kBlock;
    for (int i = tid; i < 16 * NV; i += kBlock) {
      const int w = i / NV, c = i - w * NV;
      s_HQ[i] = range_sum(part + c, NV, pch[w], pch[w + 1]);
    }
    __syncthreads();
    if (tid < 16) s_H[tid] = s_HQ[tid * NV + APAD];
    if (tid == 16) s_H[16] = sum_waves<NB / kWave>(s_red);
    __syncthreads();
  }
  if (!LEAF) {
    // the 16 bins: lane k of bin tid / TPB adds entries k, k + TPB, ... (the
    // lanes read consecutive words; the bins sharing a wavefront start their
    // walks one step apart, so no two lanes share an LDS bank), then TPB
    // lanes combine them
    constexpr int TPB = NB / 16;
    const int k = tid % TPB, rot = (tid / TPB) % (kWave / TPB);
    const float *hb = hist + (tid / TPB) * NB;
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += hb[k + TPB * ((i + rot) & 15)];
    s = group_sum<TPB>(s);
    if (tid % TPB == TPB - 1) s_H[tid / TPB] = s;
    if (tid == 0) s_H[16] = sum_waves<NB / kWave>(s_red);
    __syncthreads();
  }
  // observation draws by wave 0; X now takes the landmark terms
  if (tid < kWave) {
    uint32_t *lw = (uint32_t *)X;
    float *lvv = X + m.L;
    for (int l = tid; l < m.L; l += kWave) {
      lw[l] = lv.lm_wall[l];
      const int c = m.lm_cell[l];
      lvv[l] = (c >= 0 && c < S) ? bpl[c] : 0.f;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    sample_draws(m, lv, p, a, tid < 17 ? s_H[tid] : 0.f, lw, lvv, X + 2 * m.L, &s_draw);
    // (after the draws: the wait before them need not cover this store)
    if (tid == 16) lv.reward[p * A + a] = s_H[16];
  }
  __syncthreads();
  const int U = s_draw.U;
  // the children's place in the next level's visiting order: the atomics go
  // out now and their positions are used after the children are written
  ListPos lpos = {0, 0};
  if (!LEAF && lv.slot_list && tid == 0) lpos = list_take(lv, U);
  // per drawn z: O_w(zw | w) / P(z|b,a) for the 16 wall readings
  if (!LEAF && tid < U * 16) {
    const int r = tid >> 4, w = tid & 15;
    s_tab[tid] = wall_lik(m.flip, (uint32_t)(s_draw.z[r] & 15), (uint32_t)w) * s_draw.inv[r];
  }
  __syncthreads();
  if (!LEAF) {
    // Phi(b,a,z)(x') = O(z|x') b'(x') / P(z|b,a) for each drawn z (the
    // signatures of a batch of cells are loaded once for all children)
    for (int t0 = tid; t0 < S; t0 += NBATCH * NB) {
      if (!one_pass) {
#pragma unroll
        for (int j = 0; j < NBATCH; ++j) {
          const int t = t0 + j * NB;
          const uint32_t sv = lv.sig[t < S ? t : 0];
          sg[j] = t < S ? sv : 0u;
        }
      }
      for (int r = 0; r < U; ++r) {
        const uint32_t zl = (uint32_t)(s_draw.z[r] >> 4);
        const float *tab = s_tab + r * 16;
        float *out = lv.cbel + (size_t)(cb + r) * S;
#pragma unroll
        for (int j = 0; j < NBATCH; ++j) {
          const int t = t0 + j * NB;
          // written through (the next level reads it from other XCDs), so
          // the end of the launch has fewer dirty L2 lines to write back
          if (t < S)
            st_coherent(out + t, tab[sig_wall(sg[j])] * lm_lik(rho, zl, sig_lm(sg[j])) * bpl[t]);
        }
      }
    }
    if (lv.slot_list && tid < kWave) list_put(lv, cb, U, lpos);
    return;
  }
  // leaves (Alg. 5): sum_x Phi(b,a,z_r)(x) Q(x,c) for drawn z_r = zw + 16 zl
  // and every action c, from the histograms:
  //   zl = 0:  (1/P(z_r)) sum_w O_w(zw|w) HQ[w][c]
  //   zl = l:  (1/P(z_r)) O_w(zw|w_l) rho b'(x_l) Q(x_l,c)   (x_l the cell of l)
  // (X still holds the landmark walls and masses staged for the draws)
  if (tid < U * APAD) {
    constexpr int NV = APAD + 1;
    const int r = tid / APAD, c = tid - r * APAD;
    float v = 0.f;
    if (c < A) {
      const int z = s_draw.z[r];
      const uint32_t zw = (uint32_t)(z & 15);
      const int zl = z >> 4;
      if (zl == 0) {
#pragma unroll
        for (int w = 0; w < 16; ++w) v = fmaf(wall_lik(m.flip, zw, (uint32_t)w), s_HQ[w * NV + c], v);
      } else {
        const uint32_t *lw = (const uint32_t *)X;
        const float *lvv = X + m.L;
        const int cell = m.lm_cell[zl - 1];
        v = wall_lik(m.flip, zw, lw[zl - 1]) * rho * lvv[zl - 1] * lv.Q[(size_t)cell * A + c];
      }
      v *= s_draw.inv[r];
    }
    s_leaf[r * APAD + c] = v;
  }
  __syncthreads();
  const long long g = tr.first[lv.d] + p;
  if (tid == 0) {
    // leaf values V = max_a' (Alg. 5) and the Q-node value (Alg. 6)
    float q = s_H[16];
    const long long lf = tr.first[lv.d + 1] + cb;
    for (int r = 0; r < U; ++r) {
      float best = -INFINITY;
      for (int c = 0; c < A; ++c) best = fmaxf(best, s_leaf[r * APAD + c]);
      tr.value[lf + r] = best;
      q += tr.gamma * ((float)s_draw.count[r] / (float)lv.n) * best;
    }
    st_coherent(tr.qvalue + g * A + a, q);
  }
  wait_mem();
  __syncthreads();
  if (tid == 0) s_last = (count_arrival(&tr.node_ctr[g]) == A - 1);
  __syncthreads();
  if (!s_last) return;
  float *sh = X;
  if (tid < A) sh[lv.K + tid] = ld_coherent(tr.qvalue + g * A + tid);
  __syncthreads();
  if (tid == 0) finish_node(tr, lv.d, g, sh + lv.K);
  __syncthreads();
  climb_wg(tr, lv.d, p, sh, &s_last);
}

// ---------------------------------------------------------------------------
// k_leaf_parent: the last level with one workgroup per (parent slot, band of
// rows) that handles every action of the parent.  A leaf child's score is
// sum_x Phi(b,a,z)(x) Q(x,c) with Phi(b,a,z)(x) = O(z|x) b'_a(x) / P(z|b,a),
// and O(z|x) depends on x only through its true wall reading w(x) and its
// landmark, so every child of every action follows from
//   HQ_a[w][c] = sum over free x with reading w of lambda(x) b'_a(x) Q(x,c),
//   HQ_a[w][A'] = sum of lambda(x) b'_a(x)       (the histogram behind P(z)),
// lambda = 1 - rho on landmark cells, else 1, plus the predicted mass b'_a on
// each landmark cell.  The prediction is linear in the slip weights:
//   b'_a(x) = sum_k T'(a,k) s_k(x),  s_k(x) = b(x - d_k) + [move k blocked at x] b(x)
// (s_4 = b(x)), so with the nine basis histograms
//   E_k[w][c] = sum over x with reading w of lambda(x) s_k(x) Q(x,c)
// every action's histogram is HQ_a = sum_k T'(a,k) E_k.  The workgroup walks
// its band's free cells in wall-reading order (k_prep_sort), reads each 3x3
// neighbourhood and Q row once and accumulates the 9 (A'+1) basis sums, which
// do not depend on the number of actions.  The goal (whose own mass stays
// with weight 1 for every action) is scored on its own.  With several bands
// per parent, the band records are summed in band order by the last band to
// finish; then the wavefronts draw the observations of the actions in
// parallel, and the workgroup forms the leaf and Q-node values, the node value
// and the backup towards the root.
// ---------------------------------------------------------------------------
constexpr int kLeafParentBatch = 2;   // sorted cells whose loads go out together
constexpr int kLeafBlock = 2 * kBlock;   // threads of a k_leaf_parent workgroup
constexpr int kLeafBasisRound = 5;    // basis sums (values of k) per histogram round (two rounds)
constexpr int kLeafPiece = 16;        // chunks per piece of a wall reading's chunk range
constexpr int kLeafPieces = 32;       // pieces at most: kBlock / kLeafPiece + 15
static_assert(kBlock / kLeafPiece + 15 <= kLeafPieces, "piece table too small");

struct LeafParentShared {
  float slip[8 * 9];                    // slip table (rows a >= A zero)
  DrawOut draw[8];
  float leaf[8 * QV_MAX_SAMPLES * 8];   // [a][r][c] child scores
  float rb[8];                          // R(b,a)
  float qn[8];                          // Q-node values
  float red[2 * kBlock / kWave][8];
  float goal[8 * 9];                    // [a][c] lambda b'_a Q(goal, c) of the goal cell
  int goal_w;                           // the goal's wall reading, or -1 (not in this band)
  int last;
  int pc_lo[kLeafPieces], pc_hi[kLeafPieces];   // chunk range of each piece
  int pfirst[17];                              // first piece of each wall reading
};

// Floats of dynamic LDS: one region that holds in turn the band, the chunk
// partials and the landmark tables; then one that holds the predicted masses
// of the landmark cells during the cell pass and afterwards the basis
// histograms, the actions' histograms and the piece sums of one round.
__host__ __device__ inline size_t leaf_parent_lds_floats(int W, int TH, int L, int AM,
                                                        int NT = kLeafBlock) {
  const int NW = NT / kWave;
  const size_t band = (size_t)(TH + 2) * (W + 2);
  const size_t lmk = (size_t)(1 + NW) * L + 32 * NW;   // landmark tables, sampler tables
  const size_t part = (size_t)kBlock * kLeafBasisRound * (AM + 1);   // chunk partials, one round
  size_t x = band > lmk ? band : lmk;
  x = x > part ? x : part;
  const size_t hist = (size_t)9 * 16 * (AM + 1) + (size_t)AM * 16 * (AM + 1) +
                     (size_t)kLeafPieces * kLeafBasisRound * (AM + 1);
  const size_t lmt = (size_t)AM * L;
  return x + (hist > lmt ? hist : lmt);
}

// The histograms HQ ([AM][16][AM + 1]) and R(b,a) (sh.rb) of parent p from
// its band records, each entry summed in band order (records written with
// device-scope stores by the band items).  Ends with the workgroup's loads done
// (no barrier).
template <int AM, int NT>
__device__ void leaf_parent_sum_records(const LevelArgs &lv, int p, float *HQ,
                                        LeafParentShared &sh) {
  constexpr int NV = AM + 1;
  constexpr int RECN = AM * 16 * NV + AM;
  const float *rec0 = lv.part + (size_t)p * lv.tiles * RECN;
  for (int i = threadIdx.x; i < RECN; i += NT) {
    // the loads of up to 32 bands in flight together, summed in band order
    float sum = 0.f;
    for (int t0 = 0; t0 < lv.tiles; t0 += 32) {
      float x[32];
#pragma unroll
      for (int k = 0; k < 32; ++k)
        x[k] = t0 + k < lv.tiles ? ld_coherent(rec0 + (size_t)(t0 + k) * RECN + i) : 0.f;
#pragma unroll
      for (int k = 0; k < 32; ++k)
        if (t0 + k < lv.tiles) sum += x[k];
    }
    if (i < AM * 16 * NV)
      HQ[i] = sum;
    else
      sh.rb[i - AM * 16 * NV] = sum;
  }
}

// Completion of parent p of the last level from its whole-belief statistics
// (HQ, sh.rb; the landmark cells' predicted masses in lv.lmv): the draws of
// every action (Alg. 3/4), the leaf values of the drawn children (Alg. 5), the
// Q-node values (Alg. 6), the node value, then the backup towards the root
// (Alg. 7).  X: LDS scratch of at least (1 + NW) L + 32 NW floats and of the
// backup's K + A.
template <int AM, int NT>
__device__ void leaf_parent_finish(const DevModel &m, const LevelArgs &lv, const TreeArgs &tr,
                                   int p, float *X, const float *HQ, LeafParentShared &sh) {
  constexpr int NV = AM + 1;
  constexpr int NW = NT / kWave;
  const int A = m.A, L = m.L, K = lv.K, n = lv.n;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const float rho = m.lm_p;
  float *part = X;
  if (!lv.own_reward) {
    // R(b,a) of this parent came from the level above
    if (tid < A) sh.rb[tid] = lv.reward[p * A + tid];
    __syncthreads();
  }
  // observation draws: wavefront w takes actions w, w + 4, ...
  uint32_t *lw = (uint32_t *)X;
  for (int l = tid; l < L; l += NT) lw[l] = lv.lm_wall[l];
  wait_mem();
  __syncthreads();
  float *lvv = X + L + wave * L;
  for (int a = wave; a < A; a += NW) {
    for (int l = lane; l < L; l += kWave) lvv[l] = ld_coherent(lv.lmv + ((size_t)p * A + a) * L + l);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    float hs = 0.f;
    if (lane < 16) hs = HQ[(a * 16 + lane) * NV + AM];
    if (lane == 16) hs = sh.rb[a];
    sample_draws(m, lv, p, a, hs, lw, lvv, X + (1 + NW) * L + 32 * wave, &sh.draw[a]);
    // (after the draws: the wait before them need not cover this store)
    if (lane == 16 && lv.own_reward) lv.reward[p * A + a] = hs;
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // leaf values (Alg. 5) of every drawn child of every action:
  //   zl = 0: (1/P(z)) sum_w O_w(zw|w) HQ_a[w][c];  zl = l: (1/P(z)) O_w(zw|w_l) rho b'_a(x_l) Q(x_l,c)
  for (int i = tid; i < A * n * AM; i += NT) {
    const int a = i / (n * AM), r = (i / AM) - a * n, c = i - (i / AM) * AM;
    float v = 0.f;
    if (c < A && r < sh.draw[a].U) {
      const int z = sh.draw[a].z[r];
      const uint32_t zw = (uint32_t)(z & 15);
      const int zl = z >> 4;
      if (zl == 0) {
#pragma unroll
        for (int w = 0; w < 16; ++w)
          v = fmaf(wall_lik(m.flip, zw, (uint32_t)w), HQ[(a * 16 + w) * NV + c], v);
      } else {
        const int cell = m.lm_cell[zl - 1];
        v = wall_lik(m.flip, zw, lw[zl - 1]) * rho *
            ld_coherent(lv.lmv + ((size_t)p * A + a) * L + zl - 1) * lv.Q[(size_t)cell * A + c];
      }
      v *= sh.draw[a].inv[r];
    }
    sh.leaf[i] = v;
  }
  __syncthreads();
  // Q-node values (Alg. 6), the node value, then the backup towards the root
  const long long g = tr.first[lv.d] + p;
  if (tid < A) {
    const int a = tid;
    float qv = sh.rb[a];
    const long long lf = tr.first[lv.d + 1] + (long long)p * K + (long long)a * n;
    for (int r = 0; r < sh.draw[a].U; ++r) {
      float best = -INFINITY;
      for (int c = 0; c < A; ++c) best = fmaxf(best, sh.leaf[(a * n + r) * AM + c]);
      tr.value[lf + r] = best;
      qv += tr.gamma * ((float)sh.draw[a].count[r] / (float)n) * best;
    }
    tr.qvalue[g * A + a] = qv;
    sh.qn[a] = qv;
  }
  __syncthreads();
  if (tid == 0) finish_node(tr, lv.d, g, sh.qn);
  __syncthreads();
  climb_wg(tr, lv.d, p, part, &sh.last);
}

// k_leaf_finish's LDS: the scratch X (landmark tables and sampler tables of
// every wavefront, or the backup's K + A values), then the histograms HQ.
__host__ __device__ inline size_t leaf_finish_x_floats(int L, int K, int A, int NT) {
  const size_t lmk = (size_t)(1 + NT / kWave) * L + 32 * (NT / kWave);
  const size_t bk = (size_t)K + A;
  return lmk > bk ? lmk : bk;
}
__host__ __device__ inline size_t leaf_finish_lds_floats(int L, int K, int A, int AM) {
  return leaf_finish_x_floats(L, K, A, kLeafBlock) + (size_t)AM * 16 * (AM + 1);
}

// QV: how Q rows are read (load_q_row).  AM: Q columns padded to 4 or 8.
// NT threads (kBlock or 2 kBlock): with 2 kBlock, neighbouring lanes 2k and
// 2k + 1 share sorted chunk k (alternate cells) and every wavefront draws for
// one action.
template <int AM, int QV, int NT>
__device__ void leaf_parent_item(const DevModel &m, const LevelArgs &lv, const TreeArgs &tr,
                                 int p, int band, float *smem, LeafParentShared &sh) {
  static_assert(NT == kBlock || NT == 2 * kBlock, "one or two threads per chunk");
  constexpr int NV = AM + 1;
  constexpr int NW = NT / kWave;            // wavefronts
  constexpr int HALVES = NT / kBlock;       // threads per sorted chunk
  // sorted cells whose loads go out together (one at 2 kBlock threads, whose
  // workgroups must fit in 128 registers for two to share a CU)
  constexpr int LPB = NT == kBlock ? kLeafParentBatch : 1;
  constexpr int RECN = AM * 16 * NV + AM;   // band record: HQ, then R(b,a)
  const int A = m.A, W = m.W, BW = W + 2, S = m.S, L = m.L;
  const int K = lv.K;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  if (!lv.pvalid[p]) {
    // children of an absent parent are absent (marked by k_leaf_finish when
    // it completes the parents); the parent takes no part in any backup
    if (band == 0 && !lv.leaf_finish)
      for (int i = tid; i < K; i += NT) {
        const int c = p * K + i;
        lv.cvalid[c] = 0;
        lv.cz[c] = -1;
        lv.ccount[c] = 0;
        lv.cpz[c] = 0.f;
      }
    return;
  }
  const int TH = lv.TH, y0 = band * TH, th = min(TH, m.H - y0);
  const size_t bandf = (size_t)(TH + 2) * BW, lmkf = (size_t)(1 + NW) * L + 32 * NW;
  const size_t partf = (size_t)kBlock * kLeafBasisRound * NV;
  const size_t xf = bandf > lmkf ? (bandf > partf ? bandf : partf) : (lmkf > partf ? lmkf : partf);
  float *X = smem;             // band, then the chunk partials, then the landmark tables
  float *part = X;             // [kBlock][round values], later the backup scratch
  float *E = smem + xf;        // [9][16][NV] basis histograms
  float *HQ = E + 9 * 16 * NV;   // [AM][16][NV]
  float *PP = HQ + AM * 16 * NV;   // [piece][round values]
  float *LT = E;                   // [AM][L] b'_a of the landmark cells, during the cell pass
  const float *b = lv.pbel + (size_t)p * S;
  if (tid < AM * 9) sh.slip[tid] = tid < A * 9 ? m.slip[tid] : 0.f;
  if (tid == 0) sh.goal_w = -1;
  // landmarks outside this band keep the mark -1 (predicted masses are >= 0)
  for (int i = tid; i < AM * L; i += NT) LT[i] = -1.f;
  load_band<24 * kBlock / NT, NT>(m, lv.sig, b, y0, th, X, BW, lv.d == 0);
  __syncthreads();
  const float rho = m.lm_p;
  const float rW = 1.0f / (float)W;
  // the goal keeps its own mass (the band holds zero there)
  const float bgoal = (m.goal >= y0 * W && m.goal < (y0 + th) * W) ? b[m.goal] : 0.f;
  // R(b,a) = sum_x R(x,a) b(x) over the band's own rows, in cell order
  // (coalesced rows of R; the goal's own mass is read from b)
  float racc[AM];
#pragma unroll
  for (int a = 0; a < AM; ++a) racc[a] = 0.f;
  if (lv.own_reward) {
    const float *Rt = m.R;
    const bool r_vec = (A == AM) && ((reinterpret_cast<uintptr_t>(Rt) & 15u) == 0);
    const int ncell = th * W, t00 = y0 * W;
    for (int i0 = tid; i0 < ncell; i0 += 4 * NT) {
      float r4[4][AM], bb[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int i = i0 + k * NT;
        const int t = t00 + (i < ncell ? i : 0);
        if (r_vec) {
          const float4 *row = reinterpret_cast<const float4 *>(Rt + (size_t)t * AM);
#pragma unroll
          for (int c4 = 0; c4 < AM / 4; ++c4) {
            const float4 v4 = row[c4];
            r4[k][4 * c4] = v4.x;
            r4[k][4 * c4 + 1] = v4.y;
            r4[k][4 * c4 + 2] = v4.z;
            r4[k][4 * c4 + 3] = v4.w;
          }
        } else {
#pragma unroll
          for (int a = 0; a < AM; ++a) {
            const float rv = Rt[(size_t)t * A + (a < A ? a : 0)];
            r4[k][a] = a < A ? rv : 0.f;
          }
        }
        const int ic = i < ncell ? i : 0;
        const int ly = fdiv(ic, W, rW);
        const float xv = X[(ly + 1) * BW + (ic - ly * W) + 1];
        bb[k] = (i < ncell) ? ((t == m.goal) ? bgoal : xv) : 0.f;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int a = 0; a < AM; ++a) racc[a] = fmaf(bb[k], r4[k][a], racc[a]);
    }
  }
#pragma unroll
  for (int a = 0; a < AM; ++a) {
    const float tot = wave_total_lane63(racc[a]);
    if (lane == kWave - 1) sh.red[wave][a] = tot;
  }
  // basis sums E_k[c] of this thread's cells of its chunk (one wall reading)
  float acc[9][NV];
#pragma unroll
  for (int k = 0; k < 9; ++k)
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[k][c] = 0.f;
  const int32_t *ch = lv.sort_chunk + (size_t)band * kSortChunkInts;
  // chunk ck belongs to the reading w with pch[w] <= ck < pch[w+1]; the
  // HALVES (pch[w+1] - pch[w]) lanes of reading w take its sorted positions
  // [rst[w], rst[w+1]) in turn, so a wavefront's loads at one step fall on
  // consecutive positions (neighbouring cells of one reading)
  const int ck = tid / HALVES, half = tid % HALVES;
  const int32_t *pchk = ch + 2 * kBlock, *rst = pchk + 17;
  int lo = 0, hi = 0, cfirst = 0, nch = 1;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int a0 = pchk[v], a1 = pchk[v + 1], r0 = rst[v], r1 = rst[v + 1];
    const bool mine = (ck >= a0) & (ck < a1);
    lo = mine ? r0 : lo;
    hi = mine ? r1 : hi;
    cfirst = mine ? a0 : cfirst;
    nch = mine ? a1 - a0 : nch;
  }
  const int sd = HALVES * nch;   // between one lane's positions
  const int j0 = lo + (ck - cfirst) * HALVES + half, j1 = hi;
  if (wave == NW - 1 && lane < 16) {
    // reading w's chunks [pch[w], pch[w+1]) cut into pieces of at most
    // kLeafPiece chunks; pieces are numbered in reading order
    const int32_t *pch = ch + 2 * kBlock;
    const int c0 = pch[lane], c1 = pch[lane + 1];
    const int np = (c1 - c0 + kLeafPiece - 1) / kLeafPiece;
    int pf = np;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const int t = __shfl_up(pf, o, 16);
      if (lane >= o) pf += t;
    }
    pf -= np;
    sh.pfirst[lane] = pf;
    if (lane == 15) sh.pfirst[16] = pf + np;
    for (int j = 0; j < np; ++j) {
      sh.pc_lo[pf + j] = c0 + j * kLeafPiece;
      sh.pc_hi[pf + j] = min(c0 + (j + 1) * kLeafPiece, c1);
    }
  }
  // the lane's positions in batches, software-pipelined: while a batch is
  // computed, the next batch's Q rows and the entries of the one after are
  // in flight; positions past the reading read a valid entry and are masked
  // to zero, so the loads need no branch
  const int jmax = max(j1 - 1, 0);
  const int STEP = LPB * sd;
  uint32_t en[LPB], en2[LPB];
  float qn[LPB][AM];
#pragma unroll
  for (int k = 0; k < LPB; ++k) {
    const int jk = j0 + k * sd, jk2 = jk + STEP;
    const uint32_t v = (uint32_t)lv.sort_cells[min(jk, jmax)];
    const uint32_t v2 = (uint32_t)lv.sort_cells[min(jk2, jmax)];
    en[k] = jk < j1 ? v : 0u;
    en2[k] = jk2 < j1 ? v2 : 0u;
  }
#pragma unroll
  for (int k = 0; k < LPB; ++k) load_q_row<AM, QV>(lv, A, (int)(en[k] & kSortCell), qn[k]);
  for (int j = j0; j < j1; j += STEP) {
    uint32_t e[LPB];
    float q[LPB][AM];
#pragma unroll
    for (int k = 0; k < LPB; ++k) {
      e[k] = en[k];
#pragma unroll
      for (int c = 0; c < AM; ++c) q[k][c] = qn[k][c];
      en[k] = en2[k];
      load_q_row<AM, QV>(lv, A, (int)(en[k] & kSortCell), qn[k]);
    }
#pragma unroll
    for (int k = 0; k < LPB; ++k) {
      const int jn = j + 2 * STEP + k * sd;
      const uint32_t v = (uint32_t)lv.sort_cells[min(jn, jmax)];
      en2[k] = jn < j1 ? v : 0u;
    }
    // every lane runs the whole batch: a slot past its chunk's end reads the
    // band's first cell with weight zero
#pragma unroll
    for (int k = 0; k < LPB; ++k) {
      const bool in = j + k * sd < j1;
      const int t = in ? (int)(e[k] & kSortCell) : y0 * W;
      const int gy = fdiv(t, W, rW);
      const float *c = X + (gy - y0 + 1) * BW + (t - gy * W) + 1;
      const float self = c[0];
      // s_k: the mass that move k brings to x (from the neighbour at -d_k),
      // plus x's own mass when move k is blocked at x (bit clear in the
      // 8-neighbour pattern); s_4 = b(x)
      const uint32_t o8 = (e[k] >> kSortOutShift) & 0xFFu;
      float s[9];
      s[0] = c[BW + 1];
      s[1] = c[BW];
      s[2] = c[BW - 1];
      s[3] = c[1];
      s[4] = self;
      s[5] = c[-1];
      s[6] = c[-BW + 1];
      s[7] = c[-BW];
      s[8] = c[-BW - 1];
#pragma unroll
      for (int kk = 0; kk < 9; ++kk) {
        if (kk == 4) continue;
        const int bit = kk < 4 ? kk : kk - 1;
        s[kk] += ((o8 >> bit) & 1u) ? 0.f : self;
      }
      const bool goal = (e[k] & kSortGoal) != 0;
      const bool lmk = (e[k] & kSortLandmark) != 0;
      const float lam = (in && !goal) ? (lmk ? 1.f - rho : 1.f) : 0.f;
#pragma unroll
      for (int kk = 0; kk < 9; ++kk) {
        const float v = s[kk] * lam;
#pragma unroll
        for (int cc = 0; cc < AM; ++cc) acc[kk][cc] = fmaf(v, q[k][cc], acc[kk][cc]);
        acc[kk][AM] += v;
      }
      if (in && (lmk || goal)) {
        // b'_a(x) = sum_k T'(a,k) s_k(x): the predicted mass on a landmark
        // cell (for its observation) and on the goal, where the band holds
        // zero (s_k is the inflow only) and the own mass stays with weight 1
        const uint32_t sg = lv.sig[t];
        const uint32_t lid = sig_lm(sg);
        const float lg = lmk ? 1.f - rho : 1.f;
        for (int a = 0; a < A; ++a) {
          float v = 0.f;
#pragma unroll
          for (int kk = 0; kk < 9; ++kk) v = fmaf(sh.slip[a * 9 + kk], s[kk], v);
          if (goal) {
            v += bgoal;
            const float gv = lg * v;
            sh.goal[a * NV + AM] = gv;
#pragma unroll
            for (int cc = 0; cc < AM; ++cc) sh.goal[a * NV + cc] = gv * q[k][cc];
          }
          if (lmk) LT[a * L + lid - 1] = v;
        }
        if (goal) sh.goal_w = (int)sig_wall(sg);
      }
    }
  }
  // chunk partials -> basis histograms by wall reading, kLeafBasisRound
  // values of k per round: one thread per (piece, value) adds the piece's
  // chunk partials in chunk order, then one thread per (reading, value) adds
  // the reading's piece sums in piece order (range_sum)
  constexpr int G = kLeafBasisRound;
  constexpr int GW = G * NV;          // floats per thread and round
  __syncthreads();                    // the band is read no more: part takes its place
  // the landmark cells' predicted masses go out to lmv (the sampler of this
  // or, with several bands, the last band reads them); kept in LDS during the
  // cell pass, so no store waits there
  for (int i = tid; i < A * L; i += NT) {
    const int a = i / L, l = i - a * L;
    const float v = LT[a * L + l];
    if (v >= 0.f) st_coherent(lv.lmv + ((size_t)p * A + a) * L + l, v);
  }
#pragma unroll
  for (int k0 = 0; k0 < 9; k0 += G) {
    if constexpr (HALVES == 2) {
      // a chunk's two lanes add their sums on the DPP network (both get the
      // same bits: addition commutes), then store alternate values
#pragma unroll
      for (int gi = 0; gi < GW; gi += 2) {
        const int g0 = gi / NV, c0 = gi % NV, g1 = (gi + 1) / NV, c1 = (gi + 1) % NV;
        if (k0 + g0 < 9) {
          float v0 = acc[k0 + g0][c0];
          v0 += dpp_xor1(v0);
          if (gi + 1 < GW && k0 + g1 < 9) {
            float v1 = acc[k0 + g1][c1];
            v1 += dpp_xor1(v1);
            part[ck * GW + gi + half] = half ? v1 : v0;
          } else {
            part[ck * GW + gi] = v0;   // both lanes write the same value
          }
        }
      }
    } else {
#pragma unroll
      for (int gi = 0; gi < GW; ++gi)
        if (k0 + gi / NV < 9) part[ck * GW + gi] = acc[k0 + gi / NV][gi % NV];
    }
    __syncthreads();
    const int npc = sh.pfirst[16];
    for (int i = tid; i < npc * GW; i += NT) {
      const int pc = i / GW, gi = i - pc * GW;
      if (k0 + gi / NV < 9) PP[i] = range_sum(part + gi, GW, sh.pc_lo[pc], sh.pc_hi[pc]);
    }
    __syncthreads();
    for (int i = tid; i < 16 * GW; i += NT) {
      const int w = i / GW, gi = i - w * GW;
      const int g = gi / NV, c = gi - g * NV;
      if (k0 + g < 9) E[((k0 + g) * 16 + w) * NV + c] = range_sum(PP + gi, GW, sh.pfirst[w], sh.pfirst[w + 1]);
    }
    __syncthreads();
  }
  // the actions' histograms HQ_a = sum_k T'(a,k) E_k (k in order), plus the
  // goal's own term on its reading
  for (int i = tid; i < AM * 16 * NV; i += NT) {
    const int a = i / (16 * NV), wc = i - a * 16 * NV;
    float v = 0.f;
    if (a < A) {
#pragma unroll
      for (int k = 0; k < 9; ++k) v = fmaf(sh.slip[a * 9 + k], E[k * 16 * NV + wc], v);
      if (wc / NV == sh.goal_w) v += sh.goal[a * NV + wc % NV];
    }
    HQ[i] = v;
  }
  __syncthreads();
  if (tid < A) {
    float r8[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) r8[w] = sh.red[w][tid];
    sh.rb[tid] = sum_waves<NW>(r8);
  }
  __syncthreads();
  if (lv.tiles > 1 || lv.leaf_finish) {
    // band record out; k_leaf_finish / k_inner_finish, or else the last band
    // of the parent, sums all records in band order
    float *rec = lv.part + ((size_t)p * lv.tiles + band) * RECN;
    for (int i = tid; i < RECN; i += NT) st_coherent(rec + i, i < AM * 16 * NV ? HQ[i] : sh.rb[i - AM * 16 * NV]);
    if (lv.leaf_finish) return;
    wait_mem();
    __syncthreads();
    if (tid == 0) sh.last = (count_arrival(&lv.ctr[p]) == lv.tiles - 1);
    __syncthreads();
    if (!sh.last) return;
    leaf_parent_sum_records<AM, NT>(lv, p, HQ, sh);
    if (tid == 0) lv.ctr[p] = 0;
    __syncthreads();
  }
  leaf_parent_finish<AM, NT>(m, lv, tr, p, X, HQ, sh);
}

template <int AM, int QV>
__global__ __launch_bounds__(kLeafBlock, 4) void k_leaf_parent(DevModel m, LevelArgs lv,
                                                                 TreeArgs tr) {
  extern __shared__ float smem[];
  __shared__ LeafParentShared sh;
  // With a visiting order, the present parents come first: they are
  // dispatched first, dealt to the XCDs in turn and spread over the CUs,
  // while the workgroups of absent parents (which only mark their children
  // absent) come last.  Without one, workgroup i runs on XCD i mod 8; slot
  // p = node*K + a*n + r, and the low r (the first distinct draw of each
  // Q-node, nearly always present) would all land on the same XCDs when K
  // is a multiple of 8, so each group of 8 is rotated by its index.
  int i = blockIdx.x;
  const int grp8 = i >> 3;
  if (!lv.porder && (grp8 + 1) * 8 <= (int)gridDim.x) i = grp8 * 8 + ((i + grp8) & 7);
  const int j = i / lv.tiles, band = i - j * lv.tiles;
  const int p = lv.porder ? lv.porder[j] : j;
  leaf_parent_item<AM, QV, kLeafBlock>(m, lv, tr, p, band, smem, sh);
}

// Completion of the parents of the per-parent last level when it runs in
// several bands: one workgroup per parent, present parents first (with a
// visiting order), after every band item has written its record.  Doing it
// here rather than in the band item that arrives last keeps that work (the
// draws, the leaf values, the backup) off the XCD whose items run slowest,
// which otherwise collects most of it and falls further behind.  Absent
// parents mark their children absent.
template <int AM>
__global__ __launch_bounds__(kLeafBlock) void k_leaf_finish(DevModel m, LevelArgs lv,
                                                            TreeArgs tr) {
  extern __shared__ float smem[];
  __shared__ LeafParentShared sh;
  const int p = lv.porder ? lv.porder[blockIdx.x] : (int)blockIdx.x;
  if (!lv.pvalid[p]) {
    for (int i = threadIdx.x; i < lv.K; i += kLeafBlock) {
      const int c = p * lv.K + i;
      lv.cvalid[c] = 0;
      lv.cz[c] = -1;
      lv.ccount[c] = 0;
      lv.cpz[c] = 0.f;
    }
    return;
  }
  float *X = smem;
  float *HQ = smem + leaf_finish_x_floats(m.L, lv.K, m.A, kLeafBlock);
  leaf_parent_sum_records<AM, kLeafBlock>(lv, p, HQ, sh);
  __syncthreads();
  leaf_parent_finish<AM, kLeafBlock>(m, lv, tr, p, X, HQ, sh);
}

// Completion of parent p of an inner level whose band items ran the basis
// pass with R in place of Q (leaf_parent_item; own_reward as for the root),
// one workgroup per (parent, action), after every band item has written its
// record.  The band records hold, per action, the predicted mass by wall
// reading (column AM) and the reward-weighted sums RH_a[w][c] = sum over cells
// x of reading w of lambda(x) b'_a(x) R(x, c), plus R(b,a).  The workgroup
// sums its action's part in band order, draws the action's observations
// (wavefront 0; the present children go to the front of the next level's
// visiting order), and forms each drawn child's rewards (Sec. III update, the
// wall readings' likelihoods applied to the sums):
//   R(Phi(b,a,z), c) = (1/P(z)) sum_w O_w(zw|w) RH_a[w][c]           (zl = 0)
//   R(Phi(b,a,z), c) = (1/P(z)) O_w(zw|w_l) rho b'_a(x_l) R(x_l, c)   (zl = l)
// Items i: parent i / A, action i mod A.  Absent parents mark their
// children absent and send them to the back of the visiting order.
struct InnerFinishShared {
  DrawOut draw;
  float rb;   // R(b,a)
};
// dynamic LDS floats: the landmarks' wall readings and masses, the sampler's
// tables, then the action's sums
__host__ __device__ inline size_t inner_finish_lds_floats(int L, int AM) {
  return (size_t)2 * L + 32 + (size_t)16 * (AM + 1);
}
template <int AM>
__global__ __launch_bounds__(kBlock) void k_inner_finish(DevModel m, LevelArgs lv) {
  extern __shared__ float smem[];
  __shared__ InnerFinishShared sh;
  constexpr int NV = AM + 1;
  constexpr int RECN = AM * 16 * NV + AM;   // band record: HQ, then R(b,a)
  const int A = m.A, L = m.L, K = lv.K, n = lv.n;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int p = blockIdx.x / A, a = blockIdx.x - p * A;
  const int cb = p * K + a * n;
  if (!lv.pvalid[p]) {
    if (tid < n) {
      lv.cvalid[cb + tid] = 0;
      lv.cz[cb + tid] = -1;
      lv.ccount[cb + tid] = 0;
      lv.cpz[cb + tid] = 0.f;
    }
    list_absent_children(lv, cb);
    return;
  }
  uint32_t *lw = (uint32_t *)smem;   // [L] wall readings of the landmarks
  float *lvv = smem + L;             // [L] predicted masses of the landmark cells
  float *p0tab = smem + 2 * L;       // [32] sampler tables
  float *HQ = smem + 2 * L + 32;     // [16][NV] the action's sums
  // the action's sums and R(b,a): band records summed in band order, the
  // loads of up to 32 bands in flight together
  const float *rec0 = lv.part + (size_t)p * lv.tiles * RECN;
  for (int i = tid; i <= 16 * NV; i += kBlock) {
    const int off = i < 16 * NV ? a * 16 * NV + i : AM * 16 * NV + a;
    float sum = 0.f;
    for (int t0 = 0; t0 < lv.tiles; t0 += 32) {
      float x[32];
#pragma unroll
      for (int k = 0; k < 32; ++k)
        x[k] = t0 + k < lv.tiles ? ld_coherent(rec0 + (size_t)(t0 + k) * RECN + off) : 0.f;
#pragma unroll
      for (int k = 0; k < 32; ++k)
        if (t0 + k < lv.tiles) sum += x[k];
    }
    if (i < 16 * NV)
      HQ[i] = sum;
    else
      sh.rb = sum;
  }
  for (int l = tid; l < L; l += kBlock) {
    lw[l] = lv.lm_wall[l];
    lvv[l] = ld_coherent(lv.lmv + ((size_t)p * A + a) * L + l);
  }
  wait_mem();
  __syncthreads();
  if (wave == 0) {
    const float hs = lane < 16 ? HQ[lane * NV + AM] : 0.f;
    const int U = sample_draws(m, lv, p, a, hs, lw, lvv, p0tab, &sh.draw);
    if (lv.own_reward && lane == 0) lv.reward[p * A + a] = sh.rb;
    if (lv.slot_list) {
      ListPos lp = {0, 0};
      if (lane == 0) lp = list_take(lv, U);
      list_put(lv, cb, U, lp);
    }
  }
  __syncthreads();
  const float rho = m.lm_p;
  for (int i = tid; i < n * A; i += kBlock) {
    const int r = i / A, c = i - r * A;
    if (r >= sh.draw.U) continue;
    const int z = sh.draw.z[r];
    const uint32_t zw = (uint32_t)(z & 15);
    const int zl = z >> 4;
    float v = 0.f;
    if (zl == 0) {
#pragma unroll
      for (int w = 0; w < 16; ++w)
        v = fmaf(wall_lik(m.flip, zw, (uint32_t)w), HQ[w * NV + c], v);
    } else {
      const int cell = m.lm_cell[zl - 1];
      v = wall_lik(m.flip, zw, lw[zl - 1]) * rho * lvv[zl - 1] * m.R[(size_t)cell * A + c];
    }
    lv.creward[((size_t)cb + r) * A + c] = v * sh.draw.inv[r];
  }
}

// ---------------------------------------------------------------------------
// stored-leaf path: k_leaf_score per (leaf slot, band), then k_leaf_reduce and
// the single-workgroup k_backup
// ---------------------------------------------------------------------------
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

// V(leaf) = max_a' sum over bands (band order fixed).  With qroot the leaf is
// the root itself (depth 0) and its per-action sums are its Q-values.
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

__global__ __launch_bounds__(1024) void k_backup(TreeArgs g) {
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
size_t band_lds_bytes(int W, int TH) { return band_bytes(W, TH); }
// k_leaf: the band, then the block_sum32 scratch or the backup scratch
size_t leaf_lds_bytes(int W, int TH, int K, int A) {
  return band_bytes(W, TH) + std::max<size_t>((size_t)(kBlock / kWave) * 32,
                                              (size_t)K + A + (size_t)K * A) * sizeof(float);
}

// Dynamic LDS of k_node: b' of the whole grid, then the largest of the band,
// the per-thread bins, the landmark terms and the backup scratch.
// dynamic LDS of the fused path: with the level-0 launch's sort workgroups
// (sort_band<kNodeBlock>, about 68 KB of static LDS) a workgroup stays
// within the 160 KB of a CU
constexpr size_t kSmallLdsMax = 88 * 1024;
static size_t small_lds_bytes(int W, int H, int A, int n, int L) {
  const size_t S = (size_t)W * H;
  return (((S + 3) & ~(size_t)3) + small_x_floats(W, H, A, n, L) + (size_t)16 * kNodeBlock) *
         sizeof(float);
}

// Host-side ranges for rocprofv3 --marker-trace around a plan's launches and
// around each level's, when QVTS_ROCTX=1 in the environment (read once).
// They bracket the enqueueing on the host, which runs ahead of the GPU.
static bool roctx_ranges_on() {
  static const bool on = [] {
    const char *e = std::getenv("QVTS_ROCTX");
    return e && e[0] == '1';
  }();
  return on;
}
struct RoctxRange {
  bool on;
  explicit RoctxRange(const char *what, int d = -1) : on(roctx_ranges_on()) {
    if (!on) return;
    char msg[48];
    if (d >= 0)
      std::snprintf(msg, sizeof msg, "%s %d", what, d);
    else
      std::snprintf(msg, sizeof msg, "%s", what);
    roctxRangePushA(msg);
  }
  ~RoctxRange() {
    if (on) roctxRangePop();
  }
};

hipError_t launch_plan(const qv_model *mm, const float *Q, const float *b0, int D, int n,
                       uint64_t seed, uint32_t qid, int flags, int32_t *action_out,
                       float *rootQ_out, char *ws, const PlanLayout &L, hipStream_t st) {
  const RoctxRange plan_range("qv plan");
  const DevModel m = make_dev_model(mm);
  const qv_tree_layout &T = L.pub;
  const int A = m.A, K = A * n;
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
  int32_t *ctr = (int32_t *)(ws + L.counters);

  TreeArgs tr;
  tr.D = D;
  tr.n = n;
  tr.K = K;
  tr.A = A;
  tr.gamma = m.gamma;
  for (int d = 0; d < QV_MAX_DEPTH + 2; ++d) tr.first[d] = d <= D + 1 ? T.level_first[d] : 0;
  for (int d = 0; d < QV_MAX_DEPTH + 1; ++d) tr.slots[d] = d <= D ? T.level_slots[d] : 0;
  tr.valid = valid;
  tr.count = cnt;
  tr.value = value;
  tr.qvalue = qvalue;
  tr.reward = reward;
  tr.node_ctr = ctr + L.stats_ctr_len;
  tr.action_out = action_out;
  tr.rootQ_out = rootQ_out;

  uint32_t *lm_wall = (uint32_t *)(ws + L.lm_wall);
  const PrepExtra px = {valid, zrec, cnt, pz, ctr,
                        (long long)(L.stats_ctr_len + L.node_ctr_len + 2 * (QV_MAX_DEPTH + 1)),
                        lm_wall};
  prep_plan_launch(m, sig, staytab, err, px, st);

  const size_t lds_band = band_bytes(m.W, TH);
  const size_t lds_stats = lds_band + 16 * kBlock * sizeof(float);
  // banded inner levels take one item per (parent, band) over all actions;
  // QVTS_PER_ACTION_ITEMS=1 selects one item per (parent, band, action)
  const char *pa_env = std::getenv("QVTS_PER_ACTION_ITEMS");
  const bool per_action = pa_env && std::atoi(pa_env) == 1;
  const bool per_parent = !per_action && (long long)TH * m.W <= kParentCells * kBlock;
  const size_t lds_spar = stats_parent_lds_floats(m.W, TH, m.L) * sizeof(float);
  const size_t lds_leaf = leaf_lds_bytes(m.W, TH, K, A);
  const int q_vec = (A == 4 || A == 8) && ((uintptr_t)Q % 16 == 0);
  const size_t lds_small = small_lds_bytes(m.W, m.H, A, n, m.L);
  const bool small = !(flags & QV_PLAN_TILED) && lds_small <= kSmallLdsMax;
  int32_t *sort_cells = (int32_t *)(ws + L.sort_cells);
  int32_t *sort_chunk = (int32_t *)(ws + L.sort_chunk);
  // the last level: one workgroup per (parent, band) over all actions (A <= 8),
  // else one per Q-node (k_node) or per (band, action) (k_stats + k_leaf)
  const bool leaf_parent = !store_leaves && D > 0 && A <= 8;
  const int AM = A <= 4 ? 4 : 8;
  const size_t lds_lp =
      leaf_parent_lds_floats(m.W, L.leaf_rows, m.L, AM) * sizeof(float);
  if ((leaf_parent && (long long)L.leaf_rows * m.W > kSortMaxCells) ||
      (!leaf_parent && small && !store_leaves && D > 0 && m.S > kSortMaxCells))
    return hipErrorInvalidValue;   // cannot happen: leaf bands hold <= 8192 cells
  // on the fused path with D >= 2 the level-0 launch sorts the leaf bands
  const bool sort_in_l0 = leaf_parent && small && D >= 2;
  if (small) {
    const void *kn[5] = {(const void *)k_node<8, false, true>, (const void *)k_node<8, false>,
                         (const void *)k_node<4, true>, (const void *)k_node<8, true>,
                         (const void *)k_node<16, true>};
    for (const void *f : kn) {
      hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds_small);
      if (e != hipSuccess) return e;
    }
  }
  // on the banded path with D >= 2 the level-0 statistics launch sorts the
  // leaf bands; otherwise a launch of its own does
  const bool sort_in_stats = leaf_parent && !small && per_parent && D >= 2;
  // banded path, D >= 3, default flags: levels 1..D-2 take their statistics
  // from the basis pass over the sorted leaf bands with R in place of Q
  // (k_leaf_parent + k_inner_finish), which also forms every child's reward;
  // QV_PLAN_TILED keeps the per-action statistics of the batched path
  const bool basis_inner = sort_in_stats && D >= 3 && !(flags & QV_PLAN_TILED);
  const bool r_vec = (A == 4 || A == 8) && ((uintptr_t)m.R % 16 == 0);
  if (leaf_parent && !sort_in_l0 && !sort_in_stats) {
    QV_LAUNCH(k_prep_sort, dim3(L.leaf_tiles), dim3(kBlock), 0, st, m.S, L.leaf_rows * m.W, m.L,
              sig, sort_cells, sort_chunk);
  }
  if (leaf_parent) {
    // every instance: the inner levels may read R with another vector width than Q
    const void *kfs[2] = {AM == 4 ? (const void *)k_leaf_parent<4, 1> : (const void *)k_leaf_parent<8, 1>,
                          AM == 4 ? (const void *)k_leaf_parent<4, 0> : (const void *)k_leaf_parent<8, 0>};
    for (const void *kf : kfs) {
      hipError_t e = hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_lp);
      if (e != hipSuccess) return e;
    }
  } else if (small && !store_leaves && D > 0) {
    QV_LAUNCH(k_prep_sort, dim3(1), dim3(kBlock), 0, st, m.S, m.S, m.L, sig, sort_cells,
              sort_chunk);
  }
  for (int d = 0; d < D; ++d) {
    const RoctxRange level_range("qv plan level", d);
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
    lv.lm_wall = lm_wall;
    lv.ctr = ctr;
    lv.q_vec = q_vec;
    lv.leaf_finish = 0;
    lv.draws_apart = 0;
    lv.own_reward = 1;
    lv.creward = nullptr;
    lv.sort_cells = sort_cells;
    lv.sort_chunk = sort_chunk;
    lv.sort_bands = 0;
    lv.sort_tc = 0;
    // the per-parent last level visits its parents in an order formed by the
    // level above (present ones first).  Level e's list would start after
    // those of levels 1..e-1, its two counts at slot_n + 2 e.  (At inner
    // levels, which have at most one workgroup per CU, the extra dependent
    // load of the order at the start of every workgroup costs more than it
    // gains, so they keep slot order.)
    int32_t *slot_list = (int32_t *)(ws + L.slot_list);
    int32_t *slot_n = ctr + L.stats_ctr_len + L.node_ctr_len;
    long long loff[QV_MAX_DEPTH + 1] = {0};
    for (int e = 2; e <= D - 1; ++e) loff[e] = loff[e - 1] + T.level_slots[e - 1];
    const bool order_next = leaf_parent && d + 1 == D - 1;
    lv.slot_list = order_next ? slot_list + loff[d + 1] : nullptr;
    lv.slot_n = slot_n + 2 * (d + 1);
    lv.slot_cap = order_next ? (int)T.level_slots[d + 1] : 0;
    lv.porder = (leaf_parent && d >= 1 && d == D - 1) ? slot_list + loff[d] : nullptr;
    lv.agroups = 1;
    if (last && leaf_parent) {
      lv.TH = L.leaf_rows;
      lv.tiles = L.leaf_tiles;
      lv.part = (float *)(ws + L.leafrec);
      // several bands: the band items write records, k_leaf_finish completes
      // the parents
      lv.leaf_finish = L.leaf_tiles > 1 ? 1 : 0;
      // with basis inner levels, R(b,a) of these parents came from the level above
      lv.own_reward = basis_inner ? 0 : 1;
      const unsigned nb = (unsigned)((long long)lv.nslots * L.leaf_tiles);
      if (AM == 4 && q_vec)
        QV_LAUNCH_L(d, (k_leaf_parent<4, 1>), dim3(nb), dim3(kLeafBlock), lds_lp, st, m, lv, tr);
      else if (AM == 4)
        QV_LAUNCH_L(d, (k_leaf_parent<4, 0>), dim3(nb), dim3(kLeafBlock), lds_lp, st, m, lv, tr);
      else if (q_vec)
        QV_LAUNCH_L(d, (k_leaf_parent<8, 1>), dim3(nb), dim3(kLeafBlock), lds_lp, st, m, lv, tr);
      else
        QV_LAUNCH_L(d, (k_leaf_parent<8, 0>), dim3(nb), dim3(kLeafBlock), lds_lp, st, m, lv, tr);
      if (lv.leaf_finish) {
        const size_t lds_fin = leaf_finish_lds_floats(m.L, K, A, AM) * sizeof(float);
        if (AM == 4)
          QV_LAUNCH_L(d, k_leaf_finish<4>, dim3(lv.nslots), dim3(kLeafBlock), lds_fin, st, m, lv, tr);
        else
          QV_LAUNCH_L(d, k_leaf_finish<8>, dim3(lv.nslots), dim3(kLeafBlock), lds_fin, st, m, lv, tr);
      }
      continue;
    }
    if (small) {
      const unsigned nq = (unsigned)((long long)lv.nslots * A);
      if (d == 0 && sort_in_l0) {
        lv.sort_bands = L.leaf_tiles;
        lv.sort_tc = L.leaf_rows * m.W;
        QV_LAUNCH_L(d, (k_node<8, false, true>), dim3(nq + L.leaf_tiles), dim3(kNodeBlock), lds_small,
                    st, m, lv, tr);
      } else if (!last || store_leaves) {
        QV_LAUNCH_L(d, (k_node<8, false>), dim3(nq), dim3(kNodeBlock), lds_small, st, m, lv, tr);
      } else if (A <= 4) {
        QV_LAUNCH_L(d, (k_node<4, true>), dim3(nq), dim3(kBlock), lds_small, st, m, lv, tr);
      } else if (A <= 8) {
        QV_LAUNCH_L(d, (k_node<8, true>), dim3(nq), dim3(kBlock), lds_small, st, m, lv, tr);
      } else {
        QV_LAUNCH_L(d, (k_node<16, true>), dim3(nq), dim3(kBlock), lds_small, st, m, lv, tr);
      }
      continue;
    }
    // a level of few parents runs the per-parent kernels on thinner bands,
    // so that at least two band items share each CU (level 0: one parent,
    // 512 bands of one row at 512 x 512); the partials buffer holds
    // part_slots x tiles bands of each action.  QV_PLAN_TILED keeps the
    // layout's bands at every level, as the batched path does (its trees
    // are bitwise those of the batch)
    int TH_d = TH, tiles_d = tiles;
    if (per_parent && !small && !(flags & QV_PLAN_TILED)) {
      while (TH_d > 1 && (long long)lv.nslots * tiles_d < 512) {
        const int th2 = (TH_d + 1) / 2, t2 = (m.H + th2 - 1) / th2;
        if ((long long)lv.nslots * t2 > (long long)L.part_slots * tiles) break;
        TH_d = th2;
        tiles_d = t2;
      }
    }
    lv.TH = TH_d;
    lv.tiles = tiles_d;
    const unsigned nblk = (unsigned)((long long)lv.nslots * tiles_d * A);
    const unsigned npar = (unsigned)((long long)lv.nslots * tiles_d);
    if (basis_inner && d >= 1) {
      // statistics by the leaf kernel's basis pass over the sorted leaf bands,
      // with the rows of R in place of those of Q: per action, the predicted
      // mass and the reward-weighted sums by wall reading; k_inner_finish
      // draws and forms the children's rewards; the update writes the children
      lv.TH = L.leaf_rows;
      lv.tiles = L.leaf_tiles;
      lv.part = (float *)(ws + L.leafrec);
      lv.leaf_finish = 1;
      lv.own_reward = d == 1 ? 1 : 0;   // level 1's own R(b,a) is not formed above
      lv.creward = reward + T.level_first[d + 1] * A;
      lv.Q = m.R;
      const unsigned nb = (unsigned)((long long)lv.nslots * L.leaf_tiles);
      if (AM == 4 && r_vec)
        QV_LAUNCH_L(d, (k_leaf_parent<4, 1>), dim3(nb), dim3(kLeafBlock), lds_lp, st, m, lv, tr);
      else if (AM == 4)
        QV_LAUNCH_L(d, (k_leaf_parent<4, 0>), dim3(nb), dim3(kLeafBlock), lds_lp, st, m, lv, tr);
      else if (r_vec)
        QV_LAUNCH_L(d, (k_leaf_parent<8, 1>), dim3(nb), dim3(kLeafBlock), lds_lp, st, m, lv, tr);
      else
        QV_LAUNCH_L(d, (k_leaf_parent<8, 0>), dim3(nb), dim3(kLeafBlock), lds_lp, st, m, lv, tr);
      // draws and children's rewards, one workgroup per (parent, action)
      const size_t lds_fin = inner_finish_lds_floats(m.L, AM) * sizeof(float);
      const unsigned nfin = (unsigned)((long long)lv.nslots * A);
      if (AM == 4)
        QV_LAUNCH_L(d, k_inner_finish<4>, dim3(nfin), dim3(kBlock), lds_fin, st, m, lv);
      else
        QV_LAUNCH_L(d, k_inner_finish<8>, dim3(nfin), dim3(kBlock), lds_fin, st, m, lv);
      lv.TH = TH_d;
      lv.tiles = tiles_d;
      lv.part = part;
      lv.leaf_finish = 0;
      lv.Q = Q;
      QV_LAUNCH_L(d, k_update_parent, dim3(npar), dim3(kBlock), lds_band, st, m, lv);
      continue;
    }
    if (per_parent && d == 0 && sort_in_stats) {
      // the leaf-band sort runs beside the level-0 statistics, its tables in
      // the launch's dynamic LDS
      lv.draws_apart = 1;
      lv.sort_bands = L.leaf_tiles;
      lv.sort_tc = L.leaf_rows * m.W;
      const size_t lds_sort = sort_band_lds_bytes<kBlock>(lv.sort_tc);
      QV_LAUNCH_L(d, k_stats_parent<true>, dim3(npar + L.leaf_tiles), dim3(kBlock),
                  lds_spar > lds_sort ? lds_spar : lds_sort, st, m, lv);
      lv.sort_bands = 0;
      lv.sort_tc = 0;
      QV_LAUNCH_L(d, k_stats_draws, dim3((unsigned)((long long)lv.nslots * A)), dim3(kWave),
                  (size_t)(2 * m.L + 32) * sizeof(float), st, m, lv);
      lv.draws_apart = 0;
    } else if (per_parent) {
      lv.draws_apart = 1;
      QV_LAUNCH_L(d, k_stats_parent<false>, dim3(npar), dim3(kBlock), lds_spar, st, m, lv);
      QV_LAUNCH_L(d, k_stats_draws, dim3((unsigned)((long long)lv.nslots * A)), dim3(kWave),
                  (size_t)(2 * m.L + 32) * sizeof(float), st, m, lv);
      lv.draws_apart = 0;
    } else
      QV_LAUNCH_L(d, k_stats, dim3(nblk), dim3(kBlock), lds_stats, st, m, lv);
    // a level of few (parent, band) items splits each item's actions over up
    // to 4 workgroups, so that about 1024 of them share the writes
    int agroups = 1;
    while (agroups < 4 && agroups * 2 <= A && (long long)npar * agroups * 2 <= 1024) agroups *= 2;
    lv.agroups = agroups;
    if ((!last || store_leaves) && per_parent) {
      QV_LAUNCH_L(d, k_update_parent, dim3(npar * agroups), dim3(kBlock), lds_band, st, m, lv);
    } else if (!last || store_leaves) {
      QV_LAUNCH_L(d, k_update, dim3(nblk), dim3(kBlock), lds_band, st, m, lv);
    } else if (A <= 4) {
      QV_LAUNCH_L(d, k_leaf<4>, dim3(nblk), dim3(kBlock), lds_leaf, st, m, lv, tr);
    } else if (A <= 8) {
      QV_LAUNCH_L(d, k_leaf<8>, dim3(nblk), dim3(kBlock), lds_leaf, st, m, lv, tr);
    } else {
      QV_LAUNCH_L(d, k_leaf<16>, dim3(nblk), dim3(kBlock), lds_leaf, st, m, lv, tr);
    }
  }
  if (store_leaves || D == 0) {
    const long long nleaf = T.level_slots[D];
    const int32_t *lvalid = valid + T.level_first[D];
    const float *lb = D == 0 ? b0 : (const float *)(ws + T.belief_offset[D]);
    QV_LAUNCH(k_leaf_score, dim3((unsigned)(nleaf * tiles)), dim3(kBlock), 0, st, m, lb, lvalid,
              tiles, TH, Q, leafpart);
    QV_LAUNCH(k_leaf_reduce, dim3((unsigned)((nleaf + 255) / 256)), dim3(256), 0, st, lvalid,
              (int)nleaf, tiles, A, leafpart, value + T.level_first[D],
              D == 0 ? qvalue : (float *)nullptr);
    QV_LAUNCH(k_backup, dim3(1), dim3(1024), 0, st, tr);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched planning: the same item functions, fed from a device work queue
// that spans every query of the batch
// ---------------------------------------------------------------------------

// Query owning item i: the last q with base[q] <= i (base[nq] = total).
__device__ __forceinline__ int find_query(const int32_t *base, int nq, int i) {
  int lo = 0, hi = nq;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid] <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// A copy of a descriptor read from device memory, declared uniform word by
// word so that it lives in scalar registers (the compiler cannot prove the
// memory unchanged under the kernel's own stores, so it would load it per lane).
template <typename T>
__device__ __forceinline__ T uniform_copy(const T &src) {
  static_assert(sizeof(T) % 4 == 0, "word-sized descriptor");
  T out;
  const int *in = reinterpret_cast<const int *>(&src);
  int *o = reinterpret_cast<int *>(&out);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) o[i] = __builtin_amdgcn_readfirstlane(in[i]);
  return out;
}

__device__ __forceinline__ LevelArgs bind_level(const BatchQuery &bq, const BatchCall &c, int d) {
  LevelArgs lv = uniform_copy(bq.lv[d]);
  const BatchCall cu = uniform_copy(c);
  lv.Q = cu.Q;
  lv.q_vec = cu.q_vec;
  lv.key0 = cu.key0;
  lv.key1 = cu.key1;
  lv.qid = cu.qid;
  if (d == 0) lv.pbel = cu.b0;
  return lv;
}

__global__ void k_prep_batch(BatchPrep bp) {
  const int q = find_query(bp.base, bp.nq, blockIdx.x);
  const BatchQuery &bq = bp.q[q];
  const long long g = (long long)(blockIdx.x - bp.base[q]) * blockDim.x + threadIdx.x;
  prep_sig_one(bq.m, bq.sig, bq.staytab, bq.err, bq.px, g);
  if (g < QV_MAX_ACTIONS) bq.tr.rootQ_out[g] = 0.f;   // entries a >= A stay 0
  if (blockIdx.x == 0 && threadIdx.x < bp.nqueue) bp.queue[threadIdx.x] = 0;
}

// leaf-band sort of the queries whose last level runs k_leaf_parent items
__global__ __launch_bounds__(kBlock) void k_prep_sort_batch(BatchPrep bp) {
  const int q = find_query(bp.sort_base, bp.nq, blockIdx.x);
  const BatchQuery &bq = bp.q[q];
  const LevelArgs &lv = bq.lv[bq.D - 1];
  const int band = blockIdx.x - bp.sort_base[q];
  const int TC = lv.TH * bq.m.W, c_lo = band * TC;
  sort_band(c_lo, min(bq.m.S, c_lo + TC), bq.m.L, bq.sig, (int32_t *)lv.sort_cells,
            (int32_t *)lv.sort_chunk + (size_t)band * kSortChunkInts);
}

__global__ void k_prep_landmarks_batch(BatchPrep bp) {
  const int q = find_query(bp.lm_base, bp.nq, blockIdx.x);
  const BatchQuery &bq = bp.q[q];
  const int l = (blockIdx.x - bp.lm_base[q]) * blockDim.x + threadIdx.x;
  prep_landmark_one(bq.m, bq.sig, bq.err, bq.px.lm_wall, l);
}

// PHASE 0: statistics and draws of the Q-nodes of level d (k_stats);
// PHASE 1: child beliefs (k_update) or, at the last level of a query with
// 9 actions, leaf scoring and backup (k_leaf);
// PHASE 2: the last level of a query with at most 8 actions, per (parent,
// band) over all actions (k_leaf_parent).  Workgroups take `chunk` items at a time from the
// queue until it runs dry; every workgroup leaves after one failed take.
// (phase 2 runs k_leaf_parent's 512-thread form, so a query's results equal
// those of its single-query plan bit for bit)
template <int PHASE, int APAD>
__global__ __launch_bounds__(PHASE == 2 ? kLeafBlock : kBlock, PHASE == 2 && APAD == 4 ? 4 : 1) void k_level_batch(BatchLevel bl) {
  extern __shared__ float smem[];
  __shared__ BandShared sh;
  __shared__ LeafParentShared shl;   // phase 2 only
  __shared__ int s_item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(bl.queue, bl.chunk);
    __syncthreads();
    const int i0 = s_item;
    if (i0 >= bl.total) break;
    const int i1 = min(i0 + bl.chunk, bl.total);
    for (int i = i0; i < i1; ++i) {
      const int q = __builtin_amdgcn_readfirstlane(find_query(bl.base, bl.nq, i));
      const BatchQuery &bq = bl.q[q];
      const LevelArgs lv = bind_level(bq, bl.call[q], bl.d);
      const Item it = decode_item(i - bl.base[q], lv.tiles, bq.m.A);
      if constexpr (PHASE == 0) {
        stats_item(bq.m, lv, it, smem, sh);
      } else if constexpr (PHASE == 1) {
        if (bl.d + 1 < bq.D)
          update_item(bq.m, lv, it, smem, sh);
        else
          leaf_item<APAD>(bq.m, lv, bq.tr, it, smem, sh);
      } else {
        const int local = i - bl.base[q];
        leaf_parent_item<APAD, -1, kLeafBlock>(bq.m, lv, bq.tr, local / lv.tiles, local % lv.tiles,
                                               smem, shl);
      }
      __syncthreads();
    }
  }
}

__global__ void k_batch_out(int nq, const int32_t *act_in, const float *rq_in, int32_t *act_out,
                            float *rq_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nq) act_out[i] = act_in[i];
  if (i < nq * QV_MAX_ACTIONS) rq_out[i] = rq_in[i];
}

#define QV_LAUNCH_T(timed, tag, kernel, grid, block, lds, st, ...)             \
  do {                                                                      \
    if (timed) {                                                            \
      QV_LAUNCH_L(tag, kernel, grid, block, lds, st, __VA_ARGS__);          \
    } else {                                                                \
      hipLaunchKernelGGL(kernel, grid, block, lds, st, __VA_ARGS__);        \
    }                                                                       \
  } while (0)

hipError_t launch_batch_prep(const BatchPrep &bp, int cell_blocks, int lm_blocks,
                             int sort_blocks, hipStream_t st, bool timed) {
  QV_LAUNCH_T(timed, 0, k_prep_batch, dim3(cell_blocks), dim3(256), 0, st, bp);
  if (lm_blocks > 0)
    QV_LAUNCH_T(timed, 0, k_prep_landmarks_batch, dim3(lm_blocks), dim3(256), 0, st, bp);
  if (sort_blocks > 0)
    QV_LAUNCH_T(timed, 0, k_prep_sort_batch, dim3(sort_blocks), dim3(kBlock), 0, st, bp);
  return hipGetLastError();
}

size_t leaf_parent_lds_bytes(int W, int TH, int L, int AM) {
  return leaf_parent_lds_floats(W, TH, L, AM) * sizeof(float);
}

template <int PHASE, int APAD>
static const void *level_kernel() {
  return (const void *)k_level_batch<PHASE, APAD>;
}

static const void *batch_kernel_ptr(int phase, int apad) {
  if (phase == 0) return level_kernel<0, 4>();
  if (phase == 2) return apad <= 4 ? level_kernel<2, 4>() : level_kernel<2, 8>();
  if (apad <= 4) return level_kernel<1, 4>();
  if (apad <= 8) return level_kernel<1, 8>();
  return level_kernel<1, 16>();
}

int batch_level_occupancy(int phase, int apad, size_t lds) {
  const void *k = batch_kernel_ptr(phase, apad);
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, phase == 2 ? kLeafBlock : kBlock, lds) !=
      hipSuccess)
    return 0;
  return nb;
}

hipError_t launch_batch_level(const BatchLevel &bl, int phase, int apad, size_t lds, int grid,
                              hipStream_t st, bool timed) {
  if (grid <= 0) return hipSuccess;
  const int d = bl.d;
  if (phase == 0) {
    QV_LAUNCH_T(timed, d, (k_level_batch<0, 4>), dim3(grid), dim3(kBlock), lds, st, bl);
  } else if (phase == 2 && apad <= 4) {
    QV_LAUNCH_T(timed, d, (k_level_batch<2, 4>), dim3(grid), dim3(kLeafBlock), lds, st, bl);
  } else if (phase == 2) {
    QV_LAUNCH_T(timed, d, (k_level_batch<2, 8>), dim3(grid), dim3(kLeafBlock), lds, st, bl);
  } else if (apad <= 4) {
    QV_LAUNCH_T(timed, d, (k_level_batch<1, 4>), dim3(grid), dim3(kBlock), lds, st, bl);
  } else if (apad <= 8) {
    QV_LAUNCH_T(timed, d, (k_level_batch<1, 8>), dim3(grid), dim3(kBlock), lds, st, bl);
  } else {
    QV_LAUNCH_T(timed, d, (k_level_batch<1, 16>), dim3(grid), dim3(kBlock), lds, st, bl);
  }
  return hipGetLastError();
}

hipError_t launch_batch_out(int nq, const int32_t *act_in, const float *rq_in, int32_t *act_out,
                            float *rq_out, hipStream_t st) {
  const int n = nq * QV_MAX_ACTIONS;
  if (n == 0) return hipSuccess;
  QV_LAUNCH(k_batch_out, dim3((n + 255) / 256), dim3(256), 0, st, nq, act_in, rq_in, act_out,
            rq_out);
  return hipGetLastError();
}

}  // namespace qv

namespace qv {

// ===========================================================================
// Best-first (anytime) QV-tree search, Alg. 1 with Alg. 2-7 and the
// heuristics of Sec. IV-C.  The tree lives in a node pool in the workspace:
// node 0 is the first root; every expansion reserves K = |A| n consecutive
// node ids (child (a, r) of the expansion at base + a n + r, as the level
// kernels place children in capacity slots); a root made by update(a, z)
// takes one id.  Which node to expand next is kept on the device
// (ctl[kCtlSelect] = E of the root), so a run of expansions is a chain of
// launches with no host round trip: k_search_expand (one workgroup per
// action of the selected node: prediction, P(z|b,a), draws, children
// Phi(b,a,z) and their bounds U = max_a' b.U_table, L = max_a' b.L_table)
// then k_search_update (Alg. 6/7 at the node and at every ancestor, one
// thread), which selects the next node.  Grids whose belief, predicted
// belief and bins fit in LDS only (the anytime search serves small and
// medium maps; the level-synchronous plan covers the large ones).
// ===========================================================================
constexpr int kCtlRoot = 0, kCtlSelect = 1, kCtlNext = 2, kCtlExpansions = 3, kCtlFlags = 4,
              kCtlErr = 5;
constexpr int kSearchFull = 1;     // the pool cannot hold another expansion
constexpr int kSearchDone = 2;     // the node to expand is already expanded

__host__ __device__ inline size_t search_lds_floats(int W, int H) {
  const size_t band = (size_t)(H + 2) * (W + 2);
  const size_t S = (size_t)W * H;
  return band + ((S + 3) & ~(size_t)3) + 16 * (size_t)kBlock;
}

// Bounds of a belief held as v(t) = scale * o(t) * bp(t) over all cells:
// block sums of v(t) Ut(t, a') (A columns) and v(t) Lt(t, j) (sa.lcols
// columns), each in a fixed order, then the maxima U and L (every thread gets
// them).  o(t) = 1 when zr < 0.  The first pass also writes v to out_b and
// takes the U columns with the first 16 L columns; further passes take 32 L
// columns each.
template <int NT = kBlock>
__device__ void search_bounds(const DevModel &m, const SearchArgs &sa, const float *bpl,
                              int zr, float scale, float *out_b, float *red, float &U,
                              float &L) {
  const int A = m.A, S = m.S, LC = sa.lcols;
  const uint32_t zw = (uint32_t)(zr & 15), zl = (uint32_t)(zr >> 4);
  U = -INFINITY;
  L = -INFINITY;
  for (int c0 = -16; c0 < LC; c0 += 32) {
    // c0 < 0: values 0..15 are the U columns, 16..31 the L columns 0..15;
    // else values 0..31 are the L columns c0 .. c0+31
    float acc[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) acc[i] = 0.f;
    for (int t = threadIdx.x; t < S; t += NT) {
      const uint32_t sg = sa.sig[t];
      float o = 1.f;
      if (zr >= 0) o = wall_lik(m.flip, zw, sig_wall(sg)) * lm_lik(m.lm_p, zl, sig_lm(sg));
      const float v = o * bpl[t] * scale;
      if (c0 < 0) {
        if (out_b) out_b[t] = v;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if (c < A) acc[c] = fmaf(v, sa.Ut[(size_t)t * A + c], acc[c]);
          if (c < LC) acc[16 + c] = fmaf(v, sa.Lt[(size_t)t * LC + c], acc[16 + c]);
        }
      } else {
#pragma unroll
        for (int c = 0; c < 32; ++c)
          if (c0 + c < LC) acc[c] = fmaf(v, sa.Lt[(size_t)t * LC + c0 + c], acc[c]);
      }
    }
    const float tot = block_sum32<NT>(acc, red);
    // thread c < 32 holds the total of value c; the maxima through LDS
    if (threadIdx.x < 32) red[threadIdx.x] = tot;
    __syncthreads();
    if (c0 < 0) {
      for (int c = 0; c < A; ++c) U = fmaxf(U, red[c]);
      for (int c = 0; c < 16 && c < LC; ++c) L = fmaxf(L, red[16 + c]);
    } else {
      for (int c = 0; c < 32 && c0 + c < LC; ++c) L = fmaxf(L, red[c]);
    }
    __syncthreads();
  }
}

// The new node c's records (its belief is already in place).
__device__ __forceinline__ void search_new_node(const SearchArgs &sa, int c, int parentq,
                                                float w, int z, int depth, float U, float L) {
  sa.valid[c] = 1;
  sa.parent[c] = parentq;
  sa.w[c] = w;
  sa.z[c] = z;
  sa.depth[c] = depth;
  sa.U[c] = U;
  sa.L[c] = L;
  sa.H[c] = U - L;
  sa.E[c] = c;
  sa.expanded[c] = 0;
  sa.cbase[c] = -1;
}

__global__ __launch_bounds__(kBlock) void k_search_init(DevModel m, SearchArgs sa,
                                                        const float *b0) {
  __shared__ float red[4 * 32];
  extern __shared__ float smem[];
  float *bpl = smem;
  for (int t = threadIdx.x; t < m.S; t += kBlock) {
    // the start belief, with no mass on blocked cells
    bpl[t] = (sa.sig[t] & kSigFree) ? b0[t] : 0.f;
  }
  __syncthreads();
  float U, L;
  search_bounds(m, sa, bpl, -1, 1.f, sa.bel, red, U, L);
  if (threadIdx.x == 0) {
    search_new_node(sa, 0, -1, 1.f, -1, 0, U, L);
    sa.pz[0] = 0.f;
    sa.count[0] = 0;
    sa.ctl[kCtlRoot] = 0;
    sa.ctl[kCtlSelect] = 0;
    sa.ctl[kCtlNext] = 1;
    sa.ctl[kCtlExpansions] = 0;
    sa.ctl[kCtlFlags] = 0;
    sa.ctl[kCtlErr] = 0;
  }
}

// One workgroup per action a of the selected node v (Alg. 2-5).
__global__ __launch_bounds__(kBlock) void k_search_expand(DevModel m, SearchArgs sa) {
  extern __shared__ float smem[];
  __shared__ float s_stay[256];
  __shared__ float s_red[4 * 32];
  __shared__ float s_H[17];
  __shared__ DrawOut s_draw;
  const int a = blockIdx.x, tid = threadIdx.x;
  const int v = sa.ctl[kCtlSelect], base = sa.ctl[kCtlNext];
  if (sa.ctl[kCtlFlags] || v < 0 || sa.expanded[v] || base + sa.K > sa.NV) return;
  const int A = m.A, W = m.W, H = m.H, S = m.S, BW = W + 2;
  float *band = smem;
  float *bpl = band + (size_t)(H + 2) * BW;
  float *hist = bpl + ((S + 3) & ~3);   // [16][kBlock] per-thread bins
  const float *b = sa.bel + (size_t)v * S;
  LevelArgs lv{};
  lv.d = sa.depth[v];
  lv.n = sa.n;
  lv.K = sa.K;
  lv.key0 = sa.key0;
  lv.key1 = sa.key1;
  lv.qid = sa.qid;
  lv.cvalid = sa.valid;
  lv.cz = sa.z;
  lv.ccount = sa.count;
  lv.cpz = sa.pz;
  s_stay[tid] = sa.staytab[a * 256 + tid];
  load_band(m, sa.sig, b, 0, H, band, BW, false);
#pragma unroll
  for (int w = 1; w < 16; ++w) hist[w * kBlock + tid] = 0.f;
  __syncthreads();
  const float rW = 1.0f / (float)W;
  const float *sl = &m.slip[a * 9];
  const float rho = m.lm_p;
  const float bgoal = m.goal >= 0 ? b[m.goal] : 0.f;
  // b' (slip stencil), R(b,a) and the histogram of b' by true wall reading
  // (landmark cells with their "no landmark" factor), as the level kernels
  float racc = 0.f, h0 = 0.f;
  for (int t = tid; t < S; t += kBlock) {
    const uint32_t sg = sa.sig[t];
    const int ly = fdiv(t, W, rW), lx = t - ly * W;
    const float bt = t == m.goal ? bgoal : band[(ly + 1) * BW + lx + 1];
    racc = fmaf(bt, m.R[(size_t)t * A + a], racc);
    const float bp = predict_cell_v(band, BW, ly, lx, sg, sl, s_stay, bt);
    bpl[t] = bp;
    const uint32_t lm = sig_lm(sg);
    const float contrib = (lm && lm <= (uint32_t)m.L) ? bp * (1.f - rho) : bp;
    const uint32_t w = sig_wall(sg);
    if (w == 0u)
      h0 += contrib;
    else
      hist[w * kBlock + tid] += contrib;
  }
  hist[tid] = h0;
  racc = wave_sum(racc);
  if ((tid & (kWave - 1)) == 0) s_red[tid / kWave] = racc;
  __syncthreads();
  {
    const int k = tid & 15, rot = (tid >> 4) & 3;
    const float *hb = hist + (tid >> 4) * kBlock;
    float sum = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) sum += hb[k + 16 * ((i + rot) & 15)];
    sum = group_sum<16>(sum);
    if ((tid & 15) == 15) s_H[tid >> 4] = sum;
    if (tid == 0) s_H[16] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
  }
  __syncthreads();
  // draws (Alg. 3/4) by wavefront 0, keyed by the node id and its depth; the
  // landmark tables go where the bins were
  if (tid < kWave) {
    uint32_t *lw = (uint32_t *)hist;
    float *lvv = hist + m.L;
    for (int l = tid; l < m.L; l += kWave) {
      lw[l] = sa.lm_wall[l];
      const int c = m.lm_cell[l];
      lvv[l] = (c >= 0 && c < S) ? bpl[c] : 0.f;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    sample_draws(m, lv, v, a, tid < 17 ? s_H[tid] : 0.f, lw, lvv, hist + 2 * m.L, &s_draw,
                 base);
  }
  if (tid == 0) sa.rb[(size_t)v * A + a] = s_H[16];
  // b'_a for the children's workgroups (k_search_child)
  for (int t = tid; t < S; t += kBlock) sa.bpa[(size_t)a * S + t] = bpl[t];
}

// Child base + a n + r of the node expanded by k_search_expand (one
// workgroup per (action, draw), after it): its belief Phi(b,a,z_r) and its
// bounds (Alg. 3, Alg. 5) from b'_a, then its records.  Draws left empty
// return.
constexpr int kSearchChildBlock = 1024;   // threads of a k_search_child workgroup
__global__ __launch_bounds__(kSearchChildBlock) void k_search_child(DevModel m, SearchArgs sa) {
  __shared__ float s_red[kSearchChildBlock / kWave * 32];
  const int a = blockIdx.x / sa.n, r = blockIdx.x - a * sa.n;
  const int v = sa.ctl[kCtlSelect], base = sa.ctl[kCtlNext];
  if (sa.ctl[kCtlFlags] || v < 0 || sa.expanded[v] || base + sa.K > sa.NV) return;
  const int c = base + a * sa.n + r;
  if (!sa.valid[c]) return;
  const int S = m.S;
  const int z = sa.z[c];
  float U, L;
  search_bounds<kSearchChildBlock>(m, sa, sa.bpa + (size_t)a * S, z, 1.0f / sa.pz[c],
                                   sa.bel + (size_t)c * S, s_red, U, L);
  if (threadIdx.x == 0)
    search_new_node(sa, c, v * m.A + a, (float)sa.count[c] / (float)sa.n, z, sa.depth[v] + 1, U,
                    L);
}

// Alg. 6 for every action of expanded node v, then Alg. 7 (gamma in the
// Q-node backup; H(b,a) = 1 only for the action of largest U_Q; the child
// of largest gamma * weight * H gives H_Q and E_Q; first maximum on ties).
// One wavefront: lane a backs up action a over its children in order, then
// every lane takes the actions in order.  Child records are read past the
// cache (lane 0 wrote the previous node of the climb).
__device__ void search_update_node(const DevModel &m, const SearchArgs &sa, int v, int cb) {
  const int A = m.A, n = sa.n;
  const int lane = threadIdx.x & (kWave - 1);
  const float g = m.gamma;
  float uq = -INFINITY, lq = -INFINITY, hq = -INFINITY;
  int eq = v;
  if (lane < A) {
    const int a = lane;
    const float r = sa.rb[(size_t)v * A + a];
    float su = 0.f, sl = 0.f;
    for (int i = 0; i < n; ++i) {
      const int c = cb + a * n + i;
      if (!sa.valid[c]) continue;
      const float w = sa.w[c];
      su = fmaf(w, ld_coherent(sa.U + c), su);
      sl = fmaf(w, ld_coherent(sa.L + c), sl);
      const float h = g * w * ld_coherent(sa.H + c);
      if (h > hq) {
        hq = h;
        eq = __hip_atomic_load(sa.E + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    uq = fmaf(g, su, r);
    lq = fmaf(g, sl, r);
    sa.UQ[(size_t)v * A + a] = uq;
    sa.LQ[(size_t)v * A + a] = lq;
    sa.HQ[(size_t)v * A + a] = hq;
    sa.EQ[(size_t)v * A + a] = eq;
  }
  float bestU = -INFINITY, bestL = -INFINITY, Hs = 0.f;
  int Es = v;
  for (int a = 0; a < A; ++a) {
    const float u = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(uq), a));
    const float l = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lq), a));
    if (u > bestU) {
      bestU = u;
      Hs = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hq), a));
      Es = __builtin_amdgcn_readlane(eq, a);
    }
    bestL = fmaxf(bestL, l);
  }
  if (lane == 0) {
    st_coherent(sa.U + v, bestU);
    st_coherent(sa.L + v, bestL);
    st_coherent(sa.H + v, Hs);
    __hip_atomic_store(sa.E + v, Es, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  wait_mem();
  __builtin_amdgcn_wave_barrier();
}

// One wavefront: lane 0 keeps the control words, every lane takes part in
// the climb.
__global__ void k_search_update(DevModel m, SearchArgs sa) {
  const int lane = threadIdx.x & (kWave - 1);
  if (threadIdx.x >= kWave) return;
  const int v = sa.ctl[kCtlSelect], base = sa.ctl[kCtlNext];
  if (sa.ctl[kCtlFlags] || v < 0) return;
  if (sa.expanded[v]) {
    if (lane == 0) sa.ctl[kCtlFlags] |= kSearchDone;
    return;
  }
  if (base + sa.K > sa.NV) {
    if (lane == 0) sa.ctl[kCtlFlags] |= kSearchFull;
    return;
  }
  // child slots that the draws left empty
  for (int i = lane; i < sa.K; i += kWave)
    if (!sa.valid[base + i]) sa.E[base + i] = -1;
  const int root = sa.ctl[kCtlRoot];
  if (lane == 0) {
    sa.expanded[v] = 1;
    sa.cbase[v] = base;
    sa.ctl[kCtlNext] = base + sa.K;
    sa.log[sa.ctl[kCtlExpansions]] = v;
    sa.ctl[kCtlExpansions] += 1;
  }
  int p = v, cb = base;
  while (p >= 0) {
    search_update_node(m, sa, p, cb);
    if (p == root) break;
    const int pq = sa.parent[p];
    p = pq >= 0 ? pq / m.A : -1;
    if (p >= 0) cb = sa.cbase[p];
  }
  if (lane == 0)
    sa.ctl[kCtlSelect] = __hip_atomic_load(sa.E + root, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// getOptimalAction: the lowest action whose L_Q at the root is within 1e-9
// of the largest (-1 while the root is not expanded), and the root's Q-node
// bounds.
__global__ void k_search_result(DevModel m, SearchArgs sa, int32_t *action, float *rootU,
                                float *rootL) {
  if (threadIdx.x != 0) return;
  const int r = sa.ctl[kCtlRoot], A = m.A;
  if (!sa.expanded[r]) {
    action[0] = -1;
    for (int a = 0; a < A; ++a) {
      rootU[a] = sa.U[r];
      rootL[a] = sa.L[r];
    }
    return;
  }
  float best = -INFINITY;
  for (int a = 0; a < A; ++a) best = fmaxf(best, sa.LQ[(size_t)r * A + a]);
  int act = 0;
  for (int a = 0; a < A; ++a)
    if (sa.LQ[(size_t)r * A + a] >= best - 1e-9f) {
      act = a;
      break;
    }
  action[0] = act;
  for (int a = 0; a < A; ++a) {
    rootU[a] = sa.UQ[(size_t)r * A + a];
    rootL[a] = sa.LQ[(size_t)r * A + a];
  }
}

// update(a, z) of Alg. 1: the root moves to its child under (a, z), whose
// subtree stays; if z was not drawn there, a new root Phi(b_root, a, z) takes
// the next free id.  ctl[kCtlErr]: 1 = P(z|b,a) = 0, 2 = the pool is full.
__global__ __launch_bounds__(kBlock) void k_search_reroot(DevModel m, SearchArgs sa, int a,
                                                          int z) {
  extern __shared__ float smem[];
  __shared__ float s_stay[256];
  __shared__ float s_red[4 * 32];
  __shared__ int s_found;
  const int tid = threadIdx.x, A = m.A;
  const int r = sa.ctl[kCtlRoot];
  if (tid == 0) {
    s_found = -1;
    sa.ctl[kCtlErr] = 0;
    if (sa.expanded[r]) {
      for (int i = 0; i < sa.n; ++i) {
        const int c = sa.cbase[r] + a * sa.n + i;
        if (sa.valid[c] && sa.z[c] == z) s_found = c;
      }
    }
    if (s_found >= 0) {
      sa.parent[s_found] = -1;
      sa.ctl[kCtlRoot] = s_found;
      sa.ctl[kCtlSelect] = sa.E[s_found];
      sa.ctl[kCtlFlags] = 0;
    }
  }
  __syncthreads();
  if (s_found >= 0) return;
  const int c = sa.ctl[kCtlNext];
  if (c + 1 > sa.NV) {
    if (tid == 0) sa.ctl[kCtlErr] = 2;
    return;
  }
  const int W = m.W, H = m.H, S = m.S, BW = W + 2;
  float *band = smem;
  float *bpl = band + (size_t)(H + 2) * BW;
  const float *b = sa.bel + (size_t)r * S;
  s_stay[tid] = sa.staytab[a * 256 + tid];
  load_band(m, sa.sig, b, 0, H, band, BW, false);
  __syncthreads();
  const float rW = 1.0f / (float)W;
  const float *sl = &m.slip[a * 9];
  const float bgoal = m.goal >= 0 ? b[m.goal] : 0.f;
  const uint32_t zw = (uint32_t)(z & 15), zl = (uint32_t)(z >> 4);
  float p = 0.f;
  for (int t = tid; t < S; t += kBlock) {
    const uint32_t sg = sa.sig[t];
    const int ly = fdiv(t, W, rW), lx = t - ly * W;
    const float bt = t == m.goal ? bgoal : band[(ly + 1) * BW + lx + 1];
    const float bp = predict_cell_v(band, BW, ly, lx, sg, sl, s_stay, bt);
    bpl[t] = bp;
    p = fmaf(wall_lik(m.flip, zw, sig_wall(sg)) * lm_lik(m.lm_p, zl, sig_lm(sg)), bp, p);
  }
  p = wave_sum(p);
  if ((tid & (kWave - 1)) == 0) s_red[tid / kWave] = p;
  __syncthreads();
  const float P = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
  __syncthreads();
  if (!(P > 0.f)) {
    if (tid == 0) sa.ctl[kCtlErr] = 1;
    return;
  }
  float U, L;
  search_bounds(m, sa, bpl, z, 1.0f / P, sa.bel + (size_t)c * S, s_red, U, L);
  if (tid == 0) {
    search_new_node(sa, c, -1, 1.f, z, sa.depth[r] + 1, U, L);
    sa.pz[c] = P;
    sa.count[c] = 0;
    sa.ctl[kCtlRoot] = c;
    sa.ctl[kCtlSelect] = c;
    sa.ctl[kCtlNext] = c + 1;
    sa.ctl[kCtlFlags] = 0;
  }
  (void)A;
}

hipError_t launch_search(int what, const DevModel &m, const SearchArgs &sa, const float *b0,
                         int a, int z, int32_t *action, float *rootU, float *rootL,
                         hipStream_t st) {
  const size_t lds = search_lds_floats(m.W, m.H) * sizeof(float);
  static bool attr = false;
  if (!attr) {
    const void *ks[3] = {(const void *)k_search_init, (const void *)k_search_expand,
                         (const void *)k_search_reroot};
    for (const void *f : ks) {
      hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)(160 * 1024 - 8 * 1024));
      if (e != hipSuccess) return e;
    }
    attr = true;
  }
  switch (what) {
    case 0:
      QV_LAUNCH(k_search_init, dim3(1), dim3(kBlock), lds, st, m, sa, b0);
      break;
    case 1:
      QV_LAUNCH(k_search_expand, dim3(m.A), dim3(kBlock), lds, st, m, sa);
      QV_LAUNCH(k_search_child, dim3(m.A * sa.n), dim3(kSearchChildBlock), 0, st, m, sa);
      QV_LAUNCH(k_search_update, dim3(1), dim3(kWave), 0, st, m, sa);
      break;
    case 2:
      QV_LAUNCH(k_search_result, dim3(1), dim3(kWave), 0, st, m, sa, action, rootU, rootL);
      break;
    case 3:
      QV_LAUNCH(k_search_reroot, dim3(1), dim3(kBlock), lds, st, m, sa, a, z);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace qv

namespace qv {

// ===========================================================================
// Point-based value iteration (Sec. IV-B).  The state lives in the workspace:
// a set of belief points, each with its predictions b' = T_a^T b, and the
// vector set Gamma as a table [S][ld] (one column per vector, the layout of a
// bound table).  Two vector tables alternate between backups.
//   expansion (the paper follows Pineau et al.): every point draws one
//     observation per action (sample_draws with n = 1, counter (a, point,
//     64 + round, query)), forms the posterior, and the posterior farthest in
//     L1 from the current set joins it (first maximum over actions, not at
//     distance 0), in point order while there is room;
//   backup (the PBVI Bellman equation): per (point, action) and observation
//     z, the vector j maximising sum_x O(z|x) b'(x) alpha_j(x) (first maximum);
//     alpha_a(x) = R(x,a) + gamma sum_x' T(x,a,x') G(x') with
//     G(y) = sum_z O(z|y) alpha_{a,z}(y) on free cells (0 on blocked ones);
//     the point's new vector is the alpha_a of largest b.alpha_a.
// The observations z = zw + 16 zl factor: O(z|x) = O_w(zw|w(x)) O_l(zl|x),
// so the value of vector j at z with zl = 0 is sum_w O_w(zw|w) HW[w][j] with
// HW[w][j] = sum over cells of true wall reading w of lambda(x) b'(x)
// alpha_j(x) (lambda = 1 - rho on landmark cells, else 1); at zl = l >= 1 only
// landmark l's cell counts.
// ===========================================================================
__global__ void k_pbvi_init(DevModel m, PbviArgs pa, const float *b0, const float *init,
                            int init_cols) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = (long long)m.S * init_cols;
  if (i < m.S) pa.pts[i] = (pa.sig[i] & kSigFree) ? b0[i] : 0.f;
  if (i < n) {
    const long long x = i / init_cols;
    const int j = (int)(i - x * init_cols);
    pa.G0[x * pa.ld + j] = init[i];
  }
  if (i == 0) {
    pa.ctl[kPbviCtlPoints] = 1;
    pa.ctl[kPbviCtlRound] = 0;
    pa.ctl[kPbviCtlCur] = 0;
    pa.ctl[kPbviCtlCols] = init_cols;
    pa.ctl[kPbviCtlAdded] = 0;
  }
}

// Points p0 .. p0 + gridDim.x / A - 1, one workgroup per (point, action).
// !EXPAND: the prediction b' into pred.  EXPAND: b', the draw of one
// observation and the posterior into cand (pred is not rewritten).
template <bool EXPAND>
__global__ __launch_bounds__(kBlock) void k_pbvi_predict(DevModel m, PbviArgs pa, int p0,
                                                         int round) {
  extern __shared__ float smem[];
  __shared__ float s_stay[256];
  __shared__ float s_H[17];
  __shared__ DrawOut s_draw;
  const int A = m.A, W = m.W, H = m.H, S = m.S, BW = W + 2, tid = threadIdx.x;
  const int b = p0 + blockIdx.x / A, a = blockIdx.x % A;
  float *band = smem;
  float *bpl = band + (size_t)(H + 2) * BW;
  float *hist = bpl + ((S + 3) & ~3);
  const float *bb = pa.pts + (size_t)b * S;
  s_stay[tid] = pa.staytab[a * 256 + tid];
  load_band(m, pa.sig, bb, 0, H, band, BW, false);
  if (EXPAND) {
#pragma unroll
    for (int w = 1; w < 16; ++w) hist[w * kBlock + tid] = 0.f;
  }
  __syncthreads();
  const float rW = 1.0f / (float)W;
  const float *sl = &m.slip[a * 9];
  const float rho = m.lm_p;
  const float bgoal = m.goal >= 0 ? bb[m.goal] : 0.f;
  float *out = pa.pred + ((size_t)b * A + a) * S;
  float h0 = 0.f;
  for (int t = tid; t < S; t += kBlock) {
    const uint32_t sg = pa.sig[t];
    const int ly = fdiv(t, W, rW), lx = t - ly * W;
    const float bt = t == m.goal ? bgoal : band[(ly + 1) * BW + lx + 1];
    const float bp = predict_cell_v(band, BW, ly, lx, sg, sl, s_stay, bt);
    if (!EXPAND) {
      out[t] = bp;
    } else {
      bpl[t] = bp;
      const uint32_t lm = sig_lm(sg);
      const float contrib = (lm && lm <= (uint32_t)m.L) ? bp * (1.f - rho) : bp;
      const uint32_t w = sig_wall(sg);
      if (w == 0u)
        h0 += contrib;
      else
        hist[w * kBlock + tid] += contrib;
    }
  }
  if (!EXPAND) return;
  hist[tid] = h0;
  __syncthreads();
  {
    const int k = tid & 15, rot = (tid >> 4) & 3;
    const float *hb = hist + (tid >> 4) * kBlock;
    float sum = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) sum += hb[k + 16 * ((i + rot) & 15)];
    sum = group_sum<16>(sum);
    if ((tid & 15) == 15) s_H[tid >> 4] = sum;
    if (tid == 0) s_H[16] = 0.f;
  }
  __syncthreads();
  if (tid < kWave) {
    LevelArgs lv{};
    lv.d = 64 + round;
    lv.n = 1;
    lv.K = A;
    lv.key0 = pa.key0;
    lv.key1 = pa.key1;
    lv.qid = pa.qid;
    lv.cvalid = pa.dvalid;
    lv.cz = pa.dz;
    lv.ccount = pa.dcount;
    lv.cpz = pa.dpz;
    uint32_t *lw = (uint32_t *)hist;
    float *lvv = hist + m.L;
    for (int l = tid; l < m.L; l += kWave) {
      lw[l] = pa.lm_wall[l];
      const int c = m.lm_cell[l];
      lvv[l] = (c >= 0 && c < S) ? bpl[c] : 0.f;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    sample_draws(m, lv, b, a, tid < 17 ? s_H[tid] : 0.f, lw, lvv, hist + 2 * m.L, &s_draw,
                 b * A);
  }
  __syncthreads();
  if (s_draw.U < 1) return;
  const int z = s_draw.z[0];
  const float inv = s_draw.inv[0];
  const uint32_t zw = (uint32_t)(z & 15), zl = (uint32_t)(z >> 4);
  float *c = pa.cand + ((size_t)b * A + a) * S;
  for (int t = tid; t < S; t += kBlock) {
    const uint32_t sg = pa.sig[t];
    c[t] = wall_lik(m.flip, zw, sig_wall(sg)) * lm_lik(rho, zl, sig_lm(sg)) * bpl[t] * inv;
  }
}

// L1 distance of each drawn posterior to the nearest point of the set
// (points 0 .. np-1); -1 where no observation was drawn.
__global__ __launch_bounds__(kBlock) void k_pbvi_dist(DevModel m, PbviArgs pa, int np) {
  __shared__ float s_red[kBlock / kWave];
  const int A = m.A, S = m.S, tid = threadIdx.x;
  const int b = blockIdx.x / A, a = blockIdx.x % A;
  if (!pa.dvalid[b * A + a]) {
    if (tid == 0) pa.dist[b * A + a] = -1.f;
    return;
  }
  const float *c = pa.cand + ((size_t)b * A + a) * S;
  float best = INFINITY;
  for (int j = 0; j < np; ++j) {
    const float *q = pa.pts + (size_t)j * S;
    float d = 0.f;
    for (int t = tid; t < S; t += kBlock) d += fabsf(c[t] - q[t]);
    d = wave_sum(d);
    if ((tid & (kWave - 1)) == 0) s_red[tid / kWave] = d;
    __syncthreads();
    best = fminf(best, (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]));
    __syncthreads();
  }
  if (tid == 0) pa.dist[b * A + a] = best;
}

// Each point's farthest posterior (first maximum over actions, distance > 0)
// joins the set, in point order, while there is room; one thread.
__global__ void k_pbvi_add(DevModel m, PbviArgs pa, int np) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int added = 0;
  for (int b = 0; b < np; ++b) {
    int best = -1;
    float bd = 0.f;
    for (int a = 0; a < m.A; ++a) {
      const float d = pa.dist[b * m.A + a];
      if (d > bd) {
        bd = d;
        best = a;
      }
    }
    if (best >= 0 && np + added < pa.np_max) pa.src[added++] = b * m.A + best;
  }
  pa.ctl[kPbviCtlAdded] = added;
  pa.ctl[kPbviCtlPoints] = np + added;
  pa.ctl[kPbviCtlRound] += 1;
}

__global__ void k_pbvi_copy(DevModel m, PbviArgs pa, int np) {
  const int i = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pa.ctl[kPbviCtlAdded] || t >= m.S) return;
  pa.pts[(size_t)(np + i) * m.S + t] = pa.cand[(size_t)pa.src[i] * m.S + t];
}

// First maximum of (value, column) over the workgroup: the largest value,
// the lowest column among equal values; every thread gets the column.
__device__ __forceinline__ int pbvi_block_argmax(float v, int j, float *rv, int *rj) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(v, o, kWave);
    const int oj = __shfl_xor(j, o, kWave);
    if (ov > v || (ov == v && oj < j)) {
      v = ov;
      j = oj;
    }
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) {
    rv[wave] = v;
    rj[wave] = j;
  }
  __syncthreads();
  float bv = rv[0];
  int bj = rj[0];
  for (int w = 1; w < kBlock / kWave; ++w)
    if (rv[w] > bv || (rv[w] == bv && rj[w] < bj)) {
      bv = rv[w];
      bj = rj[w];
    }
  __syncthreads();
  return bj;
}

// Slices of cells that the workgroup's threads split for `cols` columns.
__host__ __device__ inline int pbvi_slices(int cols) {
  int cp = 1;
  while (cp < cols) cp <<= 1;
  return cp >= kBlock ? 1 : kBlock / cp;
}

// Per (point, action): HW[w][j] (cells split into slices, each summed in
// cell order, the slices then added in order), then the chosen vector of
// every observation into idx.
__global__ __launch_bounds__(kBlock) void k_pbvi_select(DevModel m, PbviArgs pa, const float *G,
                                                        int gcols) {
  extern __shared__ float smem[];   // [SL][16][gcols] slice sums
  __shared__ float rv[kBlock / kWave];
  __shared__ int rj[kBlock / kWave];
  __shared__ float ctab[256];       // O_w(zw | w) at [zw * 16 + w]
  const int A = m.A, S = m.S, tid = threadIdx.x, ld = pa.ld;
  const int b = blockIdx.x / A, a = blockIdx.x % A;
  const float *bp = pa.pred + ((size_t)b * A + a) * S;
  const int SL = pbvi_slices(gcols);
  const int CW = kBlock / SL;
  ctab[tid] = wall_lik(m.flip, (uint32_t)(tid >> 4), (uint32_t)(tid & 15));
  const float rho = m.lm_p;
  const int slice = tid / CW, jl = tid - slice * CW;
  const int c0 = (int)(((long long)S * slice) / SL), c1 = (int)(((long long)S * (slice + 1)) / SL);
  for (int j0 = 0; j0 < gcols; j0 += CW) {
    const int j = j0 + jl;
    const int jc = j < gcols ? j : 0;
    float h[16];
#pragma unroll
    for (int w = 0; w < 16; ++w) h[w] = 0.f;
    constexpr int NB = 8;
    for (int t0 = c0; t0 < c1; t0 += NB) {
      float v[NB], g[NB];
      uint32_t sg[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const bool in = t0 + k < c1;
        const int t = in ? t0 + k : c0;
        v[k] = in ? bp[t] : 0.f;
        sg[k] = pa.sig[t];
        g[k] = G[(size_t)t * ld + jc];
      }
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const uint32_t lm = sig_lm(sg[k]);
        const float x = ((lm && lm <= (uint32_t)m.L) ? v[k] * (1.f - rho) : v[k]) * g[k];
        const uint32_t w = sig_wall(sg[k]);
#pragma unroll
        for (int q = 0; q < 16; ++q) h[q] += (w == (uint32_t)q) ? x : 0.f;
      }
    }
    if (j < gcols) {
#pragma unroll
      for (int w = 0; w < 16; ++w) smem[((size_t)slice * 16 + w) * gcols + j] = h[w];
    }
  }
  __syncthreads();
  for (int i = tid; i < 16 * gcols; i += kBlock) {
    float s = smem[i];
    for (int q = 1; q < SL; ++q) s += smem[(size_t)q * 16 * gcols + i];
    smem[i] = s;
  }
  __syncthreads();
  int32_t *idx = pa.idx + ((size_t)b * A + a) * pa.ZC;
  for (int zw = 0; zw < 16; ++zw) {
    float best = -INFINITY;
    int bj = 0x7fffffff;
    for (int j = tid; j < gcols; j += kBlock) {
      float v = 0.f;
#pragma unroll
      for (int w = 0; w < 16; ++w) v = fmaf(ctab[zw * 16 + w], smem[w * gcols + j], v);
      if (v > best) {
        best = v;
        bj = j;
      }
    }
    const int r = pbvi_block_argmax(best, bj, rv, rj);
    if (tid == 0) idx[zw] = r;
  }
  // zl = l: the value of vector j is O_w(zw | w_l) rho b'(x_l) alpha_j(x_l):
  // the largest alpha_j(x_l) when that factor is positive, else all are 0
  // and the first vector is taken
  for (int l = 0; l < m.L; ++l) {
    const int cell = m.lm_cell[l];
    const bool on = cell >= 0 && cell < S;
    const float coef = on ? rho * bp[cell] : 0.f;
    int r = 0;
    if (coef > 0.f) {
      float best = -INFINITY;
      int bj = 0x7fffffff;
      for (int j = tid; j < gcols; j += kBlock) {
        const float v = G[(size_t)cell * ld + j];
        if (v > best) {
          best = v;
          bj = j;
        }
      }
      r = pbvi_block_argmax(best, bj, rv, rj);
    }
    if (tid < 16) {
      const uint32_t wl = pa.lm_wall[l];
      const bool pos = coef > 0.f && wl <= 15u && ctab[tid * 16 + wl] > 0.f;
      idx[16 * (l + 1) + tid] = pos ? r : 0;
    }
  }
}

// Per (point, action): alpha_a into cand and b.alpha_a into vals.
__global__ __launch_bounds__(kBlock) void k_pbvi_backup(DevModel m, PbviArgs pa, const float *G) {
  extern __shared__ float smem[];   // G(y) on a band with a zero halo, then idx
  __shared__ float s_stay[256];
  __shared__ float ctab[256];
  __shared__ float s_red[kBlock / kWave];
  const int A = m.A, W = m.W, H = m.H, S = m.S, BW = W + 2, tid = threadIdx.x, ld = pa.ld;
  const int b = blockIdx.x / A, a = blockIdx.x % A;
  float *band = smem;
  int *sidx = (int *)(smem + (size_t)(H + 2) * BW);
  const int32_t *idx = pa.idx + ((size_t)b * A + a) * pa.ZC;
  for (int i = tid; i < pa.ZC; i += kBlock) sidx[i] = idx[i];
  s_stay[tid] = pa.staytab[a * 256 + tid];
  ctab[tid] = wall_lik(m.flip, (uint32_t)(tid >> 4), (uint32_t)(tid & 15));
  for (int i = tid; i < (H + 2) * BW; i += kBlock) band[i] = 0.f;
  __syncthreads();
  const float rho = m.lm_p;
  const float rW = 1.0f / (float)W;
  for (int y = tid; y < S; y += kBlock) {
    const uint32_t sg = pa.sig[y];
    if (!(sg & kSigFree)) continue;
    const uint32_t w = sig_wall(sg), lm = sig_lm(sg);
    const bool isl = lm && lm <= (uint32_t)m.L;
    const float lam0 = isl ? 1.f - rho : 1.f;
    const float *gy = G + (size_t)y * ld;
    float gsum = 0.f;
    for (int zw = 0; zw < 16; ++zw) {
      const float c = ctab[zw * 16 + w];
      gsum = fmaf(c * lam0, gy[sidx[zw]], gsum);
      if (isl) gsum = fmaf(c * rho, gy[sidx[16 * lm + zw]], gsum);
    }
    const int ly = fdiv(y, W, rW), lx = y - ly * W;
    band[(ly + 1) * BW + lx + 1] = gsum;
  }
  __syncthreads();
  const float *bb = pa.pts + (size_t)b * S;
  float *out = pa.cand + ((size_t)b * A + a) * S;
  const float *sl = &m.slip[a * 9];
  float dot = 0.f;
  for (int x = tid; x < S; x += kBlock) {
    const uint32_t sg = pa.sig[x];
    float v = 0.f;
    if (sg & kSigFree) {
      const int ly = fdiv(x, W, rW), lx = x - ly * W;
      const float *c = band + (ly + 1) * BW + lx + 1;
      const float r = m.R[(size_t)x * A + a];
      float e;
      if (sg & kSigGoal) {
        e = c[0];   // the goal is absorbing
      } else {
        // the successor in direction j is x + d_j with probability slip[a][j];
        // moves into blocked or off-grid cells stay (s_stay holds slip[a][4]
        // plus their mass)
        e = sl[0] * c[-BW - 1];
        e = fmaf(sl[1], c[-BW], e);
        e = fmaf(sl[2], c[-BW + 1], e);
        e = fmaf(sl[3], c[-1], e);
        e = fmaf(sl[5], c[1], e);
        e = fmaf(sl[6], c[BW - 1], e);
        e = fmaf(sl[7], c[BW], e);
        e = fmaf(sl[8], c[BW + 1], e);
        e = fmaf(s_stay[sig_out8(sg)], c[0], e);
      }
      v = fmaf(m.gamma, e, r);
    }
    out[x] = v;
    dot = fmaf(bb[x], v, dot);
  }
  dot = wave_sum(dot);
  if ((tid & (kWave - 1)) == 0) s_red[tid / kWave] = dot;
  __syncthreads();
  if (tid == 0) pa.vals[b * A + a] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

// The point's new vector: the alpha_a of largest b.alpha_a (first maximum),
// into column b of Gout.
__global__ __launch_bounds__(kBlock) void k_pbvi_pick(DevModel m, PbviArgs pa, float *Gout) {
  __shared__ int s_a;
  const int b = blockIdx.x, A = m.A;
  if (threadIdx.x == 0) {
    int best = 0;
    for (int a = 1; a < A; ++a)
      if (pa.vals[b * A + a] > pa.vals[b * A + best]) best = a;
    s_a = best;
    pa.pick[b] = best;
  }
  __syncthreads();
  const float *c = pa.cand + ((size_t)b * A + s_a) * m.S;
  for (int x = threadIdx.x; x < m.S; x += kBlock) Gout[(size_t)x * pa.ld + b] = c[x];
}

__global__ void k_pbvi_setctl(int32_t *ctl, int cur, int cols) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl[kPbviCtlCur] = cur;
    ctl[kPbviCtlCols] = cols;
  }
}

// out[x][j] = G[x][j] for j < cols, else G[x][0]: a repeated column leaves
// the maximum over columns unchanged.
__global__ void k_pbvi_out(DevModel m, PbviArgs pa, const float *G, int cols, float *out,
                           int ldo) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)m.S * ldo) return;
  const long long x = i / ldo;
  const int j = (int)(i - x * ldo);
  out[i] = G[x * pa.ld + (j < cols ? j : 0)];
}

size_t pbvi_predict_lds_bytes(int W, int H) { return search_lds_floats(W, H) * sizeof(float); }
size_t pbvi_select_lds_bytes(int cols) {
  return (size_t)pbvi_slices(cols) * 16 * (size_t)cols * sizeof(float);
}
size_t pbvi_backup_lds_bytes(int W, int H, int ZC) {
  return ((size_t)(H + 2) * (W + 2) + (size_t)ZC) * sizeof(float);
}

// what: 0 init (b0, init, init_cols), 1 expand (np, round; the host reads
// back the count), 2 predict the points added (np = first new point,
// count), 3 one backup sweep (Gc -> Gn, cols), 4 set ctl (cur, cols),
// 5 result (Gc, cols, out, ldo).
hipError_t launch_pbvi(int what, const DevModel &m, const PbviArgs &pa, const PbviLaunch &pl,
                       hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    const void *ks[4] = {(const void *)k_pbvi_predict<true>, (const void *)k_pbvi_predict<false>,
                         (const void *)k_pbvi_select, (const void *)k_pbvi_backup};
    for (const void *f : ks) {
      hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)(152 * 1024));
      if (e != hipSuccess) return e;
    }
    attr = true;
  }
  const int A = m.A, S = m.S;
  const size_t lds_pred = pbvi_predict_lds_bytes(m.W, m.H);
  switch (what) {
    case 0: {
      const long long n = std::max((long long)S, (long long)S * pl.cols);
      QV_LAUNCH(k_pbvi_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m, pa, pl.b0,
                pl.Gc, pl.cols);
      QV_LAUNCH(k_pbvi_predict<false>, dim3(A), dim3(kBlock), lds_pred, st, m, pa, 0, 0);
      break;
    }
    case 1:
      QV_LAUNCH(k_pbvi_predict<true>, dim3(pl.np * A), dim3(kBlock), lds_pred, st, m, pa, 0,
                pl.round);
      QV_LAUNCH(k_pbvi_dist, dim3(pl.np * A), dim3(kBlock), 0, st, m, pa, pl.np);
      QV_LAUNCH(k_pbvi_add, dim3(1), dim3(kWave), 0, st, m, pa, pl.np);
      QV_LAUNCH(k_pbvi_copy, dim3((S + 255) / 256, pl.np), dim3(256), 0, st, m, pa, pl.np);
      break;
    case 2:
      QV_LAUNCH(k_pbvi_predict<false>, dim3(pl.count * A), dim3(kBlock), lds_pred, st, m, pa,
                pl.np, 0);
      break;
    case 3:
      QV_LAUNCH(k_pbvi_select, dim3(pl.np * A), dim3(kBlock), pbvi_select_lds_bytes(pl.cols), st,
                m, pa, pl.Gc, pl.cols);
      QV_LAUNCH(k_pbvi_backup, dim3(pl.np * A), dim3(kBlock),
                pbvi_backup_lds_bytes(m.W, m.H, pa.ZC), st, m, pa, pl.Gc);
      QV_LAUNCH(k_pbvi_pick, dim3(pl.np), dim3(kBlock), 0, st, m, pa, pl.Gn);
      break;
    case 4:
      QV_LAUNCH(k_pbvi_setctl, dim3(1), dim3(kWave), 0, st, pa.ctl, pl.cur, pl.cols);
      break;
    case 5: {
      const long long n = (long long)S * pl.ldo;
      QV_LAUNCH(k_pbvi_out, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m, pa, pl.Gc,
                pl.cols, pl.out, pl.ldo);
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace qv
