// qv_batch.hip -- batched planning.  Many independent queries, each with its
// own grid, depth and Q-MDP table, are expanded together: per tree level one
// persistent launch forms the statistics and draws of every Q-node of every
// query, and a second one writes the child beliefs (or, at a query's last
// level, scores its leaves and completes its backup).  Both take work items
// (query, parent slot, band, action) from a counter in device memory, so
// small and large queries share the chip.  The launches of a level can be
// captured once into a HIP graph and replayed; the band shape and the number
// of items taken per visit to the queue are chosen by timing candidates on
// the batch itself.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "qv_internal.h"

namespace qv {
namespace {

constexpr int kTileCandidates[] = {256, 512, 1024, 2048, 4096};
constexpr int kChunkCandidates[] = {1, 2, 4};

int band_rows(int W, int H, int tile_cells) { return std::max(1, std::min(H, tile_cells / W)); }

}  // namespace
}  // namespace qv

using namespace qv;

struct qv_batch {
  int nq = 0, n = 0, flags = 0, dmax = 0;
  // launches per level: phase 0 statistics, phase 1 children (or leaves of
  // 9-action queries), phase 2 the per-parent last level
  int apad[3] = {4, 4, 4};      // template widths of the three launches
  std::vector<qv_model> models;
  std::vector<int> D;
  int tile_cells = 0, chunk = 1;
  // layout of the current shape
  std::vector<PlanLayout> lay;
  std::vector<size_t> qoff;
  size_t desc_off = 0, call_off = 0, base_off = 0, pbase_off = 0, lbase_off = 0, sbase_off = 0,
         queue_off = 0, act_off = 0, rq_off = 0, total = 0, ws_max = 0;
  std::vector<int32_t> bases;   // [3 phases][dmax][nq+1]
  std::vector<int32_t> pbase;   // [nq+1] blocks of the prep pass
  std::vector<int32_t> lbase;   // [nq+1] blocks of the landmark pass
  std::vector<int32_t> sbase;   // [nq+1] blocks of the leaf-band sort pass
  std::vector<int> totals;      // [3][dmax] items per phase and level
  size_t lds[3] = {0, 0, 0};
  int grid[3][QV_MAX_DEPTH] = {};
  // device state
  char *bound_ws = nullptr;
  std::vector<BatchQuery> hq;
  BatchCall *call_host = nullptr;   // pinned
  hipEvent_t call_ev = nullptr;
  bool call_pending = false;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec[QV_MAX_DEPTH] = {};
  bool graphs_ready = false;
};

namespace qv {
namespace {

void drop_graphs(qv_batch *b) {
  for (auto &e : b->exec)
    if (e) {
      (void)hipGraphExecDestroy(e);
      e = nullptr;
    }
  b->graphs_ready = false;
}

// Workspace layout for bands of about tile_cells cells; false if a query's
// tree or a level's item count leaves this build's index ranges.
bool layout(qv_batch *b, int tile_cells, bool commit) {
  const int nq = b->nq;
  std::vector<PlanLayout> lay(nq);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes, 256);
    return o;
  };
  const size_t desc_off = take((size_t)nq * sizeof(BatchQuery));
  const size_t call_off = take((size_t)nq * sizeof(BatchCall));
  const size_t base_off = take((size_t)3 * b->dmax * (nq + 1) * 4);
  const size_t pbase_off = take((size_t)(nq + 1) * 4);
  const size_t lbase_off = take((size_t)(nq + 1) * 4);
  const size_t sbase_off = take((size_t)(nq + 1) * 4);
  const size_t queue_off = take((size_t)3 * QV_MAX_DEPTH * 4);
  const size_t act_off = take((size_t)nq * 4);
  const size_t rq_off = take((size_t)nq * QV_MAX_ACTIONS * 4);
  std::vector<size_t> qoff(nq);
  const size_t nb = (size_t)b->dmax * (nq + 1);
  std::vector<int32_t> bases(3 * nb, 0), pbase(nq + 1, 0), lbase(nq + 1, 0), sbase(nq + 1, 0);
  std::vector<long long> tot(3 * (size_t)b->dmax, 0);
  long long pb = 0, lb = 0, sb = 0;
  size_t lds0 = 0, lds1 = 0, lds2 = 0;
  int apad1 = 4, apad2 = 4;
  for (int q = 0; q < nq; ++q) {
    const qv_model &m = b->models[q];
    const int th = band_rows(m.W, m.H, tile_cells);
    if (!plan_layout_impl(&m, b->D[q], b->n, 0, &lay[q], th)) return false;
    qoff[q] = take(lay[q].pub.total_bytes);
    const qv_tree_layout &T = lay[q].pub;
    // the last level of a query with A <= 8 runs (parent, leaf band) items in
    // phase 2; every other level runs (parent, band, action) items in phases 0, 1
    const bool lp = m.A <= 8;
    for (int d = 0; d < b->dmax; ++d) {
      for (int ph = 0; ph < 3; ++ph) {
        bases[ph * nb + (size_t)d * (nq + 1) + q] = (int32_t)tot[ph * b->dmax + d];
        long long items = 0;
        const bool banded = d + 1 < b->D[q] || (d + 1 == b->D[q] && !lp);
        if (ph < 2 && banded)
          items = T.level_slots[d] * T.tiles * m.A;
        else if (ph == 2 && d + 1 == b->D[q] && lp)
          items = T.level_slots[d] * lay[q].leaf_tiles;
        tot[ph * b->dmax + d] += items;
        if (tot[ph * b->dmax + d] > (1LL << 30)) return false;
      }
    }
    sbase[q] = (int32_t)sb;
    if (lp) sb += lay[q].leaf_tiles;
    const long long S = (long long)m.W * m.H;
    const long long nzero = (long long)(lay[q].stats_ctr_len + lay[q].node_ctr_len);
    const long long cells = std::max<long long>(std::max<long long>(S, m.A * 256LL), nzero);
    pbase[q] = (int32_t)pb;
    lbase[q] = (int32_t)lb;
    pb += (cells + 255) / 256;
    lb += (m.L + 255) / 256;
    if (pb > (1LL << 30)) return false;
    lds0 = std::max(lds0, band_lds_bytes(m.W, th) + (size_t)16 * kBlock * 4);
    if (lp) {
      const int am = m.A <= 4 ? 4 : 8;
      apad2 = std::max(apad2, am);
    } else {
      apad1 = 16;
    }
    lds1 = std::max(lds1, leaf_lds_bytes(m.W, th, m.A * b->n, m.A));
  }
  // phase 2 runs at one histogram width for all its queries
  for (int q = 0; q < nq; ++q)
    if (b->models[q].A <= 8)
      lds2 = std::max(lds2, leaf_parent_lds_bytes(b->models[q].W, lay[q].leaf_rows,
                                                  b->models[q].L, apad2));
  for (int ph = 0; ph < 3; ++ph)
    for (int d = 0; d < b->dmax; ++d)
      bases[ph * nb + (size_t)d * (nq + 1) + nq] = (int32_t)tot[ph * b->dmax + d];
  pbase[nq] = (int32_t)pb;
  lbase[nq] = (int32_t)lb;
  sbase[nq] = (int32_t)sb;
  if (lds0 > 150 * 1024 || lds1 > 150 * 1024 || lds2 > 150 * 1024) return false;
  if (!commit) {
    b->ws_max = std::max(b->ws_max, off);
    return true;
  }
  b->lay = lay;
  b->qoff = qoff;
  b->desc_off = desc_off;
  b->call_off = call_off;
  b->base_off = base_off;
  b->pbase_off = pbase_off;
  b->lbase_off = lbase_off;
  b->sbase_off = sbase_off;
  b->queue_off = queue_off;
  b->act_off = act_off;
  b->rq_off = rq_off;
  b->total = off;
  b->bases = bases;
  b->pbase = pbase;
  b->lbase = lbase;
  b->sbase = sbase;
  b->totals.assign(3 * (size_t)b->dmax, 0);
  for (size_t i = 0; i < tot.size(); ++i) b->totals[i] = (int)tot[i];
  b->lds[0] = lds0;
  b->lds[1] = lds1;
  b->lds[2] = lds2;
  b->apad[0] = 4;
  b->apad[1] = apad1;
  b->apad[2] = apad2;
  b->tile_cells = tile_cells;
  b->bound_ws = nullptr;
  drop_graphs(b);
  return true;
}

// Persistent grid of each launch: every CU filled to its occupancy, capped
// by the number of queue visits the level needs.
bool size_grids(qv_batch *b) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return false;
  for (int ph = 0; ph < 3; ++ph) {
    const int occ = batch_level_occupancy(ph, b->apad[ph], b->lds[ph]);
    if (occ <= 0) return false;
    for (int d = 0; d < b->dmax; ++d) {
      const long long visits =
          ((long long)b->totals[ph * b->dmax + d] + b->chunk - 1) / b->chunk;
      b->grid[ph][d] = (int)std::min<long long>(visits, (long long)cus * occ);
    }
  }
  return true;
}

// Writes the device descriptors of every query for workspace ws.
int32_t bind_ws(qv_batch *b, char *ws, hipStream_t st) {
  const int nq = b->nq;
  b->hq.assign(nq, BatchQuery());
  int32_t *act = (int32_t *)(ws + b->act_off);
  float *rq = (float *)(ws + b->rq_off);
  for (int q = 0; q < nq; ++q) {
    BatchQuery &bq = b->hq[q];
    std::memset(&bq, 0, sizeof bq);
    const qv_model &mm = b->models[q];
    const PlanLayout &L = b->lay[q];
    const qv_tree_layout &T = L.pub;
    char *qb = ws + b->qoff[q];
    const int D = b->D[q], n = b->n, A = mm.A, K = A * n;
    bq.m = make_dev_model(&mm);
    bq.D = D;
    int32_t *valid = (int32_t *)(qb + T.valid);
    int32_t *zrec = (int32_t *)(qb + T.z);
    int32_t *cnt = (int32_t *)(qb + T.count);
    float *pz = (float *)(qb + T.pz);
    int32_t *ctr = (int32_t *)(qb + L.counters);
    TreeArgs &tr = bq.tr;
    tr.D = D;
    tr.n = n;
    tr.K = K;
    tr.A = A;
    tr.gamma = mm.gamma;
    for (int d = 0; d < QV_MAX_DEPTH + 2; ++d) tr.first[d] = d <= D + 1 ? T.level_first[d] : 0;
    for (int d = 0; d < QV_MAX_DEPTH + 1; ++d) tr.slots[d] = d <= D ? T.level_slots[d] : 0;
    tr.valid = valid;
    tr.count = cnt;
    tr.value = (float *)(qb + T.value);
    tr.qvalue = (float *)(qb + T.qvalue);
    tr.reward = (float *)(qb + T.reward);
    tr.node_ctr = ctr + L.stats_ctr_len;
    tr.action_out = act + q;
    tr.rootQ_out = rq + (size_t)q * QV_MAX_ACTIONS;
    bq.sig = (uint32_t *)(qb + L.sig);
    bq.staytab = (float *)(qb + L.staytab);
    bq.err = (int32_t *)(qb + L.err);
    uint32_t *lm_wall = (uint32_t *)(qb + L.lm_wall);
    bq.px = {valid, zrec, cnt, pz, ctr, (long long)(L.stats_ctr_len + L.node_ctr_len), lm_wall};
    bq.leaf_parent = A <= 8 ? 1 : 0;
    for (int d = 0; d < D; ++d) {
      LevelArgs &lv = bq.lv[d];
      lv.d = d;
      lv.nslots = (int)T.level_slots[d];
      lv.tiles = T.tiles;
      lv.TH = T.tile_rows;
      lv.n = n;
      lv.K = K;
      lv.pbel = d == 0 ? nullptr : (const float *)(qb + T.belief_offset[d]);
      lv.pvalid = valid + T.level_first[d];
      lv.part = (float *)(qb + L.part);
      lv.lmv = (float *)(qb + L.lmv);
      lv.cvalid = valid + T.level_first[d + 1];
      lv.cz = zrec + T.level_first[d + 1];
      lv.ccount = cnt + T.level_first[d + 1];
      lv.cpz = pz + T.level_first[d + 1];
      lv.reward = (float *)(qb + T.reward) + T.level_first[d] * A;
      lv.cbel = d + 1 < D ? (float *)(qb + T.belief_offset[d + 1]) : nullptr;
      lv.leafpart = (float *)(qb + L.leafpart);
      lv.sig = bq.sig;
      lv.staytab = bq.staytab;
      lv.lm_wall = lm_wall;
      lv.ctr = ctr;
      lv.sort_cells = (const int32_t *)(qb + L.sort_cells);
      lv.sort_chunk = (const int32_t *)(qb + L.sort_chunk);
      lv.slot_list = nullptr;   // the batch takes its items from a queue
      lv.slot_n = nullptr;
      lv.slot_cap = 0;
      lv.porder = nullptr;
      lv.agroups = 1;
      lv.leaf_finish = 0;   // the last band of a parent completes it
      lv.draws_apart = 0;   // the last band of a Q-node draws
      lv.own_reward = 1;    // every item forms R(b,a) of its own parent
      lv.creward = nullptr;
      if (d + 1 == D && bq.leaf_parent) {
        lv.TH = L.leaf_rows;
        lv.tiles = L.leaf_tiles;
        lv.part = (float *)(qb + L.leafrec);
      }
    }
  }
  int32_t s;
  s = hip_status(hipMemcpyAsync(ws + b->desc_off, b->hq.data(), (size_t)nq * sizeof(BatchQuery),
                                hipMemcpyHostToDevice, st));
  if (s) return s;
  s = hip_status(hipMemcpyAsync(ws + b->base_off, b->bases.data(), b->bases.size() * 4,
                                hipMemcpyHostToDevice, st));
  if (s) return s;
  s = hip_status(hipMemcpyAsync(ws + b->pbase_off, b->pbase.data(), b->pbase.size() * 4,
                                hipMemcpyHostToDevice, st));
  if (s) return s;
  s = hip_status(hipMemcpyAsync(ws + b->lbase_off, b->lbase.data(), b->lbase.size() * 4,
                                hipMemcpyHostToDevice, st));
  if (s) return s;
  s = hip_status(hipMemcpyAsync(ws + b->sbase_off, b->sbase.data(), b->sbase.size() * 4,
                                hipMemcpyHostToDevice, st));
  if (s) return s;
  s = hip_status(hipStreamSynchronize(st));
  if (s) return s;
  b->bound_ws = ws;
  drop_graphs(b);
  return QV_OK;
}

BatchPrep prep_args(const qv_batch *b, char *ws) {
  BatchPrep bp;
  bp.q = (const BatchQuery *)(ws + b->desc_off);
  bp.base = (const int32_t *)(ws + b->pbase_off);
  bp.lm_base = (const int32_t *)(ws + b->lbase_off);
  bp.sort_base = (const int32_t *)(ws + b->sbase_off);
  bp.queue = (int32_t *)(ws + b->queue_off);
  bp.nq = b->nq;
  bp.nqueue = 3 * b->dmax;
  return bp;
}

BatchLevel level_args(const qv_batch *b, char *ws, int d, int phase) {
  BatchLevel bl;
  bl.q = (const BatchQuery *)(ws + b->desc_off);
  bl.call = (const BatchCall *)(ws + b->call_off);
  bl.base = (const int32_t *)(ws + b->base_off) +
            ((size_t)phase * b->dmax + d) * (b->nq + 1);
  bl.queue = (int32_t *)(ws + b->queue_off) + 3 * d + phase;
  bl.nq = b->nq;
  bl.d = d;
  bl.total = b->totals[(size_t)phase * b->dmax + d];
  bl.chunk = b->chunk;
  return bl;
}

// The launches of level d (with the prep pass in front of level 0).
hipError_t enqueue_level(const qv_batch *b, char *ws, int d, hipStream_t st, bool timed) {
  hipError_t e;
  if (d == 0) {
    e = launch_batch_prep(prep_args(b, ws), b->pbase[b->nq], b->lbase[b->nq], b->sbase[b->nq],
                          st, timed);
    if (e != hipSuccess) return e;
  }
  for (int ph = 0; ph < 3; ++ph) {
    e = launch_batch_level(level_args(b, ws, d, ph), ph, b->apad[ph], b->lds[ph],
                           b->grid[ph][d], st, timed);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int32_t capture_graphs(qv_batch *b, char *ws) {
  if (!b->cap) {
    int32_t s = hip_status(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    if (s) return s;
  }
  drop_graphs(b);
  for (int d = 0; d < b->dmax; ++d) {
    hipGraph_t g = nullptr;
    int32_t s = hip_status(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    if (s) return s;
    const hipError_t e = enqueue_level(b, ws, d, b->cap, false);
    const hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_status(e);
    }
    if (e2 != hipSuccess) return hip_status(e2);
    s = hip_status(hipGraphInstantiate(&b->exec[d], g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    if (s) return s;
  }
  b->graphs_ready = true;
  return QV_OK;
}

int32_t set_shape(qv_batch *b, int tile_cells, int chunk) {
  if (chunk < 1 || chunk > 64 || tile_cells < 1) return QV_ERR_INVALID_ARG;
  if (!layout(b, tile_cells, true)) return QV_ERR_UNSUPPORTED;
  if (b->total > b->ws_max) return QV_ERR_UNSUPPORTED;
  b->chunk = chunk;
  if (!size_grids(b)) return QV_ERR_HIP;
  return QV_OK;
}

int32_t run(qv_batch *b, const float *const *Q, const float *const *b0, uint64_t seed,
            int32_t *actions, float *rootQ, void *ws_, size_t ws_bytes, hipStream_t st) {
  char *ws = (char *)ws_;
  if (!Q || !b0 || !actions || !rootQ) return QV_ERR_INVALID_ARG;
  if (!ws_ok(ws, ws_bytes, b->total)) return QV_ERR_WORKSPACE;
  for (int q = 0; q < b->nq; ++q)
    if (!Q[q] || !b0[q]) return QV_ERR_INVALID_ARG;
  int32_t s;
  if (ws != b->bound_ws) {
    s = bind_ws(b, ws, st);
    if (s) return s;
  }
  // per-call table: wait until the previous upload has left the pinned buffer
  if (b->call_pending) {
    s = hip_status(hipEventSynchronize(b->call_ev));
    if (s) return s;
    b->call_pending = false;
  }
  for (int q = 0; q < b->nq; ++q) {
    BatchCall &c = b->call_host[q];
    c.b0 = b0[q];
    c.Q = Q[q];
    c.key0 = (uint32_t)seed;
    c.key1 = (uint32_t)(seed >> 32);
    c.qid = (uint32_t)q;
    const int A = b->models[q].A;
    // Q rows are read (by the leaf-parent items) as float4 when they are
    // exactly as wide as the kernel's histograms
    c.q_vec = (A == 4 || A == 8) && A == b->apad[2] && ((uintptr_t)Q[q] % 16 == 0);
  }
  s = hip_status(hipMemcpyAsync(ws + b->call_off, b->call_host, (size_t)b->nq * sizeof(BatchCall),
                                hipMemcpyHostToDevice, st));
  if (s) return s;
  s = hip_status(hipEventRecord(b->call_ev, st));
  if (s) return s;
  b->call_pending = true;
  if (b->flags & QV_BATCH_GRAPH) {
    if (!b->graphs_ready) {
      s = capture_graphs(b, ws);
      if (s) return s;
    }
    for (int d = 0; d < b->dmax; ++d) {
      TimingScope ts("batch_graph", st, d);
      s = hip_status(hipGraphLaunch(b->exec[d], st));
      if (s) return s;
    }
  } else {
    for (int d = 0; d < b->dmax; ++d) {
      s = hip_status(enqueue_level(b, ws, d, st, true));
      if (s) return s;
    }
  }
  return hip_status(launch_batch_out(b->nq, (const int32_t *)(ws + b->act_off),
                                     (const float *)(ws + b->rq_off), actions, rootQ, st));
}

}  // namespace
}  // namespace qv

extern "C" {

int32_t qv_batch_create(int32_t nq, const qv_model *models, const int32_t *depths, int32_t n,
                        int32_t flags, qv_batch **out) {
  if (!out) return QV_ERR_INVALID_ARG;
  *out = nullptr;
  if (nq < 1 || !models || !depths || n < 1 || n > QV_MAX_SAMPLES) return QV_ERR_INVALID_ARG;
  if (flags & ~QV_BATCH_GRAPH) return QV_ERR_INVALID_ARG;
  for (int q = 0; q < nq; ++q) {
    const int32_t s = check_model(&models[q]);
    if (s) return s;
    if (depths[q] < 1 || depths[q] > QV_MAX_DEPTH) return QV_ERR_INVALID_ARG;
  }
  qv_batch *b = new (std::nothrow) qv_batch();
  if (!b) return QV_ERR_UNSUPPORTED;
  b->nq = nq;
  b->n = n;
  b->flags = flags;
  b->models.assign(models, models + nq);
  b->D.assign(depths, depths + nq);
  b->dmax = *std::max_element(b->D.begin(), b->D.end());
  // the workspace must hold every candidate shape
  bool any = false;
  for (int tc : kTileCandidates) any = layout(b, tc, false) || any;
  const int tdef = tile_rows(1, 1 << 30);   // the default band size in cells
  int32_t s = any ? QV_OK : QV_ERR_UNSUPPORTED;
  if (!s && !layout(b, tdef, false)) s = QV_ERR_UNSUPPORTED;
  if (!s) s = set_shape(b, tdef, 1);
  if (!s) s = hip_status(hipHostMalloc((void **)&b->call_host, (size_t)nq * sizeof(BatchCall),
                                       hipHostMallocDefault));
  if (!s) s = hip_status(hipEventCreateWithFlags(&b->call_ev, hipEventDisableTiming));
  if (s) {
    qv_batch_destroy(b);
    return s;
  }
  *out = b;
  return QV_OK;
}

int32_t qv_batch_destroy(qv_batch *b) {
  if (!b) return QV_OK;
  int32_t s = QV_OK;
  if (b->call_pending && hipEventSynchronize(b->call_ev) != hipSuccess) s = QV_ERR_HIP;
  drop_graphs(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->call_ev) (void)hipEventDestroy(b->call_ev);
  if (b->call_host) (void)hipHostFree(b->call_host);
  delete b;
  return s;
}

size_t qv_batch_workspace_bytes(const qv_batch *b) { return b ? b->ws_max : 0; }

int32_t qv_batch_set_shape(qv_batch *b, int32_t tile_cells, int32_t chunk) {
  if (!b) return QV_ERR_INVALID_ARG;
  if (b->call_pending) {
    if (hipEventSynchronize(b->call_ev) != hipSuccess) return QV_ERR_HIP;
    b->call_pending = false;
  }
  const int old_tc = b->tile_cells, old_ch = b->chunk;
  const int32_t s = set_shape(b, tile_cells, chunk);
  if (s) set_shape(b, old_tc, old_ch);
  return s;
}

int32_t qv_batch_get_shape(const qv_batch *b, int32_t *tile_cells, int32_t *chunk) {
  if (!b || !tile_cells || !chunk) return QV_ERR_INVALID_ARG;
  *tile_cells = b->tile_cells;
  *chunk = b->chunk;
  return QV_OK;
}

int32_t qv_batch_plan(qv_batch *b, const float *const *Q, const float *const *b0, uint64_t seed,
                      int32_t *actions, float *rootQ, void *ws, size_t ws_bytes, void *stream) {
  if (!b) return QV_ERR_INVALID_ARG;
  return run(b, Q, b0, seed, actions, rootQ, ws, ws_bytes, (hipStream_t)stream);
}

int32_t qv_batch_autotune(qv_batch *b, const float *const *Q, const float *const *b0,
                          uint64_t seed, int32_t *actions, float *rootQ, int32_t reps, void *ws,
                          size_t ws_bytes, void *stream, float *best_ms_out) {
  if (!b || reps < 1) return QV_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int32_t s = hip_status(hipEventCreate(&e0));
  if (!s) s = hip_status(hipEventCreate(&e1));
  float best = -1.f;
  int best_tc = b->tile_cells, best_ch = b->chunk;
  for (int tc : kTileCandidates) {
    for (int ch : kChunkCandidates) {
      if (s) break;
      if (qv_batch_set_shape(b, tc, ch) != QV_OK) continue;
      s = run(b, Q, b0, seed, actions, rootQ, ws, ws_bytes, st);   // warm-up (and capture)
      if (!s) s = hip_status(hipEventRecord(e0, st));
      for (int r = 0; r < reps && !s; ++r) s = run(b, Q, b0, seed, actions, rootQ, ws, ws_bytes, st);
      if (!s) s = hip_status(hipEventRecord(e1, st));
      if (!s) s = hip_status(hipEventSynchronize(e1));
      float ms = 0.f;
      if (!s) s = hip_status(hipEventElapsedTime(&ms, e0, e1));
      if (!s && (best < 0.f || ms < best)) {
        best = ms;
        best_tc = tc;
        best_ch = ch;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) return s;
  if (best < 0.f) return QV_ERR_UNSUPPORTED;
  s = qv_batch_set_shape(b, best_tc, best_ch);
  if (!s && best_ms_out) *best_ms_out = best / (float)reps;
  return s;
}

int32_t qv_batch_layout(const qv_batch *b, int32_t q, qv_tree_layout *out, size_t *offset_out) {
  if (!b || q < 0 || q >= b->nq || !out || !offset_out) return QV_ERR_INVALID_ARG;
  *out = b->lay[q].pub;
  *offset_out = b->qoff[q];
  return QV_OK;
}

}  // extern "C"
