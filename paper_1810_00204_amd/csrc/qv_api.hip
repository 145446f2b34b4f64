// qv_api.hip -- the extern "C" entry points of libqvts: host-side checks of
// the problem statement (the tuple of Sec. II with the grid world of
// Sec. V), workspace layouts, and dispatch to the kernels.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "qv_internal.h"

namespace qv {

static thread_local int32_t g_last_hip = 0;

int32_t hip_status(hipError_t e) {
  if (e == hipSuccess) return QV_OK;
  g_last_hip = (int32_t)e;
  return QV_ERR_HIP;
}

// Cells per band of rows processed by one workgroup (whole rows).
int tile_rows(int W, int H) {
  static int target = 0;
  if (target == 0) {
    const char *e = std::getenv("QVTS_TILE_CELLS");
    int t = e ? std::atoi(e) : 0;
    target = (t >= 64 && t <= (1 << 20)) ? t : 1024;
  }
  int th = target / (W > 0 ? W : 1);
  if (th < 1) th = 1;
  if (th > H) th = H;
  return th;
}

DevModel make_dev_model(const qv_model *m) {
  DevModel d;
  std::memset(&d, 0, sizeof d);
  d.W = m->W;
  d.H = m->H;
  d.S = m->W * m->H;
  d.A = m->A;
  d.L = m->L;
  d.goal = m->goal;
  d.gamma = m->gamma;
  d.lm_p = m->lm_p;
  for (int i = 0; i < 9 * m->A; ++i) d.slip[i] = m->slip[i];
  for (int j = 0; j < 4; ++j) d.flip[j] = m->flip[j];
  d.occ = m->occ;
  d.lm_cell = m->lm_cell;
  d.R = m->R;
  return d;
}

int32_t check_model(const qv_model *m) {
  if (!m) return QV_ERR_INVALID_ARG;
  if (m->W < 1 || m->H < 1 || m->W > QV_MAX_SIDE || m->H > QV_MAX_SIDE) return QV_ERR_INVALID_ARG;
  if (m->A < 1 || m->A > QV_MAX_ACTIONS) return QV_ERR_INVALID_ARG;
  if (m->L < 0 || m->L > QV_MAX_LANDMARKS) return QV_ERR_INVALID_ARG;
  if (!m->occ || !m->R || (m->L > 0 && !m->lm_cell)) return QV_ERR_INVALID_ARG;
  const long long S = (long long)m->W * m->H;
  if (m->goal < -1 || m->goal >= S) return QV_ERR_INVALID_ARG;
  if (!(m->gamma > 0.f && m->gamma < 1.f)) return QV_ERR_INVALID_ARG;
  if (!(m->lm_p >= 0.f && m->lm_p <= 1.f)) return QV_ERR_INVALID_ARG;
  for (int j = 0; j < 4; ++j)
    if (!(m->flip[j] >= 0.f && m->flip[j] <= 1.f)) return QV_ERR_INVALID_ARG;
  for (int a = 0; a < m->A; ++a) {
    double s = 0.0;
    for (int k = 0; k < 9; ++k) {
      const float v = m->slip[a * 9 + k];
      if (!(v >= 0.f) || !std::isfinite(v)) return QV_ERR_NOT_STOCHASTIC;
      s += v;
    }
    if (std::fabs(s - 1.0) > 1e-5) return QV_ERR_NOT_STOCHASTIC;
  }
  return QV_OK;
}

bool ws_ok(const void *ws, size_t have, size_t need) {
  if (need == 0) return true;
  return ws && have >= need && ((uintptr_t)ws % QV_WORKSPACE_ALIGN) == 0;
}

// Workspace of a planning query.  Returns false when the tree does not fit
// this build's index ranges.
bool plan_layout_impl(const qv_model *m, int D, int n, int flags, PlanLayout *L, int th) {
  std::memset(L, 0, sizeof *L);
  qv_tree_layout &T = L->pub;
  const long long S = (long long)m->W * m->H;
  const int A = m->A, K = A * n;
  T.D = D;
  T.n = n;
  T.K = K;
  T.A = A;
  T.S = (int32_t)S;
  T.tile_rows = th > 0 ? std::min(th, m->H) : tile_rows(m->W, m->H);
  T.tiles = (m->H + T.tile_rows - 1) / T.tile_rows;
  long long tot = 0, lv = 1;
  for (int d = 0; d <= D; ++d) {
    T.level_slots[d] = lv;
    T.level_first[d] = tot;
    tot += lv;
    if (d < D) {
      lv *= K;
      if (lv > (1LL << 26)) return false;
    }
  }
  T.level_first[D + 1] = tot;
  if (T.level_slots[D] * T.tiles >= (1LL << 31)) return false;
  if (D > 0 && T.level_slots[D - 1] * T.tiles * A >= (1LL << 31)) return false;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes, 256);
    return o;
  };
  L->sig = take((size_t)S * 4);
  L->staytab = take((size_t)A * 256 * 4);
  T.valid = take((size_t)tot * 4);
  T.z = take((size_t)tot * 4);
  T.count = take((size_t)tot * 4);
  T.pz = take((size_t)tot * 4);
  T.value = take((size_t)tot * 4);
  T.qvalue = take((size_t)tot * A * 4);
  T.reward = take((size_t)tot * A * 4);
  const bool store = (flags & QV_PLAN_STORE_LEAVES) != 0;
  for (int d = 1; d <= D; ++d)
    if (d < D || store) T.belief_offset[d] = take((size_t)T.level_slots[d] * S * 4);
  long long ps = 1;
  for (int d = 0; d < D; ++d) ps = std::max<long long>(ps, T.level_slots[d]);
  L->part_slots = (size_t)ps;
  L->part = take((size_t)ps * A * T.tiles * 17 * 4);
  L->lmv = take((size_t)ps * A * (m->L > 0 ? m->L : 1) * 4);
  L->leafpart = take((size_t)T.level_slots[D] * T.tiles * A * 4);
  L->stats_ctr_len = (size_t)ps * A;
  L->node_ctr_len = (size_t)tot;
  L->counters = take((L->stats_ctr_len + L->node_ctr_len + 2 * (QV_MAX_DEPTH + 1)) * 4);
  long long list_len = 1;
  for (int d = 1; d < D; ++d) list_len += T.level_slots[d];
  L->slot_list = take((size_t)list_len * 4);
  L->lm_wall = take((size_t)(m->L > 0 ? m->L : 1) * 4);
  // the last level runs one workgroup per (parent, band of about 8192 cells)
  L->leaf_rows = std::max(1, std::min(m->H, 8192 / m->W));
  L->leaf_tiles = (m->H + L->leaf_rows - 1) / L->leaf_rows;
  L->sort_cells = take((size_t)S * 4);
  L->sort_chunk = take((size_t)L->leaf_tiles * kSortChunkInts * 4);
  if (D > 0 && A <= 8 && L->leaf_tiles > 1) {
    // band records sized for histograms of 8 actions, the widest a kernel
    // uses for A <= 8 (a batch may pad a 4-action query to 8)
    const size_t recn = (size_t)8 * 16 * 9 + 8;
    L->leafrec = take((size_t)T.level_slots[D - 1] * L->leaf_tiles * recn * 4);
  }
  L->err = take(256);
  T.total_bytes = off;
  return true;
}

}  // namespace qv

using namespace qv;

extern "C" {

const char *qv_status_string(int32_t s) {
  switch (s) {
    case QV_OK: return "ok";
    case QV_ERR_INVALID_ARG: return "invalid argument";
    case QV_ERR_NOT_STOCHASTIC: return "slip row is not a probability distribution";
    case QV_ERR_BELIEF_INVALID: return "belief is not a distribution over free cells";
    case QV_ERR_ZERO_LIKELIHOOD: return "observation has zero likelihood";
    case QV_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case QV_ERR_HIP: return "HIP runtime error";
    case QV_ERR_UNSUPPORTED: return "request outside the limits of this build";
    default: return "unknown status";
  }
}

int32_t qv_last_hip_error(void) { return g_last_hip; }

size_t qv_belief_update_workspace_bytes(const qv_model *m, int32_t batch) {
  if (check_model(m) != QV_OK || batch < 0) return 0;
  return belief_update_ws(m, batch);
}

int32_t qv_belief_update(const qv_model *m, int32_t batch, const float *b, const int32_t *a,
                         const int32_t *z, float *b_out, float *p_out, int32_t check, void *ws,
                         size_t ws_bytes, void *stream) {
  const int32_t st = belief_update_args(m, batch, b, a, z, b_out, p_out);
  if (st != QV_OK) return st;
  if (!ws_ok(ws, ws_bytes, belief_update_ws(m, batch))) return QV_ERR_WORKSPACE;
  return belief_update_run(m, batch, b, a, z, b_out, p_out, check, (char *)ws,
                           (hipStream_t)stream);
}

size_t qv_vi_workspace_bytes(const qv_model *m, int32_t max_sweeps) {
  if (check_model(m) != QV_OK || max_sweeps < 1) return 0;
  return vi_ws(m, max_sweeps);
}

int32_t qv_value_iterate(const qv_model *m, float tol, int32_t max_sweeps, float *Q,
                         double *residual_out, int32_t *sweeps_out, void *ws, size_t ws_bytes,
                         void *stream) {
  int32_t st = check_model(m);
  if (st != QV_OK) return st;
  if (max_sweeps < 1 || !(tol >= 0.f) || !Q || !residual_out || !sweeps_out)
    return QV_ERR_INVALID_ARG;
  if (!ws_ok(ws, ws_bytes, vi_ws(m, max_sweeps))) return QV_ERR_WORKSPACE;
  const DevModel dm = make_dev_model(m);
  double r = 0.0;
  int k = 0;
  st = hip_status(run_value_iteration(dm, tol, max_sweeps, Q, &r, &k, (char *)ws,
                                      (hipStream_t)stream));
  if (st != QV_OK) return st;
  *residual_out = r;
  *sweeps_out = k;
  return QV_OK;
}

size_t qv_check_workspace_bytes(void) { return 256; }

int32_t qv_model_check(const qv_model *m, const float *b0, void *ws, size_t ws_bytes,
                       void *stream) {
  int32_t st = check_model(m);
  if (st != QV_OK) return st;
  if (!ws_ok(ws, ws_bytes, qv_check_workspace_bytes())) return QV_ERR_WORKSPACE;
  return run_model_check(make_dev_model(m), b0, true, (char *)ws, (hipStream_t)stream);
}

size_t qv_fib_workspace_bytes(const qv_model *m, int32_t max_sweeps) {
  if (check_model(m) != QV_OK || max_sweeps < 1) return 0;
  return fib_ws(m, max_sweeps);
}

int32_t qv_fib_iterate(const qv_model *m, float tol, int32_t max_sweeps, float *alpha,
                       double *residual_out, int32_t *sweeps_out, void *ws, size_t ws_bytes,
                       void *stream) {
  int32_t st = check_model(m);
  if (st != QV_OK) return st;
  if (max_sweeps < 1 || !(tol >= 0.f) || !alpha || !residual_out || !sweeps_out)
    return QV_ERR_INVALID_ARG;
  if (!ws_ok(ws, ws_bytes, fib_ws(m, max_sweeps))) return QV_ERR_WORKSPACE;
  const DevModel dm = make_dev_model(m);
  double r = 0.0;
  int k = 0;
  st = hip_status(run_fib(dm, tol, max_sweeps, alpha, &r, &k, (char *)ws, (hipStream_t)stream));
  if (st != QV_OK) return st;
  *residual_out = r;
  *sweeps_out = k;
  return QV_OK;
}

size_t qv_blind_workspace_bytes(const qv_model *m, int32_t max_sweeps) {
  return qv_fib_workspace_bytes(m, max_sweeps);
}

int32_t qv_blind_iterate(const qv_model *m, float tol, int32_t max_sweeps, float *alpha,
                         double *residual_out, int32_t *sweeps_out, void *ws, size_t ws_bytes,
                         void *stream) {
  int32_t st = check_model(m);
  if (st != QV_OK) return st;
  if (max_sweeps < 1 || !(tol >= 0.f) || !alpha || !residual_out || !sweeps_out)
    return QV_ERR_INVALID_ARG;
  if (!ws_ok(ws, ws_bytes, fib_ws(m, max_sweeps))) return QV_ERR_WORKSPACE;
  const DevModel dm = make_dev_model(m);
  double r = 0.0;
  int k = 0;
  st = hip_status(run_fib(dm, tol, max_sweeps, alpha, &r, &k, (char *)ws, (hipStream_t)stream, 1));
  if (st != QV_OK) return st;
  *residual_out = r;
  *sweeps_out = k;
  return QV_OK;
}

size_t qv_plan_workspace_bytes(const qv_model *m, int32_t D, int32_t n, int32_t flags) {
  if (check_model(m) != QV_OK || D < 0 || D > QV_MAX_DEPTH || n < 1 || n > QV_MAX_SAMPLES)
    return 0;
  PlanLayout L;
  if (!plan_layout_impl(m, D, n, flags, &L)) return 0;
  return L.pub.total_bytes;
}

int32_t qv_plan_layout(const qv_model *m, int32_t D, int32_t n, int32_t flags,
                       qv_tree_layout *out) {
  int32_t st = check_model(m);
  if (st != QV_OK) return st;
  if (!out || D < 0 || D > QV_MAX_DEPTH || n < 1 || n > QV_MAX_SAMPLES)
    return QV_ERR_INVALID_ARG;
  PlanLayout L;
  if (!plan_layout_impl(m, D, n, flags, &L)) return QV_ERR_UNSUPPORTED;
  *out = L.pub;
  return QV_OK;
}

int32_t qv_plan_step(const qv_model *m, const float *Q, const float *b0, int32_t D, int32_t n,
                     uint64_t seed, uint32_t query_id, int32_t flags, int32_t *action_out,
                     float *rootQ_out, void *ws, size_t ws_bytes, void *stream) {
  int32_t st = check_model(m);
  if (st != QV_OK) return st;
  if (D < 0 || D > QV_MAX_DEPTH || n < 1 || n > QV_MAX_SAMPLES) return QV_ERR_INVALID_ARG;
  if (!Q || !b0 || !action_out || !rootQ_out) return QV_ERR_INVALID_ARG;
  if (flags & ~(QV_PLAN_STORE_LEAVES | QV_PLAN_TILED | QV_PLAN_CHECK)) return QV_ERR_INVALID_ARG;
  PlanLayout L;
  if (!plan_layout_impl(m, D, n, flags, &L)) return QV_ERR_UNSUPPORTED;
  if (!ws_ok(ws, ws_bytes, L.pub.total_bytes)) return QV_ERR_WORKSPACE;
  if (flags & QV_PLAN_CHECK) {
    // b0 in B(X) (Sec. II), checked on the device before anything is planned
    st = run_model_check(make_dev_model(m), b0, false, (char *)ws + L.err, (hipStream_t)stream);
    if (st != QV_OK) return st;
  }
  return hip_status(launch_plan(m, Q, b0, D, n, seed, query_id, flags, action_out, rootQ_out,
                                (char *)ws, L, (hipStream_t)stream));
}

size_t qv_filter_workspace_bytes(const qv_model *m, int32_t ntraj, int32_t T,
                                 int32_t ckpt_every) {
  if (check_model(m) != QV_OK || ntraj < 0 || T < 1 || ckpt_every < 1 || !filter_supported(m))
    return 0;
  return filter_ws(m, ntraj, T, std::min(ckpt_every, T), filter_groups(ntraj));
}

int32_t qv_filter_nll_grad(const qv_model *m, const float *theta, const float *phi,
                           int32_t ntraj, int32_t T, const float *b0, int32_t b0_per_traj,
                           const int32_t *acts, const int32_t *obs, int32_t ckpt_every,
                           float *nll_out, float *g_slip, float *g_flip, int32_t check,
                           void *ws, size_t ws_bytes, void *stream) {
  int32_t st = check_model(m);
  if (st != QV_OK) return st;
  if (ntraj < 0 || T < 1 || ckpt_every < 1) return QV_ERR_INVALID_ARG;
  if (!theta || !phi || !b0) return QV_ERR_INVALID_ARG;
  if (ntraj > 0 && (!acts || !obs || !nll_out)) return QV_ERR_INVALID_ARG;
  if ((g_slip == nullptr) != (g_flip == nullptr)) return QV_ERR_INVALID_ARG;
  if (!filter_supported(m)) return QV_ERR_UNSUPPORTED;
  const int k = std::min(ckpt_every, T);
  const int G = filter_groups(ntraj);
  const size_t need = filter_ws(m, ntraj, T, k, G);
  if (!ws_ok(ws, ws_bytes, need)) return QV_ERR_WORKSPACE;
  hipStream_t hs = (hipStream_t)stream;
  const DevModel dm = make_dev_model(m);
  st = hip_status(launch_filter(dm, theta, phi, ntraj, T, b0, b0_per_traj, acts, obs, k, nll_out,
                                g_slip, g_flip, (char *)ws, G, hs));
  if (st != QV_OK || !check) return st;
  int32_t herr = 0;
  st = hip_status(hipMemcpyAsync(&herr, (char *)ws + need - 256, 4, hipMemcpyDeviceToHost, hs));
  if (st != QV_OK) return st;
  st = hip_status(hipStreamSynchronize(hs));
  if (st != QV_OK) return st;
  if (herr & 4) return QV_ERR_INVALID_ARG;
  if (herr & 8) return QV_ERR_ZERO_LIKELIHOOD;
  return QV_OK;
}

}  // extern "C"
