// qv_search.hip -- host side of the best-first (anytime) QV-tree search
// (Alg. 1 with Alg. 2-7 and the heuristics of Sec. IV-C): workspace layout,
// argument checks and the extern "C" entry points.  The kernels are in
// qv_plan.hip, beside the level kernels whose building blocks they share.
#include <algorithm>
#include <cstring>

#include "qv_internal.h"

namespace qv {

// dynamic LDS a search kernel may take (the rest of a CU's 160 KiB holds its
// static tables)
constexpr size_t kSearchLdsMax = 152 * 1024;

static size_t search_lds_bytes(int W, int H) {
  const size_t band = (size_t)(H + 2) * (W + 2);
  const size_t S = (size_t)W * H;
  return (band + ((S + 3) & ~(size_t)3) + 16 * (size_t)kBlock) * sizeof(float);
}

static bool search_layout_impl(const qv_model *m, int n, int max_nodes, qv_search_layout *L) {
  std::memset(L, 0, sizeof *L);
  const long long S = (long long)m->W * m->H;
  const int A = m->A, K = A * n;
  if (n < 1 || n > QV_MAX_SAMPLES || max_nodes < 1 + K) return false;
  if (search_lds_bytes(m->W, m->H) > kSearchLdsMax) return false;
  if ((long long)max_nodes * S >= (1LL << 40)) return false;
  L->n = n;
  L->K = K;
  L->A = A;
  L->S = (int32_t)S;
  L->max_nodes = max_nodes;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes, 256);
    return o;
  };
  const size_t NV = (size_t)max_nodes;
  L->sig = take((size_t)S * 4);
  L->staytab = take((size_t)A * 256 * 4);
  L->lm_wall = take((size_t)(m->L > 0 ? m->L : 1) * 4);
  L->belief = take(NV * (size_t)S * 4);
  L->valid = take(NV * 4);
  L->z = take(NV * 4);
  L->count = take(NV * 4);
  L->pz = take(NV * 4);
  L->weight = take(NV * 4);
  L->parent = take(NV * 4);
  L->depth = take(NV * 4);
  L->U = take(NV * 4);
  L->L = take(NV * 4);
  L->H = take(NV * 4);
  L->E = take(NV * 4);
  L->expanded = take(NV * 4);
  L->child_base = take(NV * 4);
  L->rb = take(NV * A * 4);
  L->UQ = take(NV * A * 4);
  L->LQ = take(NV * A * 4);
  L->HQ = take(NV * A * 4);
  L->EQ = take(NV * A * 4);
  L->ctl = take(64);
  L->log = take(NV * 4);
  L->err = take(256);
  take((size_t)A * S * 4);   // predicted beliefs of the expanded node (search_bpa_offset)
  L->total_bytes = off;
  return true;
}

// The scratch of predicted beliefs b'_a that follows the error word.
static size_t search_bpa_offset(const qv_search_layout &L) { return L.err + 256; }

static SearchArgs search_args(const qv_search_layout &L, const float *Ut, const float *Lt,
                              int lcols, uint64_t seed, uint32_t qid, char *ws) {
  SearchArgs sa;
  std::memset(&sa, 0, sizeof sa);
  sa.n = L.n;
  sa.K = L.K;
  sa.NV = L.max_nodes;
  sa.key0 = (uint32_t)seed;
  sa.key1 = (uint32_t)(seed >> 32);
  sa.qid = qid;
  sa.Ut = Ut;
  sa.Lt = Lt;
  sa.lcols = lcols;
  sa.sig = (const uint32_t *)(ws + L.sig);
  sa.staytab = (const float *)(ws + L.staytab);
  sa.lm_wall = (const uint32_t *)(ws + L.lm_wall);
  sa.bel = (float *)(ws + L.belief);
  sa.valid = (int32_t *)(ws + L.valid);
  sa.z = (int32_t *)(ws + L.z);
  sa.count = (int32_t *)(ws + L.count);
  sa.parent = (int32_t *)(ws + L.parent);
  sa.depth = (int32_t *)(ws + L.depth);
  sa.E = (int32_t *)(ws + L.E);
  sa.expanded = (int32_t *)(ws + L.expanded);
  sa.cbase = (int32_t *)(ws + L.child_base);
  sa.pz = (float *)(ws + L.pz);
  sa.w = (float *)(ws + L.weight);
  sa.U = (float *)(ws + L.U);
  sa.L = (float *)(ws + L.L);
  sa.H = (float *)(ws + L.H);
  sa.rb = (float *)(ws + L.rb);
  sa.UQ = (float *)(ws + L.UQ);
  sa.LQ = (float *)(ws + L.LQ);
  sa.HQ = (float *)(ws + L.HQ);
  sa.EQ = (int32_t *)(ws + L.EQ);
  sa.ctl = (int32_t *)(ws + L.ctl);
  sa.log = (int32_t *)(ws + L.log);
  sa.bpa = (float *)(ws + search_bpa_offset(L));
  return sa;
}

// Checks shared by the calls; fills the layout.
static int32_t search_check(const qv_model *m, int n, int max_nodes, void *ws, size_t ws_bytes,
                            qv_search_layout *L) {
  int32_t st = check_model(m);
  if (st != QV_OK) return st;
  if (n < 1 || n > QV_MAX_SAMPLES || max_nodes < 1) return QV_ERR_INVALID_ARG;
  if (!search_layout_impl(m, n, max_nodes, L)) return QV_ERR_UNSUPPORTED;
  if (!ws_ok(ws, ws_bytes, L->total_bytes)) return QV_ERR_WORKSPACE;
  return QV_OK;
}

}  // namespace qv

using namespace qv;

extern "C" {

size_t qv_search_workspace_bytes(const qv_model *m, int32_t n, int32_t max_nodes) {
  if (check_model(m) != QV_OK) return 0;
  qv_search_layout L;
  if (!search_layout_impl(m, n, max_nodes, &L)) return 0;
  return L.total_bytes;
}

int32_t qv_search_layout_of(const qv_model *m, int32_t n, int32_t max_nodes,
                            qv_search_layout *out) {
  int32_t st = check_model(m);
  if (st != QV_OK) return st;
  if (!out) return QV_ERR_INVALID_ARG;
  if (!search_layout_impl(m, n, max_nodes, out)) return QV_ERR_UNSUPPORTED;
  return QV_OK;
}

int32_t qv_search_init(const qv_model *m, const float *U_table, const float *L_table,
                       int32_t l_cols, const float *b0, int32_t n, int32_t max_nodes, void *ws,
                       size_t ws_bytes, void *stream) {
  qv_search_layout L;
  int32_t st = search_check(m, n, max_nodes, ws, ws_bytes, &L);
  if (st != QV_OK) return st;
  if (!U_table || !L_table || !b0 || l_cols < 1 || l_cols > QV_MAX_BOUND_COLS)
    return QV_ERR_INVALID_ARG;
  const DevModel dm = make_dev_model(m);
  char *w = (char *)ws;
  hipStream_t hs = (hipStream_t)stream;
  const SearchArgs sa = search_args(L, U_table, L_table, l_cols, 0, 0, w);
  st = hip_status(launch_prep_lm(dm, (uint32_t *)(w + L.sig), (float *)(w + L.staytab),
                                 (int32_t *)(w + L.err), (uint32_t *)(w + L.lm_wall), hs));
  if (st != QV_OK) return st;
  return hip_status(launch_search(0, dm, sa, b0, 0, 0, nullptr, nullptr, nullptr, hs));
}

int32_t qv_search_expand(const qv_model *m, const float *U_table, const float *L_table,
                         int32_t l_cols, int32_t n, int32_t max_nodes, uint64_t seed,
                         uint32_t query_id, int32_t expansions, void *ws, size_t ws_bytes,
                         void *stream) {
  qv_search_layout L;
  int32_t st = search_check(m, n, max_nodes, ws, ws_bytes, &L);
  if (st != QV_OK) return st;
  if (!U_table || !L_table || expansions < 0 || l_cols < 1 || l_cols > QV_MAX_BOUND_COLS)
    return QV_ERR_INVALID_ARG;
  const DevModel dm = make_dev_model(m);
  const SearchArgs sa = search_args(L, U_table, L_table, l_cols, seed, query_id, (char *)ws);
  for (int e = 0; e < expansions; ++e) {
    st = hip_status(launch_search(1, dm, sa, nullptr, 0, 0, nullptr, nullptr, nullptr,
                                  (hipStream_t)stream));
    if (st != QV_OK) return st;
  }
  return QV_OK;
}

int32_t qv_search_result(const qv_model *m, int32_t n, int32_t max_nodes, int32_t *action_out,
                         float *rootU_out, float *rootL_out, void *ws, size_t ws_bytes,
                         void *stream) {
  qv_search_layout L;
  int32_t st = search_check(m, n, max_nodes, ws, ws_bytes, &L);
  if (st != QV_OK) return st;
  if (!action_out || !rootU_out || !rootL_out) return QV_ERR_INVALID_ARG;
  const DevModel dm = make_dev_model(m);
  const SearchArgs sa = search_args(L, nullptr, nullptr, 1, 0, 0, (char *)ws);
  return hip_status(launch_search(2, dm, sa, nullptr, 0, 0, action_out, rootU_out, rootL_out,
                                  (hipStream_t)stream));
}

int32_t qv_search_update(const qv_model *m, const float *U_table, const float *L_table,
                         int32_t l_cols, int32_t n, int32_t max_nodes, int32_t a, int32_t z,
                         void *ws, size_t ws_bytes, void *stream) {
  qv_search_layout L;
  int32_t st = search_check(m, n, max_nodes, ws, ws_bytes, &L);
  if (st != QV_OK) return st;
  if (!U_table || !L_table || a < 0 || a >= m->A || z < 0 || z >= 16 * (m->L + 1) ||
      l_cols < 1 || l_cols > QV_MAX_BOUND_COLS)
    return QV_ERR_INVALID_ARG;
  const DevModel dm = make_dev_model(m);
  hipStream_t hs = (hipStream_t)stream;
  const SearchArgs sa = search_args(L, U_table, L_table, l_cols, 0, 0, (char *)ws);
  st = hip_status(launch_search(3, dm, sa, nullptr, a, z, nullptr, nullptr, nullptr, hs));
  if (st != QV_OK) return st;
  int32_t err = 0;
  st = hip_status(hipMemcpyAsync(&err, (char *)ws + L.ctl + 5 * 4, 4, hipMemcpyDeviceToHost, hs));
  if (st != QV_OK) return st;
  st = hip_status(hipStreamSynchronize(hs));
  if (st != QV_OK) return st;
  if (err == 1) return QV_ERR_ZERO_LIKELIHOOD;
  if (err == 2) return QV_ERR_UNSUPPORTED;
  return QV_OK;
}

}  // extern "C"
