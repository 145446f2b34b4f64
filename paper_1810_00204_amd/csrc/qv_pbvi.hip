// qv_pbvi.hip -- host side of point-based value iteration (Sec. IV-B):
// workspace layout, argument checks and the extern "C" entry points.  The
// kernels are in qv_plan.hip, beside the prediction and draw building blocks
// they share with the planner and the search.
#include <algorithm>
#include <cstring>

#include "qv_internal.h"

namespace qv {

constexpr size_t kPbviLdsMax = 152 * 1024;

static bool pbvi_layout_impl(const qv_model *m, int max_points, int init_cols,
                             qv_pbvi_layout *L) {
  std::memset(L, 0, sizeof *L);
  if (max_points < 1 || max_points > QV_PBVI_MAX_POINTS || init_cols < 1 ||
      init_cols > QV_PBVI_MAX_POINTS)
    return false;
  const long long S = (long long)m->W * m->H;
  const int A = m->A, ZC = 16 * (m->L + 1);
  const int ld = std::max(max_points, init_cols);
  if (pbvi_predict_lds_bytes(m->W, m->H) > kPbviLdsMax) return false;
  if (pbvi_backup_lds_bytes(m->W, m->H, ZC) > kPbviLdsMax) return false;
  if (pbvi_select_lds_bytes(ld) > kPbviLdsMax) return false;
  L->A = A;
  L->S = (int32_t)S;
  L->ZC = ZC;
  L->max_points = max_points;
  L->ld = ld;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes, 256);
    return o;
  };
  const size_t P = (size_t)max_points;
  L->sig = take((size_t)S * 4);
  L->staytab = take((size_t)A * 256 * 4);
  L->lm_wall = take((size_t)(m->L > 0 ? m->L : 1) * 4);
  L->points = take(P * (size_t)S * 4);
  L->pred = take(P * A * (size_t)S * 4);
  L->cand = take(P * A * (size_t)S * 4);
  L->idx = take(P * A * (size_t)ZC * 4);
  L->vals = take(P * A * 4);
  L->dist = take(P * A * 4);
  L->dvalid = take(P * A * 4);
  L->dz = take(P * A * 4);
  L->dcount = take(P * A * 4);
  L->dpz = take(P * A * 4);
  L->src = take(P * 4);
  L->pick = take(P * 4);
  L->gamma0 = take((size_t)S * ld * 4);
  L->gamma1 = take((size_t)S * ld * 4);
  L->ctl = take(64);
  L->err = take(256);
  L->total_bytes = off;
  return true;
}

static PbviArgs pbvi_args(const qv_pbvi_layout &L, uint64_t seed, uint32_t qid, char *ws) {
  PbviArgs pa;
  std::memset(&pa, 0, sizeof pa);
  pa.np_max = L.max_points;
  pa.ZC = L.ZC;
  pa.ld = L.ld;
  pa.key0 = (uint32_t)seed;
  pa.key1 = (uint32_t)(seed >> 32);
  pa.qid = qid;
  pa.sig = (const uint32_t *)(ws + L.sig);
  pa.staytab = (const float *)(ws + L.staytab);
  pa.lm_wall = (const uint32_t *)(ws + L.lm_wall);
  pa.pts = (float *)(ws + L.points);
  pa.pred = (float *)(ws + L.pred);
  pa.cand = (float *)(ws + L.cand);
  pa.idx = (int32_t *)(ws + L.idx);
  pa.vals = (float *)(ws + L.vals);
  pa.dist = (float *)(ws + L.dist);
  pa.dvalid = (int32_t *)(ws + L.dvalid);
  pa.dz = (int32_t *)(ws + L.dz);
  pa.dcount = (int32_t *)(ws + L.dcount);
  pa.dpz = (float *)(ws + L.dpz);
  pa.src = (int32_t *)(ws + L.src);
  pa.pick = (int32_t *)(ws + L.pick);
  pa.G0 = (float *)(ws + L.gamma0);
  pa.G1 = (float *)(ws + L.gamma1);
  pa.ctl = (int32_t *)(ws + L.ctl);
  return pa;
}

static int32_t pbvi_check(const qv_model *m, int max_points, int init_cols, void *ws,
                          size_t ws_bytes, qv_pbvi_layout *L) {
  int32_t st = check_model(m);
  if (st != QV_OK) return st;
  if (max_points < 1 || max_points > QV_PBVI_MAX_POINTS || init_cols < 1 ||
      init_cols > QV_PBVI_MAX_POINTS)
    return QV_ERR_INVALID_ARG;
  if (!pbvi_layout_impl(m, max_points, init_cols, L)) return QV_ERR_UNSUPPORTED;
  if (!ws_ok(ws, ws_bytes, L->total_bytes)) return QV_ERR_WORKSPACE;
  return QV_OK;
}

// The control words (points, round, current table, vectors, added).
static int32_t pbvi_read_ctl(const qv_pbvi_layout &L, const char *ws, int32_t ctl[5],
                             hipStream_t st) {
  hipError_t e = hipMemcpyAsync(ctl, ws + L.ctl, 5 * sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_status(e);
  return hip_status(hipStreamSynchronize(st));
}

}  // namespace qv

using namespace qv;

extern "C" {

size_t qv_pbvi_workspace_bytes(const qv_model *m, int32_t max_points, int32_t init_cols) {
  if (check_model(m) != QV_OK) return 0;
  qv_pbvi_layout L;
  if (!pbvi_layout_impl(m, max_points, init_cols, &L)) return 0;
  return L.total_bytes;
}

int32_t qv_pbvi_layout_of(const qv_model *m, int32_t max_points, int32_t init_cols,
                          qv_pbvi_layout *out) {
  int32_t st = check_model(m);
  if (st != QV_OK) return st;
  if (!out) return QV_ERR_INVALID_ARG;
  if (!pbvi_layout_impl(m, max_points, init_cols, out)) return QV_ERR_UNSUPPORTED;
  return QV_OK;
}

int32_t qv_pbvi_init(const qv_model *m, const float *b0, const float *init, int32_t init_cols,
                     int32_t max_points, void *ws, size_t ws_bytes, void *stream) {
  qv_pbvi_layout L;
  int32_t st = pbvi_check(m, max_points, init_cols, ws, ws_bytes, &L);
  if (st != QV_OK) return st;
  if (!b0 || !init) return QV_ERR_INVALID_ARG;
  const DevModel dm = make_dev_model(m);
  char *w = (char *)ws;
  hipStream_t hs = (hipStream_t)stream;
  const PbviArgs pa = pbvi_args(L, 0, 0, w);
  st = hip_status(launch_prep_lm(dm, (uint32_t *)(w + L.sig), (float *)(w + L.staytab),
                                 (int32_t *)(w + L.err), (uint32_t *)(w + L.lm_wall), hs));
  if (st != QV_OK) return st;
  PbviLaunch pl;
  pl.b0 = b0;
  pl.Gc = init;
  pl.cols = init_cols;
  return hip_status(launch_pbvi(0, dm, pa, pl, hs));
}

int32_t qv_pbvi_expand(const qv_model *m, int32_t init_cols, int32_t max_points, uint64_t seed,
                       uint32_t query_id, int32_t *added_out, void *ws, size_t ws_bytes,
                       void *stream) {
  qv_pbvi_layout L;
  int32_t st = pbvi_check(m, max_points, init_cols, ws, ws_bytes, &L);
  if (st != QV_OK) return st;
  if (!added_out) return QV_ERR_INVALID_ARG;
  *added_out = 0;
  const DevModel dm = make_dev_model(m);
  hipStream_t hs = (hipStream_t)stream;
  const PbviArgs pa = pbvi_args(L, seed, query_id, (char *)ws);
  int32_t ctl[5];
  st = pbvi_read_ctl(L, (const char *)ws, ctl, hs);
  if (st != QV_OK) return st;
  PbviLaunch pl;
  pl.np = ctl[kPbviCtlPoints];
  pl.round = ctl[kPbviCtlRound];
  if (pl.np < 1 || pl.np > L.max_points) return QV_ERR_INVALID_ARG;   // not initialised
  st = hip_status(launch_pbvi(1, dm, pa, pl, hs));
  if (st != QV_OK) return st;
  int32_t after[5];
  st = pbvi_read_ctl(L, (const char *)ws, after, hs);
  if (st != QV_OK) return st;
  const int added = after[kPbviCtlAdded];
  if (added > 0) {
    pl.count = added;
    st = hip_status(launch_pbvi(2, dm, pa, pl, hs));
    if (st != QV_OK) return st;
  }
  *added_out = added;
  return QV_OK;
}

int32_t qv_pbvi_backup(const qv_model *m, int32_t init_cols, int32_t max_points, int32_t sweeps,
                       void *ws, size_t ws_bytes, void *stream) {
  qv_pbvi_layout L;
  int32_t st = pbvi_check(m, max_points, init_cols, ws, ws_bytes, &L);
  if (st != QV_OK) return st;
  if (sweeps < 0) return QV_ERR_INVALID_ARG;
  if (sweeps == 0) return QV_OK;
  const DevModel dm = make_dev_model(m);
  hipStream_t hs = (hipStream_t)stream;
  const PbviArgs pa = pbvi_args(L, 0, 0, (char *)ws);
  int32_t ctl[5];
  st = pbvi_read_ctl(L, (const char *)ws, ctl, hs);
  if (st != QV_OK) return st;
  const int np = ctl[kPbviCtlPoints];
  int cur = ctl[kPbviCtlCur], cols = ctl[kPbviCtlCols];
  if (np < 1 || np > L.max_points || cols < 1 || cols > L.ld || (cur & ~1))
    return QV_ERR_INVALID_ARG;   // not initialised
  PbviLaunch pl;
  pl.np = np;
  for (int s = 0; s < sweeps; ++s) {
    pl.Gc = cur ? pa.G1 : pa.G0;
    pl.Gn = cur ? pa.G0 : pa.G1;
    pl.cols = cols;
    st = hip_status(launch_pbvi(3, dm, pa, pl, hs));
    if (st != QV_OK) return st;
    cur ^= 1;
    cols = np;
  }
  pl.cur = cur;
  pl.cols = cols;
  return hip_status(launch_pbvi(4, dm, pa, pl, hs));
}

int32_t qv_pbvi_result(const qv_model *m, int32_t init_cols, int32_t max_points, float *gamma_out,
                       int32_t ld_out, int32_t *npoints_out, void *ws, size_t ws_bytes,
                       void *stream) {
  qv_pbvi_layout L;
  int32_t st = pbvi_check(m, max_points, init_cols, ws, ws_bytes, &L);
  if (st != QV_OK) return st;
  if (!gamma_out || !npoints_out || ld_out < 1 || ld_out > QV_MAX_BOUND_COLS)
    return QV_ERR_INVALID_ARG;
  const DevModel dm = make_dev_model(m);
  hipStream_t hs = (hipStream_t)stream;
  const PbviArgs pa = pbvi_args(L, 0, 0, (char *)ws);
  int32_t ctl[5];
  st = pbvi_read_ctl(L, (const char *)ws, ctl, hs);
  if (st != QV_OK) return st;
  const int cur = ctl[kPbviCtlCur], cols = ctl[kPbviCtlCols];
  if (cols < 1 || cols > L.ld || (cur & ~1)) return QV_ERR_INVALID_ARG;
  if (cols > ld_out) return QV_ERR_INVALID_ARG;   // the table would drop vectors
  PbviLaunch pl;
  pl.Gc = cur ? pa.G1 : pa.G0;
  pl.cols = cols;
  pl.out = gamma_out;
  pl.ldo = ld_out;
  st = hip_status(launch_pbvi(5, dm, pa, pl, hs));
  if (st != QV_OK) return st;
  st = hip_status(hipStreamSynchronize(hs));
  if (st != QV_OK) return st;
  *npoints_out = ctl[kPbviCtlPoints];
  return QV_OK;
}

}  // extern "C"
