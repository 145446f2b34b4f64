// qv_internal.h -- host-side structures shared by the translation units of
// libqvts (workspace layouts, per-level launch arguments, launchers).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/qvts.h"
#include "qv_device.h"

namespace qv {

// Record arrays and scratch of one planning query, as device pointers.
struct PlanPtrs {
  int32_t *valid, *z, *count;
  float *pz, *value, *qvalue, *reward;
  float *belief[QV_MAX_DEPTH + 1];
  uint32_t *sig;
  float *staytab;   // [A][256] stay probability by blocked-neighbour pattern
  float *part;      // [slots_d][A][tiles][17] wall-pattern histograms + R(b,a)
  float *lmv;       // [slots_d][A][L] predicted mass on landmark cells
  float *leafpart;  // [slots_D][tiles][A]
  int32_t *err;
};

// Byte layout of the plan workspace.
struct PlanLayout {
  qv_tree_layout pub;
  size_t sig, staytab, part, lmv, leafpart, err, counters, lm_wall;
  size_t sort_cells, sort_chunk;   // [S] and [leaf_tiles][kSortChunkInts] int32
  int leaf_rows, leaf_tiles;       // bands of the per-parent leaf level
  size_t leafrec;                  // [slots_{D-1}][leaf_tiles][record] band records
  size_t part_slots;      // max slots of a non-leaf level
  size_t stats_ctr_len;   // int32 counters: bands done per (slot, action)
  size_t node_ctr_len;    // int32 counters: parts done per node
  size_t slot_list;       // int32: each level d = 1..D-1's slots in visiting order,
                          // present ones first (counts follow the node counters)
};

// Per-level kernel arguments (passed by value).
struct LevelArgs {
  int d, nslots, tiles, TH, n, K;
  uint32_t key0, key1, qid;
  const float *pbel;      // parent beliefs [nslots*S]
  const int32_t *pvalid;  // [nslots]
  float *part, *lmv;
  int32_t *cvalid, *cz, *ccount;
  float *cpz;             // child records (level d+1), [nslots*K]
  float *reward;          // level d [nslots*A]
  float *cbel;            // child beliefs [nslots*K*S] or null
  float *leafpart;        // [nslots*K*tiles*A] or null
  const float *Q;
  const uint32_t *sig;
  const float *staytab;
  const uint32_t *lm_wall;  // [L] true wall reading of each landmark cell
  int32_t *ctr;           // [nslots*A] bands finished per Q-node
  int q_vec;              // Q rows can be read as float4 (A = 4 or 8, aligned)
  int leaf_finish;        // per-parent last level with several bands: 1 = the band items
                          // only write their records and k_leaf_finish completes each
                          // parent; 0 = the last band of a parent to finish completes it
  int draws_apart;        // banded per-parent statistics: 1 = k_stats_draws draws after
                          // the launch; 0 = the last band of a parent draws
  int own_reward;         // per-parent band items: 1 = they form R(b,a) of their parent
                          // (an R(b,a) pass over the band); 0 = the level above wrote it
                          // into `reward` (from its reward-weighted histograms)
  float *creward;         // reward rows [slot][A] of the child level (level d+1), written by
                          // k_inner_finish, or null
  // free cells in true-wall-reading order and their chunks (see k_prep_sort)
  const int32_t *sort_cells, *sort_chunk;
  int sort_bands, sort_tc;   // bands sorted by extra workgroups of this launch (0: none)
  // slots of level d+1 in the order the next level visits them: live ones
  // from the front (count slot_n[0]), absent ones from the back (slot_n[1]);
  // null when the next level does not use it
  int32_t *slot_list, *slot_n;
  int slot_cap;           // entries of slot_list
  const int32_t *porder;  // this level's parent slots in visiting order (null: slot order)
  int agroups;            // k_update_parent: action groups per (parent, band) item (0, 1: one)
};

// Whole-tree view for the expectimax backup (Alg. 6/7).
struct TreeArgs {
  int D, n, K, A;
  float gamma;
  long long first[QV_MAX_DEPTH + 2];
  long long slots[QV_MAX_DEPTH + 1];
  const int32_t *valid, *count;
  float *value, *qvalue;
  const float *reward;
  int32_t *node_ctr;      // [total slots] finished parts per node
  int32_t *action_out;
  float *rootQ_out;
};

// Seeds of the map-signature pass of one query (see k_prep_sig).
struct PrepExtra {
  int32_t *valid, *z, *count;  // root records (nullptr: none)
  float *pz;
  int32_t *zero;               // counters cleared every call
  long long nzero;
  uint32_t *lm_wall;           // [L] wall reading of each landmark cell (or null)
};

// ---------------------------------------------------------------------------
// batched planning
// ---------------------------------------------------------------------------
// One query of a batch, resident in device memory for the life of a shape.
struct BatchQuery {
  DevModel m;
  TreeArgs tr;                     // action_out/rootQ_out: the batch's own slots
  LevelArgs lv[QV_MAX_DEPTH];      // per level; the per-call fields are bound on use
  PrepExtra px;
  uint32_t *sig;
  float *staytab;
  int32_t *err;
  int D;
  int leaf_parent;                 // last level by (parent, band) items over all actions
};

// The per-call inputs of one query.
struct BatchCall {
  const float *b0, *Q;
  uint32_t key0, key1, qid;
  int q_vec;
};

// One persistent launch over the items of all queries at level d.
struct BatchLevel {
  const BatchQuery *q;
  const BatchCall *call;
  const int32_t *base;   // [nq+1]: first item of each query at this level
  int32_t *queue;        // work counter of this launch (cleared by the prep pass)
  int nq, d, total, chunk;
};

// Prep pass over all queries: base[q] is the first 256-thread block of query q.
struct BatchPrep {
  const BatchQuery *q;
  const int32_t *base, *lm_base;   // [nq+1] blocks of the cell and landmark passes
  const int32_t *sort_base;        // [nq+1] blocks of the leaf-band sort pass
  int32_t *queue;
  int nq, nqueue;
};

// Best-first search: the node pool and control words in the workspace.
struct SearchArgs {
  int n, K, NV;                 // samples per action, |A| n, node capacity
  uint32_t key0, key1, qid;     // Philox key and query id of the draws
  const float *Ut, *Lt;         // upper [S*A] / lower [S*lcols] bound tables
  int lcols;                    // columns of the lower-bound table
  const uint32_t *sig;
  const float *staytab;
  const uint32_t *lm_wall;
  float *bel;                   // [NV][S] beliefs
  int32_t *valid, *z, *count, *parent, *depth, *E, *expanded, *cbase;   // [NV]
  float *pz, *w, *U, *L, *H;                                            // [NV]
  float *rb, *UQ, *LQ, *HQ;     // [NV][A] Q-node records
  int32_t *EQ;                  // [NV][A]
  int32_t *ctl;                 // root, select, next, expansions, flags, err
  int32_t *log;                 // [NV] node expanded by each expansion
  float *bpa;                   // [A][S] predicted beliefs of the node being expanded
};

// Point-based value iteration state in its workspace (device pointers).
struct PbviArgs {
  int np_max, ZC, ld;             // point capacity, |Z| = 16 (L + 1), table columns
  uint32_t key0, key1, qid;       // Philox key and query id of the draws
  const uint32_t *sig;
  const float *staytab;
  const uint32_t *lm_wall;
  float *pts;                     // [np_max][S] belief points
  float *pred;                    // [np_max][A][S] b' = T_a^T b
  float *cand;                    // [np_max][A][S] posteriors, then alpha_a
  int32_t *idx;                   // [np_max][A][ZC] chosen vector per observation
  float *vals, *dist;             // [np_max][A] b.alpha_a, L1 distance to the set
  int32_t *dvalid, *dz, *dcount;  // [np_max][A] draw records
  float *dpz;
  int32_t *src;                   // [np_max] source (point * A + action) of a new point
  int32_t *pick;                  // [np_max] action whose alpha_a became the point's vector
  float *G0, *G1;                 // [S][ld] vector tables
  int32_t *ctl;                   // points, round, current table, columns, added
};

// Control words of the PBVI workspace.
constexpr int kPbviCtlPoints = 0, kPbviCtlRound = 1, kPbviCtlCur = 2, kPbviCtlCols = 3,
              kPbviCtlAdded = 4;

// Per-call arguments of launch_pbvi.
struct PbviLaunch {
  const float *b0 = nullptr;
  const float *Gc = nullptr;      // current table (init: the caller's [S][cols])
  float *Gn = nullptr;            // next table
  float *out = nullptr;
  int np = 0, count = 0, round = 0, cols = 0, cur = 0, ldo = 0;
};

int tile_rows(int W, int H);
DevModel make_dev_model(const qv_model *m);
int32_t check_model(const qv_model *m);
bool ws_ok(const void *ws, size_t have, size_t need);
int32_t hip_status(hipError_t e);
// Plan workspace layout with bands of th rows (th <= 0: the default).
bool plan_layout_impl(const qv_model *m, int D, int n, int flags, PlanLayout *L, int th = 0);
size_t band_lds_bytes(int W, int TH);
size_t leaf_lds_bytes(int W, int TH, int K, int A);

// batch launchers
hipError_t launch_batch_prep(const BatchPrep &bp, int cell_blocks, int lm_blocks,
                             int sort_blocks, hipStream_t st, bool timed);
size_t leaf_parent_lds_bytes(int W, int TH, int L, int AM);
hipError_t launch_batch_level(const BatchLevel &bl, int phase, int apad, size_t lds, int grid,
                              hipStream_t st, bool timed);
int batch_level_occupancy(int phase, int apad, size_t lds);
hipError_t launch_batch_out(int nq, const int32_t *act_in, const float *rq_in, int32_t *act_out,
                            float *rq_out, hipStream_t st);

// launchers (return hipError_t)
hipError_t launch_plan(const qv_model *m, const float *Q, const float *b0, int D, int n,
                       uint64_t seed, uint32_t qid, int flags, int32_t *action_out,
                       float *rootQ_out, char *ws, const PlanLayout &L, hipStream_t st);
hipError_t launch_prep(const DevModel &dm, uint32_t *sig, float *staytab, int32_t *err,
                       hipStream_t st);
hipError_t launch_prep_lm(const DevModel &dm, uint32_t *sig, float *staytab, int32_t *err,
                          uint32_t *lm_wall, hipStream_t st);
// what: 0 init (b0), 1 one expansion (expand + update), 2 result, 3 update(a, z)
hipError_t launch_pbvi(int what, const DevModel &m, const PbviArgs &pa, const PbviLaunch &pl,
                       hipStream_t st);
size_t pbvi_predict_lds_bytes(int W, int H);
size_t pbvi_select_lds_bytes(int cols);
size_t pbvi_backup_lds_bytes(int W, int H, int ZC);
hipError_t launch_search(int what, const DevModel &m, const SearchArgs &sa, const float *b0,
                         int a, int z, int32_t *action, float *rootU, float *rootL,
                         hipStream_t st);
hipError_t launch_belief_update(const DevModel &dm, int batch, const float *b,
                                const int32_t *a, const int32_t *z, float *b_out,
                                float *p_out, char *ws, hipStream_t st);
size_t belief_update_ws(const qv_model *m, int batch);
// Host checks of a belief-update call (everything but the workspace).
int32_t belief_update_args(const qv_model *m, int batch, const float *b, const int32_t *a,
                           const int32_t *z, const float *b_out, const float *p_out);
// Enqueue the update on a workspace of belief_update_ws(m, batch) bytes; with
// check, wait and report out-of-range or zero-likelihood rows.
int32_t belief_update_run(const qv_model *m, int batch, const float *b, const int32_t *a,
                          const int32_t *z, float *b_out, float *p_out, int check, char *ws,
                          hipStream_t hs);
hipError_t run_value_iteration(const DevModel &dm, float tol, int max_sweeps, float *Q,
                               double *residual, int *sweeps, char *ws, hipStream_t st);
size_t vi_ws(const qv_model *m, int max_sweeps);
hipError_t run_fib(const DevModel &dm, float tol, int max_sweeps, float *alpha,
                   double *residual, int *sweeps, char *ws, hipStream_t st, int op = 0);
size_t fib_ws(const qv_model *m, int max_sweeps);
int32_t run_model_check(const DevModel &m, const float *b0, bool check_r, char *rec,
                        hipStream_t st);
bool filter_supported(const qv_model *m);
int filter_groups(int ntraj);
size_t filter_ws(const qv_model *m, int ntraj, int T, int k, int G);
hipError_t launch_filter(const DevModel &m, const float *theta, const float *phi, int ntraj,
                         int T, const float *b0, int b0_per_traj, const int32_t *acts,
                         const int32_t *obs, int k, float *nll, float *g_slip, float *g_flip,
                         char *ws, int G, hipStream_t st);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Brackets one kernel launch with timing events while timing is enabled.
class TimingScope {
 public:
  TimingScope(const char *name, hipStream_t st, int tag = -1);
  ~TimingScope();

 private:
  const char *name_;
  hipStream_t st_;
  void *ev_;
  int tag_;
};

#define QV_LAUNCH(kernel, grid, block, lds, st, ...)                        \
  do {                                                                      \
    ::qv::TimingScope qv_ts_(#kernel, st);                                  \
    hipLaunchKernelGGL(kernel, grid, block, lds, st, __VA_ARGS__);          \
  } while (0)

// As QV_LAUNCH, with the tree level in the timing record ("name@L<tag>").
#define QV_LAUNCH_L(tag, kernel, grid, block, lds, st, ...)                 \
  do {                                                                      \
    ::qv::TimingScope qv_ts_(#kernel, st, tag);                             \
    hipLaunchKernelGGL(kernel, grid, block, lds, st, __VA_ARGS__);          \
  } while (0)

}  // namespace qv
