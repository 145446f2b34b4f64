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
  size_t part_slots;      // max slots of a non-leaf level
  size_t stats_ctr_len;   // int32 counters: bands done per (slot, action)
  size_t node_ctr_len;    // int32 counters: parts done per node
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

int tile_rows(int W, int H);
void plan_layout(const qv_model *m, int D, int n, int flags, PlanLayout *L);
DevModel make_dev_model(const qv_model *m);

// launchers (return hipError_t)
hipError_t launch_plan(const qv_model *m, const float *Q, const float *b0, int D, int n,
                       uint64_t seed, uint32_t qid, int flags, int32_t *action_out,
                       float *rootQ_out, char *ws, const PlanLayout &L, hipStream_t st);
hipError_t launch_prep(const DevModel &dm, uint32_t *sig, float *staytab, int32_t *err,
                       hipStream_t st);
hipError_t launch_belief_update(const DevModel &dm, int batch, const float *b,
                                const int32_t *a, const int32_t *z, float *b_out,
                                float *p_out, char *ws, hipStream_t st);
size_t belief_update_ws(const qv_model *m, int batch);
hipError_t run_value_iteration(const DevModel &dm, float tol, int max_sweeps, float *Q,
                               double *residual, int *sweeps, char *ws, hipStream_t st);
size_t vi_ws(const qv_model *m, int max_sweeps);
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
