/*
 * qvts.h -- C ABI of the MI355X (gfx950) QV-tree search library, libqvts.so.
 *
 * The library runs the data-parallel hot path of QV-Tree Search (Sun &
 * Kumar, "Stochastic 2-D Motion Planning with a POMDP Framework"): the
 * frontier-by-frontier expansion of the belief tree (Sec. IV-C, Alg. 2-7)
 * over a 2-D occupancy grid (Sec. V), the Bayes filter step (Sec. III,
 * posterior belief update), and the Q-MDP value iteration that scores the
 * leaves (Sec. V-B, the MDP value iteration; the alpha-vector form of
 * Sec. IV-A).
 *
 * Conventions for every call:
 *  - Array arguments are DEVICE pointers unless marked "host".  The caller
 *    owns all memory; the library never allocates device memory in a call:
 *    scratch space is a caller-provided workspace whose size comes from the
 *    matching *_workspace_bytes function.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *    work asynchronously on it and return; outputs are valid once the
 *    stream has been synchronised.  Calls documented as synchronous
 *    synchronise `stream` themselves before returning.
 *  - Scalar and host-table checks run on the host before anything is
 *    enqueued; on such an error nothing is enqueued and outputs are
 *    untouched.  No exception or abort crosses this boundary.
 *  - Grid layout: cell s = y*W + x, y = 0 is the top row; "north" is y-1.
 *    Neighbour index k = (dy+1)*3 + (dx+1) for dy, dx in {-1,0,1}; k = 4 is
 *    the cell itself (the 3x3 numbering of Sec. V).
 *  - Observation z = zw + 16*zl: zw holds four wall bits (bit 0 up, bit 1
 *    left, bit 2 right, bit 3 down: the neighbours N1, N3, N5, N7 of Sec. V,
 *    1 = occupied, off-grid reads as occupied); zl is 0 ("no landmark") or
 *    the id 1..L of the landmark the robot stands on.  |Z| = 16*(L+1).
 */
#ifndef QVTS_H
#define QVTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define QV_OK 0
#define QV_ERR_INVALID_ARG 1     /* a scalar, size or pointer is out of range */
#define QV_ERR_NOT_STOCHASTIC 2  /* a slip row is negative or does not sum to 1 */
#define QV_ERR_BELIEF_INVALID 3  /* (validated calls) belief not a distribution */
#define QV_ERR_ZERO_LIKELIHOOD 4 /* P(z|b,a) = 0 for a requested observation */
#define QV_ERR_WORKSPACE 5       /* workspace NULL, misaligned or too small */
#define QV_ERR_HIP 6             /* a HIP runtime call failed; see qv_last_hip_error */
#define QV_ERR_UNSUPPORTED 7     /* valid request outside this build's limits */

/* ---- limits ------------------------------------------------------------ */
#define QV_MAX_ACTIONS 9      /* one action per 3x3 neighbour (Sec. V) */
#define QV_MAX_DEPTH 6        /* tree depth D (action-observation layers) */
#define QV_MAX_SAMPLES 16     /* samples per action n */
#define QV_MAX_LANDMARKS 511
#define QV_MAX_SIDE 2048      /* W and H */
#define QV_WORKSPACE_ALIGN 256
#define QV_MAX_BOUND_COLS 1024 /* columns of a lower-bound table (qv_search_*, qv_pbvi) */

/* ---- plan flags -------------------------------------------------------- */
/* Store the depth-D (leaf) beliefs in the workspace and score them in a
 * separate pass, instead of scoring each leaf belief as it is produced. */
#define QV_PLAN_STORE_LEAVES 1
/* Use the banded multi-pass kernels even where the whole belief would fit
 * in one workgroup's LDS (the default for such grids is one workgroup per
 * Q-node), with the layout's bands and per-action statistics at every level
 * (the batched path's arithmetic); results are the same up to FP32
 * summation order. */
#define QV_PLAN_TILED 2

/* Check the start belief on the device before planning: the call becomes
 * synchronous and returns QV_ERR_BELIEF_INVALID, with nothing planned and
 * the outputs untouched, unless b0 is a distribution over the free cells
 * (the b0 in B(X) of Sec. II): every entry finite and >= 0, zero on blocked
 * cells, and the total (summed in FP64) within 1e-5 of 1. */
#define QV_PLAN_CHECK 4

/* ---- problem statement ------------------------------------------------- */
/* The POMDP tuple (X, A, Z, T, O, R, b0, gamma) of Sec. II, specialised to
 * the grid world of Sec. V.  X is every cell of the W x H grid (blocked
 * cells included; beliefs are zero there).  T follows the slip table: under
 * action a the robot takes neighbour move k with probability slip[a*9+k];
 * a move aimed at a blocked or off-grid cell leaves it in place (Sec. V,
 * transitions with occupied cells); the goal cell, if any, is absorbing.
 * O multiplies the wall-bit likelihoods (bit j read correctly with
 * probability 1 - flip[j]) by the landmark channel (a landmark cell reports
 * its id with probability lm_p and "no landmark" otherwise; other cells
 * always report "no landmark"). */
typedef struct qv_model {
  int32_t W, H;             /* grid size, 1..QV_MAX_SIDE */
  const uint8_t *occ;       /* device [H*W]: 1 = blocked (the map m, Sec. II) */
  int32_t A;                /* number of actions, 1..QV_MAX_ACTIONS */
  float slip[81];           /* host: T'(a,k), rows a < A used, each summing to 1 */
  float flip[4];            /* host: wall-bit misread probabilities, in [0,1] */
  int32_t L;                /* number of landmarks, 0..QV_MAX_LANDMARKS */
  const int32_t *lm_cell;   /* device [L]: cell of landmark id l+1, distinct free cells */
  float lm_p;               /* probability a landmark reports its id, in [0,1] */
  const float *R;           /* device [S*A]: stage reward R(s,a), row-major by cell */
  int32_t goal;             /* absorbing goal cell, or -1 */
  float gamma;              /* discount, in (0,1) */
} qv_model;

/* Human-readable name of a status code (static storage). */
const char *qv_status_string(int32_t status);

/* The hipError_t of the last failing HIP call made by this thread. */
int32_t qv_last_hip_error(void);

/* ---- device validation of a problem statement (Sec. II tuple) ----------
 * The host checks of every call (sizes, slip rows summing to 1, flip and
 * landmark probabilities in [0,1], gamma in (0,1)) plus checks of the device
 * arrays: every R(s,a) finite and every landmark on a free in-grid cell
 * (else QV_ERR_INVALID_ARG); if b0 (device [S], may be NULL) is given, it
 * must be a distribution over the free cells: entries finite and >= 0, zero
 * on blocked cells, total within 1e-5 of 1 (else QV_ERR_BELIEF_INVALID).
 * Synchronous.  Workspace: qv_check_workspace_bytes() bytes. */
size_t qv_check_workspace_bytes(void);
int32_t qv_model_check(const qv_model *m, const float *b0, void *ws, size_t ws_bytes,
                       void *stream);

/* ---- Bayes filter step (Sec. III, posterior belief update) -------------
 * For each i < batch:  b'(x') = sum_x T(x,a_i,x') b_i(x),
 *   p_i = P(z_i|b_i,a_i) = sum_x' O(z_i|x') b'(x'),
 *   b_out_i(x') = O(z_i|x') b'(x') / p_i.
 * b, b_out: [batch*S] FP32 (may not overlap); a, z: [batch] int32 (device);
 * p_out: [batch] FP32.  Rows with p_i = 0 are left untouched in b_out.
 * Workspace: qv_belief_update_workspace_bytes(m, batch).
 * check != 0 makes the call synchronous: it then returns
 * QV_ERR_ZERO_LIKELIHOOD if some p_i = 0 or some a_i, z_i is out of range
 * (such rows are skipped either way). */
size_t qv_belief_update_workspace_bytes(const qv_model *m, int32_t batch);
int32_t qv_belief_update(const qv_model *m, int32_t batch, const float *b,
                         const int32_t *a, const int32_t *z, float *b_out,
                         float *p_out, int32_t check, void *ws, size_t ws_bytes,
                         void *stream);

/* As qv_belief_update, for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the scratch space lives in the library's own device memory, one fixed
 * region of about 4.1 MiB per GPU, held until the process ends, instead of
 * a caller workspace.  Limits: W*H <= 1048576 cells and batch * bands <=
 * 16384 (bands of about 1024 cells, whole rows); larger calls return
 * QV_ERR_UNSUPPORTED before anything is enqueued.  The call allocates
 * nothing.  Every call on one GPU shares that GPU's region, so calls that
 * overlap on one GPU (on different streams or threads) race; serialise
 * them.  Same arguments, outputs and statuses as qv_belief_update. */
int32_t qv_belief_update_noalloc(const qv_model *m, int32_t batch, const float *b,
                                 const int32_t *a, const int32_t *z, float *b_out,
                                 float *p_out, int32_t check, void *stream);

/* ---- Q-MDP value iteration (Sec. V-B; Sec. IV-A with a perfect sensor) --
 * Jacobi sweeps from V_0 = 0:
 *   Q_k(s,a) = R(s,a) + gamma * sum_s' T(s,a,s') V_k(s'),
 *   V_{k+1}(s) = max_a Q_k(s,a),  (blocked cells: Q = V = 0),
 * in FP32, with the residual r_k = max_s |V_{k+1}(s) - V_k(s)| formed in
 * FP64.  All sweeps run in one launch (a grid barrier between sweeps), so the
 * host waits once.  Stops after the first sweep with r_k = 0 or
 * r_k <= tol * max(1, max_s |V_{k+1}(s)|), or after max_sweeps sweeps.
 * Q: [S*A] FP32 output, Q_k of the last sweep.  Synchronous: on return
 * *residual_out (host) and *sweeps_out (host) hold r_k and k. */
size_t qv_vi_workspace_bytes(const qv_model *m, int32_t max_sweeps);
int32_t qv_value_iterate(const qv_model *m, float tol, int32_t max_sweeps,
                         float *Q, double *residual_out, int32_t *sweeps_out,
                         void *ws, size_t ws_bytes, void *stream);

/* ---- fast informed bound (Sec. IV-A, the FIB alpha-vector equation) ----
 * One alpha vector per action, the fixed point of
 *   alpha^a(x) = R(x,a) + gamma * sum_z max_a' sum_x' O(z|x') T(x,a,x') alpha^a'(x'),
 * by Jacobi sweeps in FP32 from alpha_0 = 0 (blocked cells: alpha = 0; the
 * goal is absorbing).  The sum over z runs over every observation a
 * successor of x can produce.  Residual r_k = max over free x and all a of
 * |alpha_k - alpha_{k-1}|, formed in FP64; stops after the first sweep with
 * r_k = 0 or r_k <= tol * max(1, max |alpha_k|), or after max_sweeps.
 * alpha: [S*A] FP32 output, row-major by cell (the layout of a Q table, so
 * it can be passed to qv_plan_step as the leaf table: leaves then score
 * max_a' sum_s b(s) alpha^a'(s), the U_V = V_FIB of Alg. 5).  FIB lies
 * between the POMDP value and Q-MDP (Sec. IV-A).  Synchronous: on return
 * *residual_out and *sweeps_out (host) hold r_k and k.
 * Workspace: qv_fib_workspace_bytes(m, max_sweeps). */
size_t qv_fib_workspace_bytes(const qv_model *m, int32_t max_sweeps);
int32_t qv_fib_iterate(const qv_model *m, float tol, int32_t max_sweeps, float *alpha,
                       double *residual_out, int32_t *sweeps_out, void *ws, size_t ws_bytes,
                       void *stream);

/* ---- blind-policy lower bound (the L_V of Alg. 5 without a point set) ---
 * One vector per action, the value of taking that action forever:
 *   alpha^a(x) = R(x,a) + gamma * sum_x' T(x,a,x') alpha^a(x'),
 * each action's own fixed point (no max over actions), by the same FP32
 * sweeps, residual rule and layout as qv_fib_iterate.  max_a b.alpha^a is a
 * lower bound on the optimal value of b.  Synchronous.
 * Workspace: qv_blind_workspace_bytes(m, max_sweeps). */
size_t qv_blind_workspace_bytes(const qv_model *m, int32_t max_sweeps);
int32_t qv_blind_iterate(const qv_model *m, float tol, int32_t max_sweeps, float *alpha,
                         double *residual_out, int32_t *sweeps_out, void *ws, size_t ws_bytes,
                         void *stream);

/* ---- one planning step (Alg. 1 inner loop + getOptimalAction) ---------
 * Builds the QV-tree of depth D from b0 level by level: every V-node is
 * expanded with all |A| actions (Alg. 2); each Q-node predicts, forms
 * P(z|b,a) over all z, draws n observations (Alg. 3/4; inverse-CDF draws on
 * the exact P(z|b,a), uniforms from Philox4x32-10 with key = seed and
 * counter (a*ceil(n/4) + k/4, slot, level, query_id), word k%4, u = (r>>8)
 * * 2^-24), keeps each distinct z once with its frequency f, and makes the
 * child belief Phi(b,a,z) (Sec. III).  Leaves at depth D score
 * max_a' sum_s b(s) Q(s,a') (Alg. 5 with the Q-MDP alpha vectors).  The
 * backup is Q(v,a) = R(b_v,a) + gamma * sum_children (f/n) V(child) and
 * V(v) = max_a Q(v,a) (Alg. 6/7); the action is the lowest a whose root
 * Q-value is within 1e-9 of the maximum.
 * Q: [S*A] FP32 leaf table; b0: [S] FP32 start belief (a distribution with
 * no mass on blocked cells; checked on the device with QV_PLAN_CHECK, not
 * checked otherwise); action_out: [1] int32; rootQ_out: [A] FP32.
 * The tree records stay in the workspace afterwards (qv_plan_layout). */
size_t qv_plan_workspace_bytes(const qv_model *m, int32_t D, int32_t n, int32_t flags);
int32_t qv_plan_step(const qv_model *m, const float *Q, const float *b0,
                     int32_t D, int32_t n, uint64_t seed, uint32_t query_id,
                     int32_t flags, int32_t *action_out, float *rootQ_out,
                     void *ws, size_t ws_bytes, void *stream);

/* Where qv_plan_step leaves the tree in its workspace.  Node records are
 * indexed by capacity slot: level d holds K^d slots (K = A*n), the children
 * of slot s under action a are slots s*K + a*n + r for r = 0,1,... in
 * ascending z, and level d starts at global slot level_first[d].  Offsets
 * are byte offsets from the workspace base; arrays span all levels unless
 * noted.  A field of value 0 for belief_offset[d] means "not stored". */
typedef struct qv_tree_layout {
  int32_t D, n, K, A, S;
  int32_t tile_rows, tiles;        /* rows per tile and tiles per belief */
  int64_t level_slots[QV_MAX_DEPTH + 1];
  int64_t level_first[QV_MAX_DEPTH + 2];
  size_t valid;       /* int32 [slots]: 1 if the node exists */
  size_t z;           /* int32 [slots]: observation that created it (levels >= 1) */
  size_t count;       /* int32 [slots]: frequency f among the n draws */
  size_t pz;          /* float [slots]: P(z|b_parent,a) */
  size_t value;       /* float [slots]: V of the node */
  size_t qvalue;      /* float [slots*A]: Q-node values (levels < D) */
  size_t reward;      /* float [slots*A]: R(b,a) (levels < D) */
  size_t belief_offset[QV_MAX_DEPTH + 1];  /* float [level_slots[d]*S] */
  size_t total_bytes;
} qv_tree_layout;
int32_t qv_plan_layout(const qv_model *m, int32_t D, int32_t n, int32_t flags,
                       qv_tree_layout *out /* host */);

/* ---- best-first (anytime) search: Alg. 1 with Alg. 2-7, Sec. IV-C ----
 * A QV-tree grown one V-node expansion at a time, always at the node the
 * root's heuristic points to (findVNodeToExpand), in a node pool held in
 * the workspace.  A new V-node (Alg. 5) takes U = max_a' b.U_table[.,a']
 * and L = max_j b.L_table[.,j] (U_table: device [S*A] FP32, e.g. the FIB
 * vectors of qv_fib_iterate; L_table: device [S*l_cols] FP32, row-major by
 * cell, e.g. the blind-policy vectors of qv_blind_iterate (l_cols = A) or
 * the PBVI vectors of qv_pbvi_result (l_cols = its ld_out)), H = U - L and
 * E = itself.  Expanding V-node v runs,
 * per action a, the prediction, P(z|b,a), n draws keyed by (node id, depth,
 * query_id) as in qv_plan_step, the distinct children Phi(b,a,z) with weight
 * f/n and their bounds (Alg. 2-5); then every ancestor is updated (Alg. 6:
 * U_Q = R(b,a) + gamma sum w U_child, L_Q likewise, H_Q / E_Q from the child
 * of largest gamma w H; Alg. 7: U_V = max U_Q, L_V = max L_Q, H_V and E_V
 * from the action of largest U_Q, first maximum on ties), and the next node
 * to expand is the root's E.  The selection stays on the device, so a call
 * of qv_search_expand enqueues all its expansions with no host round trip.
 * Node ids: the first root is 0; each expansion reserves K = A*n ids, child
 * (a, r) at base + a*n + r (r-th distinct z, ascending); a root made by
 * qv_search_update takes one id.  Expansions stop (no-ops) once the pool of
 * max_nodes cannot hold another K children or the root's E is already
 * expanded.  Grids whose belief, prediction and bins fit in LDS only
 * ((H+2)(W+2) + W*H + 4096 floats <= 152 KiB); larger ones get
 * QV_ERR_UNSUPPORTED (qv_plan_step serves them).
 *   qv_search_workspace_bytes: 0 if unsupported.
 *   qv_search_init: a tree holding only the root b0 (device [S]); async.
 *   qv_search_expand: `expansions` expansions; async.
 *   qv_search_result: getOptimalAction, the lowest action whose L_Q at the
 *     root is within 1e-9 of the largest (action_out device int32 [1]; -1 if
 *     the root is not expanded), and the root's U_Q, L_Q (device FP32 [A]);
 *     async.
 *   qv_search_update: update(a, z) of Alg. 1: the root moves to its child
 *     under (a, z) with that child's subtree; if z was not drawn there, a new
 *     root Phi(b_root, a, z) is formed (QV_ERR_ZERO_LIKELIHOOD if P(z|b,a) =
 *     0, QV_ERR_UNSUPPORTED if the pool is full, the tree then unchanged).
 *     Synchronous.
 *   qv_search_layout_of: where the node records are in the workspace. */
typedef struct qv_search_layout {
  int32_t n, K, A, S, max_nodes;
  size_t sig, staytab, lm_wall;
  size_t belief;      /* float [max_nodes][S] */
  size_t valid, z, count, pz, weight, parent, depth, U, L, H, E, expanded, child_base;
                      /* per node: int32 / float [max_nodes]; parent = v*A + a or -1 */
  size_t rb, UQ, LQ, HQ, EQ;   /* per (node, action): [max_nodes][A] */
  size_t ctl;         /* int32: root, select, next, expansions, flags, err */
  size_t log;         /* int32 [max_nodes]: node expanded by expansion e */
  size_t err;
  size_t total_bytes;
} qv_search_layout;
size_t qv_search_workspace_bytes(const qv_model *m, int32_t n, int32_t max_nodes);
int32_t qv_search_layout_of(const qv_model *m, int32_t n, int32_t max_nodes,
                            qv_search_layout *out /* host */);
int32_t qv_search_init(const qv_model *m, const float *U_table, const float *L_table,
                       int32_t l_cols, const float *b0, int32_t n, int32_t max_nodes, void *ws,
                       size_t ws_bytes, void *stream);
int32_t qv_search_expand(const qv_model *m, const float *U_table, const float *L_table,
                         int32_t l_cols, int32_t n, int32_t max_nodes, uint64_t seed,
                         uint32_t query_id, int32_t expansions, void *ws, size_t ws_bytes,
                         void *stream);
int32_t qv_search_result(const qv_model *m, int32_t n, int32_t max_nodes, int32_t *action_out,
                         float *rootU_out, float *rootL_out, void *ws, size_t ws_bytes,
                         void *stream);
int32_t qv_search_update(const qv_model *m, const float *U_table, const float *L_table,
                         int32_t l_cols, int32_t n, int32_t max_nodes, int32_t a, int32_t z,
                         void *ws, size_t ws_bytes, void *stream);

/* ---- point-based value iteration: Sec. IV-B ----------------------------
 * A lower bound V(b) = max_j b.alpha_j from a set of belief points and one
 * alpha vector per point, held in the workspace (vectors row-major by cell,
 * a table [S][ld] as the search's L_table).  The set starts as {b0} and the
 * vectors as `init` (device [S*init_cols] FP32 row-major by cell; a lower
 * bound such as the blind-policy vectors of qv_blind_iterate, so that every
 * later vector is a policy's value and V stays a lower bound).
 *   qv_pbvi_expand: every point draws one observation per action (P(z|b,a)
 *     by inverse CDF on one uniform from the Philox stream of qv_plan_step
 *     with counter (a, point, 64 + round, query_id)), and the posterior
 *     farthest in L1 from the set joins it (first maximum over actions; none
 *     at distance 0), in point order while fewer than max_points are held.
 *     The round counts the calls since qv_pbvi_init.  Synchronous; the number
 *     of points added goes to *added_out (host).
 *   qv_pbvi_backup: `sweeps` PBVI backups of every point: per action a and
 *     observation z the vector j of largest sum_x O(z|x) b'(x) alpha_j(x)
 *     (b' = T_a^T b; first maximum), alpha_a = R_a + gamma sum_z T_a
 *     (O_z * alpha_{a,z}) on free cells (0 on blocked ones), and the point's
 *     new vector is the alpha_a of largest b.alpha_a (first maximum); after
 *     a backup there is one vector per point.  Async after reading 20 bytes.
 *   qv_pbvi_result: the vectors into gamma_out (device [S][ld_out] FP32,
 *     columns beyond the vector count repeat column 0, which leaves the
 *     maximum unchanged) and the point count into *npoints_out (host).
 *     Synchronous.
 * Grids whose belief, prediction and bins fit in LDS only (as the search);
 * max_points and init_cols in 1..QV_PBVI_MAX_POINTS; otherwise
 * QV_ERR_UNSUPPORTED / QV_ERR_INVALID_ARG.  The same (m, max_points,
 * init_cols) must be passed to every call on one workspace.
 *   qv_pbvi_layout_of: where the points and the last backup's choices are. */
#define QV_PBVI_MAX_POINTS 256
typedef struct qv_pbvi_layout {
  int32_t A, S, ZC, max_points, ld;   /* ZC = 16 (L + 1) observations; ld = table columns */
  size_t sig, staytab, lm_wall;
  size_t points;      /* float [max_points][S] */
  size_t pred;        /* float [max_points][A][S]: b' = T_a^T b */
  size_t cand;        /* float [max_points][A][S]: alpha_a of the last backup */
  size_t idx;         /* int32 [max_points][A][ZC]: vector chosen per observation */
  size_t vals;        /* float [max_points][A]: b.alpha_a of the last backup */
  size_t dist;        /* float [max_points][A]: L1 distance of the last expansion's posteriors */
  size_t dvalid, dz, dcount, dpz;   /* [max_points][A]: that expansion's draws */
  size_t src;         /* int32 [max_points]: point * A + action of each added point */
  size_t pick;        /* int32 [max_points]: action picked by the last backup */
  size_t gamma0, gamma1;            /* float [S][ld] vector tables */
  size_t ctl;         /* int32: points, round, current table (0/1), vectors, added */
  size_t err;
  size_t total_bytes;
} qv_pbvi_layout;
size_t qv_pbvi_workspace_bytes(const qv_model *m, int32_t max_points, int32_t init_cols);
int32_t qv_pbvi_layout_of(const qv_model *m, int32_t max_points, int32_t init_cols,
                          qv_pbvi_layout *out /* host */);
int32_t qv_pbvi_init(const qv_model *m, const float *b0, const float *init, int32_t init_cols,
                     int32_t max_points, void *ws, size_t ws_bytes, void *stream);
int32_t qv_pbvi_expand(const qv_model *m, int32_t init_cols, int32_t max_points, uint64_t seed,
                       uint32_t query_id, int32_t *added_out /* host */, void *ws,
                       size_t ws_bytes, void *stream);
int32_t qv_pbvi_backup(const qv_model *m, int32_t init_cols, int32_t max_points, int32_t sweeps,
                       void *ws, size_t ws_bytes, void *stream);
int32_t qv_pbvi_result(const qv_model *m, int32_t init_cols, int32_t max_points, float *gamma_out,
                       int32_t ld_out, int32_t *npoints_out /* host */, void *ws,
                       size_t ws_bytes, void *stream);

/* ---- batched planning ------------------------------------------------------
 * Many independent planning steps (Alg. 1 inner loop, as qv_plan_step), each
 * with its own grid, depth and Q table, expanded together: per tree level one
 * persistent launch forms the statistics and observation draws of every
 * Q-node of every query and a second one writes the child beliefs or, at a
 * query's last level, scores its leaves and completes its backup.  Both take
 * (query, parent slot, band, action) items from a work counter in device
 * memory.  Query q draws with query_id = q; with the default shape its
 * results equal qv_plan_step(models[q], Q[q], b0[q], depths[q], n, seed, q,
 * QV_PLAN_TILED, ...) bit for bit.
 *
 * qv_batch_create checks the models (as qv_plan_step), copies the qv_model
 * structs (not the device arrays they point to: occ, lm_cell and R must stay
 * valid and unchanged while the batch is used) and fixes the work shape to
 * bands of about 1024 cells (QVTS_TILE_CELLS overrides), one item per visit
 * to the queue.  depths[q] in 1..QV_MAX_DEPTH.  With QV_BATCH_GRAPH the
 * launches of each level are captured once into a HIP graph (on a stream of
 * the batch's own) and replayed on the caller's stream; a new workspace
 * address or shape recaptures.  The handle is host memory plus a small
 * pinned buffer; it is not safe for concurrent use from several threads.
 *
 * qv_batch_workspace_bytes: bytes for every candidate shape (so a shape
 * change never needs a larger workspace).
 * qv_batch_plan: Q[q] and b0[q] are host arrays of nq DEVICE pointers (Q[q]:
 * [S_q*A_q] FP32, b0[q]: [S_q] FP32); actions: device int32 [nq]; rootQ:
 * device FP32 [nq*QV_MAX_ACTIONS]: row q holds query q's root Q-values,
 * entries a >= A_q are 0.
 * Asynchronous on stream; the first call on a workspace uploads the query
 * descriptors and waits for that upload.
 * qv_batch_set_shape / qv_batch_get_shape: bands of about tile_cells cells
 * (whole rows), chunk (1..64) items taken per visit to the queue.
 * qv_batch_autotune: runs every candidate shape (tile_cells 256..4096,
 * chunk 1, 2, 4) reps times after one warm-up, keeps the fastest and returns
 * its time per batch in *best_ms_out (may be NULL); synchronous.  Results of
 * different shapes differ only in the rounding of the band sums.
 * qv_batch_layout: query q's tree records (qv_tree_layout) and the byte
 * offset of its region in the workspace. */
typedef struct qv_batch qv_batch;
#define QV_BATCH_GRAPH 1
int32_t qv_batch_create(int32_t nq, const qv_model *models /* host [nq] */,
                        const int32_t *depths /* host [nq] */, int32_t n, int32_t flags,
                        qv_batch **out);
int32_t qv_batch_destroy(qv_batch *b);
size_t qv_batch_workspace_bytes(const qv_batch *b);
int32_t qv_batch_set_shape(qv_batch *b, int32_t tile_cells, int32_t chunk);
int32_t qv_batch_get_shape(const qv_batch *b, int32_t *tile_cells, int32_t *chunk);
int32_t qv_batch_plan(qv_batch *b, const float *const *Q, const float *const *b0,
                      uint64_t seed, int32_t *actions, float *rootQ, void *ws,
                      size_t ws_bytes, void *stream);
int32_t qv_batch_autotune(qv_batch *b, const float *const *Q, const float *const *b0,
                          uint64_t seed, int32_t *actions, float *rootQ, int32_t reps,
                          void *ws, size_t ws_bytes, void *stream, float *best_ms_out);
int32_t qv_batch_layout(const qv_batch *b, int32_t q, qv_tree_layout *out /* host */,
                        size_t *offset_out /* host */);

/* ---- differentiable filter -----------------------------------------------
 * Negative log-likelihood of logged runs under the Bayes filter of Sec. III,
 * and its gradient with respect to the slip logits theta (T'(a,.) =
 * softmax(theta[a*9 .. a*9+8])) and the wall-bit flip logits phi (flip_j =
 * 1/(1+exp(-phi_j))).  For run i with start belief b_0 (b0, [S], or [ntraj*S]
 * when b0_per_traj != 0), actions acts[i*T+t-1] and observations
 * obs[i*T+t-1], t = 1..T:
 *   c_t = T_{a_t}^T b_{t-1},  eta_t = sum_s O(z_t|s) c_t(s),
 *   b_t = O(z_t|.) c_t / eta_t,  nll_out[i] = -sum_t log eta_t.
 * g_slip [A*9] and g_flip [4] receive d(sum_i nll_i)/d(theta, phi); pass
 * NULL for both to skip the reverse sweep.  The model's own slip and flip
 * fields are not used; its map, landmarks and goal are.  Beliefs are stored
 * every ckpt_every steps and each segment is recomputed for the reverse
 * sweep, so workspace grows with T/ckpt_every + ckpt_every beliefs per
 * concurrent run, not with T.  theta, phi, b0, acts, obs, nll_out, g_* are
 * device arrays (acts, obs and nll_out may be NULL when ntraj = 0; the
 * gradients are then 0).  Grids need (W+2)*(H+2) + W*H + 256*A floats of LDS (at
 * most 150 KiB, e.g. 128 x 128 with 8 actions); else QV_ERR_UNSUPPORTED.  check != 0 makes the
 * call synchronous and reports an out-of-range action or observation
 * (QV_ERR_INVALID_ARG; that run's nll is NaN) or a zero-probability
 * observation (QV_ERR_ZERO_LIKELIHOOD). */
size_t qv_filter_workspace_bytes(const qv_model *m, int32_t ntraj, int32_t T,
                                 int32_t ckpt_every);
int32_t qv_filter_nll_grad(const qv_model *m, const float *theta, const float *phi,
                           int32_t ntraj, int32_t T, const float *b0, int32_t b0_per_traj,
                           const int32_t *acts, const int32_t *obs, int32_t ckpt_every,
                           float *nll_out, float *g_slip, float *g_flip, int32_t check,
                           void *ws, size_t ws_bytes, void *stream);

/* ---- kernel timing (benchmarking aid) ----------------------------------
 * While enabled, each kernel the library launches is bracketed by two
 * hipEvents recorded on its launch stream.  qv_timing_read (after the
 * caller has synchronised those streams) returns, per kernel name (with
 * "@L<d>" appended for per-level planning kernels), the
 * number of launches and the summed event-to-event time, then clears the
 * records.  qv_timing_enable(on) also clears them.  Host-side only; not
 * meant for concurrent use from several threads. */
typedef struct qv_kernel_time {
  char name[32];
  int64_t launches;
  double total_ms;
} qv_kernel_time;
int32_t qv_timing_enable(int32_t on);
int32_t qv_timing_read(qv_kernel_time *out /* host [max_entries] */, int32_t max_entries,
                       int32_t *n_out /* host */);

#ifdef __cplusplus
}
#endif
#endif /* QVTS_H */
