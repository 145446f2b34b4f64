/*
 * qvo.c -- plain FP64 CPU oracle for the QV-tree search hot path
 * (Sun & Kumar, "Stochastic 2-D Motion Planning with a POMDP Framework").
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference
 * that the GPU library is checked against.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * path never does.  It shares no source, header, table or helper with the
 * GPU library: everything below is written out from the paper's equations
 * and algorithms, in FP64, with plain loops in the paper's order.
 *
 * Model (Sec. II and Sec. V):
 *   cell s = y*W + x, y = 0 is the top row;
 *   neighbour k = (dy+1)*3 + (dx+1), k = 4 is the cell itself (Sec. V);
 *   T'(a,k) = slip[a*9+k] is the free-space move distribution (Sec. V);
 *   T(s,a,.) moves the mass aimed at a blocked or off-grid neighbour back
 *     onto s (Sec. V, equation for transitions with occupied cells);
 *     the goal, when present, is absorbing;
 *   O(z|s): four wall bits (neighbours N1, N3, N5, N7 = up, left, right,
 *     down; off-grid counts as occupied), bit j read correctly with
 *     probability 1 - flip[j] (Sec. V sensor), times a landmark channel:
 *     a landmark cell reports its id with probability lm_p, otherwise "none";
 *     every other cell reports "none".  z = zw + 16*zl.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int W, H;
  const unsigned char *occ; /* [S] 1 = blocked */
  int A;
  const double *slip;       /* [A*9] */
  const double *flip;       /* [4] */
  int L;
  const int *lm_cell;       /* [L] cell of landmark id l+1 */
  double lm_p;
  const double *R;          /* [S*A] */
  int goal;                 /* -1: none */
  double gamma;
} qvo_model;

enum { QVO_OK = 0, QVO_ERR_ARG = 1, QVO_ERR_ZERO_LIKELIHOOD = 2, QVO_ERR_MEM = 3 };

/* ------------------------------------------------------------------------ */
/* Transition model, Sec. V                                                 */
/* ------------------------------------------------------------------------ */

/* Where the move towards neighbour k from s ends: the neighbour itself when
 * it is inside the grid and free, otherwise s (its probability is added to
 * staying, Sec. V). */
static int qvo_dest(const qvo_model *m, int s, int k) {
  int y = s / m->W, x = s % m->W;
  int ny = y + (k / 3 - 1), nx = x + (k % 3 - 1);
  if (ny < 0 || ny >= m->H || nx < 0 || nx >= m->W) return s;
  int t = ny * m->W + nx;
  return m->occ[t] ? s : t;
}

/* cells whose transition does not follow the slip table: blocked cells keep
 * their (zero) mass, the goal keeps all of its mass */
static int qvo_fixed(const qvo_model *m, int s) {
  return m->occ[s] || s == m->goal;
}

/* b'(x') = sum_x T(x,a,x') b(x), the inner sum of the posterior belief update
 * (Sec. III), computed by pushing each cell's mass along its transitions. */
void qvo_predict(const qvo_model *m, const double *b, int a, double *out) {
  int S = m->W * m->H;
  for (int s = 0; s < S; s++) out[s] = 0.0;
  for (int s = 0; s < S; s++) {
    if (b[s] == 0.0) continue;
    if (qvo_fixed(m, s)) { out[s] += b[s]; continue; }
    for (int k = 0; k < 9; k++) out[qvo_dest(m, s, k)] += m->slip[a * 9 + k] * b[s];
  }
}

/* ------------------------------------------------------------------------ */
/* Sensor model, Sec. V                                                     */
/* ------------------------------------------------------------------------ */

/* true occupancy of wall neighbour j (0 up, 1 left, 2 right, 3 down) */
static int qvo_wall_bit(const qvo_model *m, int s, int j) {
  static const int dy[4] = {-1, 0, 0, 1}, dx[4] = {0, -1, 1, 0};
  int y = s / m->W + dy[j], x = s % m->W + dx[j];
  if (y < 0 || y >= m->H || x < 0 || x >= m->W) return 1;
  return m->occ[y * m->W + x] ? 1 : 0;
}

/* per-cell landmark id (0 = none) */
static int *qvo_landmark_map(const qvo_model *m) {
  int S = m->W * m->H;
  int *lm = (int *)calloc((size_t)S, sizeof(int));
  if (!lm) return NULL;
  for (int l = 0; l < m->L; l++) lm[m->lm_cell[l]] = l + 1;
  return lm;
}

/* O(z|s) */
static double qvo_obs(const qvo_model *m, const int *lm, int z, int s) {
  int zw = z & 15, zl = z >> 4;
  double o = 1.0;
  for (int j = 0; j < 4; j++) {
    int read = (zw >> j) & 1;
    o *= (read == qvo_wall_bit(m, s, j)) ? (1.0 - m->flip[j]) : m->flip[j];
  }
  if (lm[s] == 0) return zl == 0 ? o : 0.0;
  if (zl == 0) return o * (1.0 - m->lm_p);
  return zl == lm[s] ? o * m->lm_p : 0.0;
}

double qvo_obs_prob(const qvo_model *m, int z, int s) {
  int *lm = qvo_landmark_map(m);
  if (!lm) return NAN;
  double o = qvo_obs(m, lm, z, s);
  free(lm);
  return o;
}

/* P(z|b,a) = sum_s O(z|s) b'(s) for every z (denominator of the posterior
 * belief update, Sec. III).  Each cell contributes only to the z it can
 * produce (all 16 wall readings, with "no landmark" or its own id). */
static void qvo_likelihood_lm(const qvo_model *m, const int *lm,
                              const double *bp, double *p) {
  int S = m->W * m->H, Z = 16 * (m->L + 1);
  for (int z = 0; z < Z; z++) p[z] = 0.0;
  for (int s = 0; s < S; s++) {
    if (bp[s] == 0.0) continue;
    for (int zw = 0; zw < 16; zw++) {
      p[zw] += qvo_obs(m, lm, zw, s) * bp[s];
      if (lm[s]) p[zw + 16 * lm[s]] += qvo_obs(m, lm, zw + 16 * lm[s], s) * bp[s];
    }
  }
}

int qvo_likelihood(const qvo_model *m, const double *bp, double *p) {
  int *lm = qvo_landmark_map(m);
  if (!lm) return QVO_ERR_MEM;
  qvo_likelihood_lm(m, lm, bp, p);
  free(lm);
  return QVO_OK;
}

/* Phi(b,a,z)(x') = O(x',z) b'(x') / P(z|b,a)  (posterior belief update). */
static void qvo_bayes(const qvo_model *m, const int *lm, const double *bp,
                      int z, double pz, double *out) {
  int S = m->W * m->H;
  for (int s = 0; s < S; s++) out[s] = qvo_obs(m, lm, z, s) * bp[s] / pz;
}

/* One filter step for each of `batch` beliefs: prediction, likelihood of the
 * given observation, normalisation.  p_out[i] = P(z_i|b_i,a_i). */
int qvo_belief_update(const qvo_model *m, int batch, const double *b,
                      const int *a, const int *z, double *b_out, double *p_out) {
  int S = m->W * m->H, Z = 16 * (m->L + 1);
  int *lm = qvo_landmark_map(m);
  double *bp = (double *)malloc(sizeof(double) * (size_t)S);
  double *p = (double *)malloc(sizeof(double) * (size_t)Z);
  int st = QVO_OK;
  if (!lm || !bp || !p) { st = QVO_ERR_MEM; goto done; }
  for (int i = 0; i < batch; i++) {
    qvo_predict(m, b + (size_t)i * S, a[i], bp);
    qvo_likelihood_lm(m, lm, bp, p);
    p_out[i] = p[z[i]];
    if (p[z[i]] <= 0.0) { st = QVO_ERR_ZERO_LIKELIHOOD; continue; }
    qvo_bayes(m, lm, bp, z[i], p[z[i]], b_out + (size_t)i * S);
  }
done:
  free(lm); free(bp); free(p);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC 2011): 10 rounds of the 4x32 Philox S-box with the   */
/* published multipliers and Weyl key increments.                           */
/* ------------------------------------------------------------------------ */

static void qvo_mulhilo(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

void qvo_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; r++) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint32_t hi0, lo0, hi1, lo1;
    qvo_mulhilo(M0, c0, &hi0, &lo0);
    qvo_mulhilo(M1, c2, &hi1, &lo1);
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in [0,1) with 24 random bits: exactly representable in FP32 */
static double qvo_u24(uint32_t r) { return (double)(r >> 8) * (1.0 / 16777216.0); }

/* The k-th observation uniform of (node slot, level, action a) for a query:
 * key = seed, counter = (a*ceil(n/4) + k/4, slot, level, query), word k%4. */
double qvo_obs_uniform(uint64_t seed, uint32_t qid, int level, uint32_t slot,
                       int a, int n, int k) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {(uint32_t)(a * ((n + 3) / 4) + k / 4), slot,
                     (uint32_t)level, qid};
  uint32_t out[4];
  qvo_philox4x32_10(ctr, key, out);
  return qvo_u24(out[k % 4]);
}

/* ------------------------------------------------------------------------ */
/* Forward sampling of observations (Alg. 3 and Alg. 4)                      */
/* ------------------------------------------------------------------------ */

/* Inverse-CDF draw from P(z|b,a) in ascending z: the smallest z of positive
 * mass whose running total exceeds u * P (P = the full total).  *margin is
 * the distance from u*P to the nearest running total that a small change in
 * the sums could move across, relative to P. */
static int qvo_draw(const double *p, int Z, double u, double *margin) {
  double P = 0.0;
  int last = -1;
  for (int z = 0; z < Z; z++) if (p[z] > 0.0) { P += p[z]; last = z; }
  if (last < 0) { if (margin) *margin = 0.0; return -1; }
  double target = u * P, F = 0.0, mg = INFINITY;
  int chosen = -1;
  for (int z = 0; z < Z; z++) {
    if (p[z] <= 0.0) continue;
    F += p[z];
    if (z != last) { double d = fabs(F - target); if (d < mg) mg = d; }
    if (chosen < 0 && target < F) chosen = z;
  }
  if (chosen < 0) chosen = last;
  if (margin) *margin = mg / P;
  return chosen;
}

/* exported for the tests */
int qvo_draw_obs(const double *p, int Z, double u, double *margin) {
  return qvo_draw(p, Z, u, margin);
}

/* Alg. 4 literally: per sample draw x ~ b, x' ~ T(x,a,.), z ~ O(.|x').
 * Uniforms: Philox with counter (i, 0, 0, 0x41344C47) under key `seed`, words
 * 0, 1, 2.  Used only as a statistical cross-check of the inverse-CDF draw. */
int qvo_alg4_sample(const qvo_model *m, const double *b, int a, int nsamp,
                    uint64_t seed, int *out_z) {
  int S = m->W * m->H, Z = 16 * (m->L + 1);
  int *lm = qvo_landmark_map(m);
  if (!lm) return QVO_ERR_MEM;
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  double tot = 0.0;
  for (int s = 0; s < S; s++) tot += b[s];
  for (int i = 0; i < nsamp; i++) {
    uint32_t ctr[4] = {(uint32_t)i, 0u, 0u, 0x41344C47u}, r[4];
    qvo_philox4x32_10(ctr, key, r);
    double u1 = qvo_u24(r[0]) * tot, u2 = qvo_u24(r[1]), u3 = qvo_u24(r[2]);
    int x = S - 1;
    double F = 0.0;
    for (int s = 0; s < S; s++) { F += b[s]; if (b[s] > 0.0 && u1 < F) { x = s; break; } }
    int xp = x;
    if (!qvo_fixed(m, x)) {
      double Ft = 0.0;
      for (int k = 0; k < 9; k++) {
        Ft += m->slip[a * 9 + k];
        if (m->slip[a * 9 + k] > 0.0 && u2 * 1.0 < Ft) { xp = qvo_dest(m, x, k); break; }
      }
    }
    double Fo = 0.0;
    int zz = Z - 1;
    for (int z = 0; z < Z; z++) {
      double o = qvo_obs(m, lm, z, xp);
      Fo += o;
      if (o > 0.0 && u3 < Fo) { zz = z; break; }
    }
    out_z[i] = zz;
  }
  free(lm);
  return QVO_OK;
}

/* ------------------------------------------------------------------------ */
/* Q-MDP value iteration (Sec. V-B, "self-implemented value iteration"; the  */
/* FIB alpha-vector recursion of Sec. IV-A with a perfect sensor)           */
/* ------------------------------------------------------------------------ */

/* Jacobi sweeps from V = 0:
 *   Q_k(s,a) = R(s,a) + gamma * sum_s' T(s,a,s') V_k(s'),
 *   V_{k+1}(s) = max_a Q_k(s,a);
 * blocked cells hold Q = V = 0.  Stops after the first sweep whose residual
 * r = max over free s of |V_{k+1}(s) - V_k(s)| satisfies r <= tol * max(1,
 * max|V_{k+1}|) or r = 0, or after max_sweeps.  Q holds Q_k of the last
 * sweep. */
int qvo_value_iterate(const qvo_model *m, double tol, int max_sweeps,
                      double *Q, double *residual, int *sweeps) {
  int S = m->W * m->H, A = m->A;
  double *V = (double *)calloc((size_t)S, sizeof(double));
  double *Vn = (double *)calloc((size_t)S, sizeof(double));
  if (!V || !Vn) { free(V); free(Vn); return QVO_ERR_MEM; }
  double r = INFINITY;
  int it = 0;
  while (it < max_sweeps) {
    it++;
    double vmax = 0.0;
    r = 0.0;
    for (int s = 0; s < S; s++) {
      if (m->occ[s]) {
        for (int a = 0; a < A; a++) Q[(size_t)s * A + a] = 0.0;
        Vn[s] = 0.0;
        continue;
      }
      double best = -INFINITY;
      for (int a = 0; a < A; a++) {
        double ev = 0.0;
        if (s == m->goal) ev = V[s];
        else for (int k = 0; k < 9; k++) ev += m->slip[a * 9 + k] * V[qvo_dest(m, s, k)];
        double q = m->R[(size_t)s * A + a] + m->gamma * ev;
        Q[(size_t)s * A + a] = q;
        if (q > best) best = q;
      }
      Vn[s] = best;
      double d = fabs(Vn[s] - V[s]);
      if (d > r) r = d;
      if (fabs(Vn[s]) > vmax) vmax = fabs(Vn[s]);
    }
    double *t = V; V = Vn; Vn = t;
    if (r == 0.0 || r <= tol * (vmax > 1.0 ? vmax : 1.0)) break;
  }
  free(V); free(Vn);
  if (residual) *residual = r;
  if (sweeps) *sweeps = it;
  return QVO_OK;
}

/* ------------------------------------------------------------------------ */
/* Blind-policy lower bound: for each action a, the value of taking a       */
/* forever, alpha^a = R_a + gamma T_a alpha^a (each action's own fixed      */
/* point, no max over actions), by Jacobi sweeps from 0.  Every such vector */
/* is the value of a feasible policy, so max_a b.alpha^a bounds the optimal */
/* value from below; it is the lower bound L_V of the search (Alg. 5) when  */
/* no point-based bound is used.  Stops on r = 0 or r <= tol * max(1,       */
/* max |alpha|) over free cells and all actions.                            */
/* ------------------------------------------------------------------------ */
int qvo_blind_iterate(const qvo_model *m, double tol, int max_sweeps, double *alpha,
                      double *residual, int *sweeps) {
  int S = m->W * m->H, A = m->A;
  double *cur = (double *)calloc((size_t)S * A, sizeof(double));
  double *nxt = (double *)calloc((size_t)S * A, sizeof(double));
  if (!cur || !nxt) { free(cur); free(nxt); return QVO_ERR_MEM; }
  double r = INFINITY;
  int it = 0;
  while (it < max_sweeps) {
    it++;
    double vmax = 0.0;
    r = 0.0;
    for (int s = 0; s < S; s++) {
      for (int a = 0; a < A; a++) {
        double v = 0.0;
        if (!m->occ[s]) {
          double ev = 0.0;
          if (s == m->goal) ev = cur[(size_t)s * A + a];
          else for (int k = 0; k < 9; k++) ev += m->slip[a * 9 + k] * cur[(size_t)qvo_dest(m, s, k) * A + a];
          v = m->R[(size_t)s * A + a] + m->gamma * ev;
          double d = fabs(v - cur[(size_t)s * A + a]);
          if (d > r) r = d;
          if (fabs(v) > vmax) vmax = fabs(v);
        }
        nxt[(size_t)s * A + a] = v;
      }
    }
    double *t = cur; cur = nxt; nxt = t;
    if (r == 0.0 || r <= tol * (vmax > 1.0 ? vmax : 1.0)) break;
  }
  memcpy(alpha, cur, sizeof(double) * (size_t)S * A);
  free(cur); free(nxt);
  if (residual) *residual = r;
  if (sweeps) *sweeps = it;
  return QVO_OK;
}

/* ------------------------------------------------------------------------ */
/* Fast informed bound (Sec. IV-A, the alpha-vector "Bellman equation" of    */
/* FIB): one alpha vector per action,                                       */
/*   alpha^a(x) = R(x,a) + gamma * sum_z max_a' sum_x' O(z|x') T(x,a,x')     */
/*                                              * alpha^a'(x').              */
/* ------------------------------------------------------------------------ */

/* The right-hand side of the FIB equation at one cell x for every action,
 * given the current vectors alpha [S*A] (row-major by cell).  The sum over z
 * runs over every observation that some successor x' of x can produce: all
 * 16 wall readings with "no landmark", and with the id of each landmark
 * among the successors (every other z has O(z|x') = 0 for all of them, so
 * its max over a' is 0).  Blocked x: 0.  The goal: absorbing, R = 0, so
 * its right-hand side is gamma * max_a' alpha^a'(goal). */
void qvo_fib_backup_cell(const qvo_model *m, const int *lm, const double *alpha, int x,
                         double *out) {
  int A = m->A;
  if (m->occ[x]) { for (int a = 0; a < A; a++) out[a] = 0.0; return; }
  for (int a = 0; a < A; a++) {
    /* T(x,a,.) as a list of distinct successors */
    int xs[9], nx = 0;
    double tp[9];
    if (x == m->goal) { xs[0] = x; tp[0] = 1.0; nx = 1; }
    else {
      for (int k = 0; k < 9; k++) {
        int d = qvo_dest(m, x, k), i;
        for (i = 0; i < nx; i++) if (xs[i] == d) break;
        if (i == nx) { xs[nx] = d; tp[nx] = 0.0; nx++; }
        tp[i] += m->slip[a * 9 + k];
      }
    }
    /* landmark ids the successors can report (0 = none, always possible) */
    int zl_list[10], nzl = 1;
    zl_list[0] = 0;
    for (int i = 0; i < nx; i++) if (lm[xs[i]]) {
      int j;
      for (j = 1; j < nzl; j++) if (zl_list[j] == lm[xs[i]]) break;
      if (j == nzl) zl_list[nzl++] = lm[xs[i]];
    }
    double acc = 0.0;
    for (int il = 0; il < nzl; il++) {
      for (int zw = 0; zw < 16; zw++) {
        int z = zw + 16 * zl_list[il];
        double best = -INFINITY;
        for (int ap = 0; ap < A; ap++) {
          double v = 0.0;
          for (int i = 0; i < nx; i++)
            v += qvo_obs(m, lm, z, xs[i]) * tp[i] * alpha[(size_t)xs[i] * A + ap];
          if (v > best) best = v;
        }
        acc += best;
      }
    }
    out[a] = m->R[(size_t)x * A + a] + m->gamma * acc;
  }
}

/* FIB value iteration: Jacobi sweeps alpha_{k+1} = H_FIB alpha_k from alpha_0
 * = init (NULL: all zeros) until the residual r = max over free x and all a
 * of |alpha_{k+1}(x,a) - alpha_k(x,a)| satisfies r = 0 or r <= tol * max(1,
 * max |alpha_{k+1}|), or max_sweeps sweeps.  The mapping is monotone and a
 * contraction (Sec. IV-A), so this converges from any start. */
int qvo_fib_iterate(const qvo_model *m, const double *init, double tol, int max_sweeps,
                    double *alpha, double *residual, int *sweeps) {
  int S = m->W * m->H, A = m->A;
  int *lm = qvo_landmark_map(m);
  double *cur = (double *)calloc((size_t)S * A, sizeof(double));
  double *nxt = (double *)calloc((size_t)S * A, sizeof(double));
  if (!lm || !cur || !nxt) { free(lm); free(cur); free(nxt); return QVO_ERR_MEM; }
  if (init) memcpy(cur, init, sizeof(double) * (size_t)S * A);
  double r = INFINITY;
  int it = 0;
  while (it < max_sweeps) {
    it++;
    double vmax = 0.0;
    r = 0.0;
    for (int x = 0; x < S; x++) {
      qvo_fib_backup_cell(m, lm, cur, x, nxt + (size_t)x * A);
      if (m->occ[x]) continue;
      for (int a = 0; a < A; a++) {
        double d = fabs(nxt[(size_t)x * A + a] - cur[(size_t)x * A + a]);
        if (d > r) r = d;
        if (fabs(nxt[(size_t)x * A + a]) > vmax) vmax = fabs(nxt[(size_t)x * A + a]);
      }
    }
    double *t = cur; cur = nxt; nxt = t;
    if (r == 0.0 || r <= tol * (vmax > 1.0 ? vmax : 1.0)) break;
  }
  memcpy(alpha, cur, sizeof(double) * (size_t)S * A);
  free(lm); free(cur); free(nxt);
  if (residual) *residual = r;
  if (sweeps) *sweeps = it;
  return QVO_OK;
}

/* One FIB backup at each of the listed cells (for spot checks of a large
 * table): out[i*A + a] = right-hand side of the FIB equation at cells[i]. */
int qvo_fib_backup_cells(const qvo_model *m, const double *alpha, int ncells,
                         const int *cells, double *out) {
  int *lm = qvo_landmark_map(m);
  if (!lm) return QVO_ERR_MEM;
  for (int i = 0; i < ncells; i++)
    qvo_fib_backup_cell(m, lm, alpha, cells[i], out + (size_t)i * m->A);
  free(lm);
  return QVO_OK;
}

/* ------------------------------------------------------------------------ */
/* QV-tree search by sampled expectimax, depth first (Alg. 2, 3, 5, 6, 7)    */
/* ------------------------------------------------------------------------ */

/* Tree records, indexed by capacity slot.  Level d holds K^d slots
 * (K = |A|*n); the children of slot s for action a are the slots
 * s*K + a*n + r, r = 0..(number of distinct sampled z)-1, in ascending z.
 * Level d starts at offset sum_{e<d} K^e.  Any pointer may be NULL. */
typedef struct {
  unsigned char *valid;   /* [slots] */
  int *z;                 /* [slots] sampled observation that made the node */
  int *count;             /* [slots] how many of the n draws gave it */
  double *pz;             /* [slots] P(z|b_parent,a) */
  double *V;              /* [slots] node value */
  double *qtree;          /* [slots*A] Q-node values (levels < D) */
  double *rb;             /* [slots*A] R(b,a) (levels < D) */
  double *margin;         /* [slots*A*n] draw margins (levels < D) */
  double *beliefs;        /* [slots*S] node beliefs, or NULL */
} qvo_dump;

typedef struct {
  const qvo_model *m;
  const double *Q;
  const int *lm;
  int S, Z, A, D, n, K, full;
  uint64_t seed;
  uint32_t qid;
  double **bp, **p, **child; /* per-level scratch */
  const qvo_dump *dump;
  long *level_off;
  long expansions;
} qvo_tree;

/* Alg. 3, forwardSampling then "unique measurements and frequencies": the n
 * observation draws of the Q-node (level d, slot, action a) from P(z|b,a)
 * given as p[Z], returned as distinct values zu[] in ascending order with
 * their counts fu[]; returns how many there are. */
static int qvo_qnode_draws(int Z, const double *p, uint64_t seed, uint32_t qid, int d,
                           long slot, int a, int n, int *zu, int *fu, double *margins) {
  int zs[64];
  for (int k = 0; k < n; k++) {
    double u = qvo_obs_uniform(seed, qid, d, (uint32_t)slot, a, n, k);
    double mg;
    zs[k] = qvo_draw(p, Z, u, &mg);
    if (margins) margins[k] = mg;
  }
  for (int i = 1; i < n; i++)     /* insertion sort, ascending z */
    for (int j = i; j > 0 && zs[j - 1] > zs[j]; j--) { int x = zs[j]; zs[j] = zs[j - 1]; zs[j - 1] = x; }
  int U = 0;
  for (int i = 0; i < n; ) {
    int j = i;
    while (j < n && zs[j] == zs[i]) j++;
    if (zs[i] >= 0) { zu[U] = zs[i]; fu[U] = j - i; U++; }
    i = j;
  }
  return U;
}

/* U_V(b) = max_a sum_s b(s) Q(s,a): the alpha-vector value of Eq. (PWLC form)
 * with the Q-MDP vectors as the offline bound (Alg. 5). */
static double qvo_leaf_value(const qvo_tree *t, const double *b) {
  double best = -INFINITY;
  for (int a = 0; a < t->A; a++) {
    double v = 0.0;
    for (int s = 0; s < t->S; s++) v += b[s] * t->Q[(size_t)s * t->A + a];
    if (v > best) best = v;
  }
  return best;
}

static double qvo_vnode(qvo_tree *t, const double *b, int d, long slot,
                        int *root_action, double *root_q) {
  const qvo_model *m = t->m;
  const qvo_dump *dp = t->dump;
  long gslot = t->level_off[d] + slot;
  if (dp && dp->beliefs && d > 0)
    memcpy(dp->beliefs + (size_t)gslot * t->S, b, sizeof(double) * (size_t)t->S);
  if (d == t->D) {
    double v = qvo_leaf_value(t, b);
    if (dp && dp->V) dp->V[gslot] = v;
    return v;
  }
  t->expansions++;
  double qt[9];
  double *bp = t->bp[d], *p = t->p[d], *child = t->child[d];
  for (int a = 0; a < t->A; a++) {
    /* Alg. 3: prediction and the observation distribution */
    qvo_predict(m, b, a, bp);
    qvo_likelihood_lm(m, t->lm, bp, p);
    /* R(b,a) = sum_x R(x,a) b(x)  (Sec. III) */
    double rb = 0.0;
    for (int s = 0; s < t->S; s++) rb += m->R[(size_t)s * t->A + a] * b[s];
    double q = rb;
    if (!t->full) {
      /* n forward samples, then unique observations with frequencies */
      int zu[64], fu[64];
      double *mg = (dp && dp->margin) ? dp->margin + ((size_t)gslot * t->A + a) * t->n : NULL;
      int U = qvo_qnode_draws(t->Z, p, t->seed, t->qid, d, slot, a, t->n, zu, fu, mg);
      for (int r = 0; r < U; r++) {
        int z = zu[r], f = fu[r];
        long cslot = slot * t->K + (long)a * t->n + r;
        long cg = t->level_off[d + 1] + cslot;
        qvo_bayes(m, t->lm, bp, z, p[z], child);
        double v = qvo_vnode(t, child, d + 1, cslot, NULL, NULL);
        if (dp) {
          if (dp->valid) dp->valid[cg] = 1;
          if (dp->z) dp->z[cg] = z;
          if (dp->count) dp->count[cg] = f;
          if (dp->pz) dp->pz[cg] = p[z];
        }
        /* Alg. 6 with the discount of the Bellman equation and the
         * normalised sampling frequency as the child weight */
        q += m->gamma * ((double)f / (double)t->n) * v;
      }
    } else {
      /* full expansion: every observation of positive probability, weighted
       * by P(z|b,a) (the POMDP Bellman equation, Sec. III) */
      double P = 0.0;
      for (int z = 0; z < t->Z; z++) P += p[z];
      for (int z = 0; z < t->Z; z++) {
        if (p[z] <= 0.0) continue;
        qvo_bayes(m, t->lm, bp, z, p[z], child);
        double v = qvo_vnode(t, child, d + 1, 0, NULL, NULL);
        q += m->gamma * (p[z] / P) * v;
      }
    }
    qt[a] = q;
    if (dp && dp->qtree) dp->qtree[(size_t)gslot * t->A + a] = q;
    if (dp && dp->rb) dp->rb[(size_t)gslot * t->A + a] = rb;
  }
  /* Alg. 7: V-node value is the best Q-node value; the returned action is
   * the lowest index within 1e-9 of it */
  double best = -INFINITY;
  for (int a = 0; a < t->A; a++) if (qt[a] > best) best = qt[a];
  if (root_q) for (int a = 0; a < t->A; a++) root_q[a] = qt[a];
  if (root_action) {
    int act = 0;
    for (int a = 0; a < t->A; a++) if (qt[a] >= best - 1e-9) { act = a; break; }
    *root_action = act;
  }
  if (dp && dp->V) dp->V[gslot] = best;
  return best;
}

/* Number of capacity slots of levels 0..D. */
long qvo_tree_slots(int A, int n, int D) {
  long tot = 0, lv = 1;
  for (int d = 0; d <= D; d++) { tot += lv; lv *= (long)A * n; }
  return tot;
}

/* One planning step from b0: builds the depth-D tree (full = 0: n sampled
 * observations per Q-node; full = 1: every observation) and returns the
 * root action and its Q-node values.  expansions_out counts V-node
 * expansions (Alg. 2). */
int qvo_plan(const qvo_model *m, const double *Q, const double *b0, int D,
             int n, uint64_t seed, uint32_t qid, int full, int *action,
             double *rootQ, const qvo_dump *dump, long *expansions_out) {
  if (D < 0 || n < 1 || n > 64 || m->A < 1 || m->A > 9) return QVO_ERR_ARG;
  qvo_tree t;
  memset(&t, 0, sizeof t);
  t.m = m; t.Q = Q; t.S = m->W * m->H; t.Z = 16 * (m->L + 1); t.A = m->A;
  t.D = D; t.n = n; t.K = m->A * n; t.full = full; t.seed = seed; t.qid = qid;
  t.dump = dump;
  int *lm = qvo_landmark_map(m);
  t.lm = lm;
  t.bp = (double **)calloc((size_t)D + 1, sizeof(double *));
  t.p = (double **)calloc((size_t)D + 1, sizeof(double *));
  t.child = (double **)calloc((size_t)D + 1, sizeof(double *));
  t.level_off = (long *)calloc((size_t)D + 2, sizeof(long));
  int st = QVO_OK;
  if (!lm || !t.bp || !t.p || !t.child || !t.level_off) { st = QVO_ERR_MEM; goto done; }
  {
    long lv = 1;
    for (int d = 0; d <= D; d++) { t.level_off[d + 1] = t.level_off[d] + lv; lv *= t.K; }
  }
  for (int d = 0; d < D; d++) {
    t.bp[d] = (double *)malloc(sizeof(double) * (size_t)t.S);
    t.p[d] = (double *)malloc(sizeof(double) * (size_t)t.Z);
    t.child[d] = (double *)malloc(sizeof(double) * (size_t)t.S);
    if (!t.bp[d] || !t.p[d] || !t.child[d]) { st = QVO_ERR_MEM; goto done; }
  }
  if (dump && dump->valid) dump->valid[0] = 1;
  {
    int act = 0;
    double qt_root[9];
    if (D == 0) {
      for (int a = 0; a < m->A; a++) {
        double v = 0.0;
        for (int s = 0; s < t.S; s++) v += b0[s] * Q[(size_t)s * m->A + a];
        qt_root[a] = v;
      }
      double best = -INFINITY;
      for (int a = 0; a < m->A; a++) if (qt_root[a] > best) best = qt_root[a];
      for (int a = 0; a < m->A; a++) if (qt_root[a] >= best - 1e-9) { act = a; break; }
      if (dump && dump->V) dump->V[0] = best;
    } else {
      qvo_vnode(&t, b0, 0, 0, &act, qt_root);
    }
    if (action) *action = act;
    if (rootQ) for (int a = 0; a < m->A; a++) rootQ[a] = qt_root[a];
  }
  if (expansions_out) *expansions_out = t.expansions;
done:
  if (t.bp) for (int d = 0; d < D; d++) { free(t.bp[d]); free(t.p[d]); free(t.child[d]); }
  free(t.bp); free(t.p); free(t.child); free(t.level_off); free(lm);
  return st;
}

/* One V-node expansion (Alg. 2 with Alg. 3 for every action) of belief b
 * sitting at capacity slot `slot` of level d, without recursing: for each
 * action a and rank r < n, the child records at index a*n + r (valid, z,
 * count, P(z|b,a), draw margins) and, if beliefs != NULL, the child beliefs
 * [A*n*S]; rb[a] = R(b,a).  Lets a test check any single node of a large
 * tree from its parent belief. */
int qvo_expand_node(const qvo_model *m, const double *b, int d, long slot, int n,
                    uint64_t seed, uint32_t qid, int *valid, int *z, int *count,
                    double *pz, double *margin, double *beliefs, double *rb) {
  int S = m->W * m->H, Z = 16 * (m->L + 1), A = m->A;
  if (n < 1 || n > 64) return QVO_ERR_ARG;
  int *lm = qvo_landmark_map(m);
  double *bp = (double *)malloc(sizeof(double) * (size_t)S);
  double *p = (double *)malloc(sizeof(double) * (size_t)Z);
  int st = QVO_OK;
  if (!lm || !bp || !p) { st = QVO_ERR_MEM; goto done; }
  for (int a = 0; a < A; a++) {
    qvo_predict(m, b, a, bp);
    qvo_likelihood_lm(m, lm, bp, p);
    double r = 0.0;
    for (int s = 0; s < S; s++) r += m->R[(size_t)s * A + a] * b[s];
    rb[a] = r;
    int zu[64], fu[64];
    int U = qvo_qnode_draws(Z, p, seed, qid, d, slot, a, n, zu, fu, margin + (size_t)a * n);
    for (int i = 0; i < n; i++) {
      int c = a * n + i;
      valid[c] = i < U;
      z[c] = i < U ? zu[i] : -1;
      count[c] = i < U ? fu[i] : 0;
      pz[c] = i < U ? p[zu[i]] : 0.0;
      if (beliefs && i < U) qvo_bayes(m, lm, bp, zu[i], p[zu[i]], beliefs + (size_t)c * S);
    }
  }
done:
  free(lm); free(bp); free(p);
  return st;
}

/* The leaf score max_a sum_s b(s) Q(s,a) of Alg. 5 (Q-MDP alpha vectors). */
double qvo_leaf_score(const qvo_model *m, const double *Q, const double *b) {
  int S = m->W * m->H;
  double best = -INFINITY;
  for (int a = 0; a < m->A; a++) {
    double v = 0.0;
    for (int s = 0; s < S; s++) v += b[s] * Q[(size_t)s * m->A + a];
    if (v > best) best = v;
  }
  return best;
}

/* ------------------------------------------------------------------------ */
/* Differentiable belief filter and its adjoint                             */
/* ------------------------------------------------------------------------ */

/* Negative log-likelihood of logged observations under the Bayes filter of
 * Sec. III, and its gradient with respect to the slip logits theta[A*9]
 * (T'(a,.) = softmax(theta[a,.])) and the wall-bit flip logits phi[4]
 * (flip_j = logistic(phi_j)).  For each trajectory:
 *   c_t = T_{a_t}^T b_{t-1},  u_t = O(z_t|.) * c_t,  eta_t = sum u_t,
 *   b_t = u_t / eta_t,  NLL = -sum_t log eta_t,
 * and the reverse sweep
 *   ubar_t = (lambda_t - <lambda_t, b_t> - 1) / eta_t,
 *   cbar_t = O(z_t|.) * ubar_t,  dNLL/dO(z_t|s) += c_t(s) ubar_t(s),
 *   lambda_{t-1} = T_{a_t} cbar_t,  dNLL/dT'(a_t,k) += sum_s b_{t-1}(s) cbar_t(dest(s,k)).
 * The model's own slip and flip fields are ignored; its landmarks enter the
 * likelihood as in the planner (their report probability is not a
 * parameter).  nll[i] per trajectory;
 * g_theta, g_phi are sums over trajectories.  All beliefs are stored. */
int qvo_filter_nll_grad(const qvo_model *m0, const double *theta,
                        const double *phi, int ntraj, int T, const double *b0,
                        const int *acts, const int *obs, double *nll,
                        double *g_theta, double *g_phi) {
  int S = m0->W * m0->H, A = m0->A;
  qvo_model m = *m0;
  double slip[81], flip[4];
  for (int a = 0; a < A; a++) {
    double mx = -INFINITY, sum = 0.0;
    for (int k = 0; k < 9; k++) if (theta[a * 9 + k] > mx) mx = theta[a * 9 + k];
    for (int k = 0; k < 9; k++) sum += exp(theta[a * 9 + k] - mx);
    for (int k = 0; k < 9; k++) slip[a * 9 + k] = exp(theta[a * 9 + k] - mx) / sum;
  }
  for (int j = 0; j < 4; j++) flip[j] = 1.0 / (1.0 + exp(-phi[j]));
  m.slip = slip;
  m.flip = flip;
  int *lm = qvo_landmark_map(&m);
  double *bs = (double *)malloc(sizeof(double) * (size_t)S * (size_t)(T + 1));
  double *eta = (double *)malloc(sizeof(double) * (size_t)(T + 1));
  double *c = (double *)malloc(sizeof(double) * (size_t)S);
  double *lam = (double *)malloc(sizeof(double) * (size_t)S);
  double *cbar = (double *)malloc(sizeof(double) * (size_t)S);
  double gT[81], gf[4];
  int st = QVO_OK;
  if (!lm || !bs || !eta || !c || !lam || !cbar) { st = QVO_ERR_MEM; goto done; }
  for (int i = 0; i < 81; i++) gT[i] = 0.0;
  for (int j = 0; j < 4; j++) gf[j] = 0.0;
  for (int i = 0; i < ntraj; i++) {
    const int *at = acts + (size_t)i * T, *zt = obs + (size_t)i * T;
    const double *bi = b0 + (size_t)i * S;
    memcpy(bs, bi, sizeof(double) * (size_t)S);
    double L = 0.0;
    for (int t = 1; t <= T; t++) {
      double *bprev = bs + (size_t)(t - 1) * S, *bt = bs + (size_t)t * S;
      qvo_predict(&m, bprev, at[t - 1], c);
      double e = 0.0;
      for (int s = 0; s < S; s++) { bt[s] = qvo_obs(&m, lm, zt[t - 1], s) * c[s]; e += bt[s]; }
      if (e <= 0.0) { st = QVO_ERR_ZERO_LIKELIHOOD; goto done; }
      for (int s = 0; s < S; s++) bt[s] /= e;
      eta[t] = e;
      L -= log(e);
    }
    nll[i] = L;
    for (int s = 0; s < S; s++) lam[s] = 0.0;
    for (int t = T; t >= 1; t--) {
      double *bprev = bs + (size_t)(t - 1) * S, *bt = bs + (size_t)t * S;
      int a = at[t - 1], z = zt[t - 1];
      qvo_predict(&m, bprev, a, c);
      double lb = 0.0;
      for (int s = 0; s < S; s++) lb += lam[s] * bt[s];
      for (int s = 0; s < S; s++) {
        double ubar = (lam[s] - lb - 1.0) / eta[t];
        double o = qvo_obs(&m, lm, z, s);
        cbar[s] = o * ubar;
        /* dO(z|s)/dflip_j: the landmark factor times the product over the
         * other bits, times +1 on a misread bit, -1 on a correct one */
        double go = c[s] * ubar;
        if (go != 0.0) {
          double lmf = lm[s] == 0 ? ((z >> 4) == 0 ? 1.0 : 0.0)
                                  : ((z >> 4) == 0 ? 1.0 - m.lm_p : ((z >> 4) == lm[s] ? m.lm_p : 0.0));
          for (int j = 0; j < 4; j++) {
            double rest = lmf;
            for (int jj = 0; jj < 4; jj++) {
              if (jj == j) continue;
              int rd = (z >> jj) & 1;
              rest *= (rd == qvo_wall_bit(&m, s, jj)) ? (1.0 - flip[jj]) : flip[jj];
            }
            int rd = (z >> j) & 1;
            gf[j] += go * rest * ((rd == qvo_wall_bit(&m, s, j)) ? -1.0 : 1.0);
          }
        }
      }
      for (int s = 0; s < S; s++) {
        if (qvo_fixed(&m, s)) { lam[s] = cbar[s]; continue; }
        double acc = 0.0;
        for (int k = 0; k < 9; k++) {
          double cb = cbar[qvo_dest(&m, s, k)];
          acc += slip[a * 9 + k] * cb;
          gT[a * 9 + k] += bprev[s] * cb;
        }
        lam[s] = acc;
      }
    }
  }
  /* chain rule through the softmax and the logistic */
  for (int a = 0; a < A; a++)
    for (int j = 0; j < 9; j++) {
      double g = 0.0;
      for (int k = 0; k < 9; k++)
        g += gT[a * 9 + k] * slip[a * 9 + k] * ((k == j ? 1.0 : 0.0) - slip[a * 9 + j]);
      g_theta[a * 9 + j] = g;
    }
  for (int j = 0; j < 4; j++) g_phi[j] = gf[j] * flip[j] * (1.0 - flip[j]);
done:
  free(lm); free(bs); free(eta); free(c); free(lam); free(cbar);
  return st;
}
