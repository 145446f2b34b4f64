"""Pins of the FP64 oracle to facts outside itself (CPU only).

Each test checks the oracle against something it does not compute the same
way: hand-worked fixtures from the model definitions of Sec. V, invariants
(row-stochastic transitions, conservation of mass, normalised posteriors),
special cases with closed forms (flip 0.5, flip 0, a perfect sensor, the
corridor value function), brute force on tiny inputs (dense Bellman
recursion, HMM path sums), library routines (a linear solve, rocRAND's
Philox), and statistics (Alg. 4 sampling, unbiasedness of the sampled
backup).
"""
import os
import shutil
import subprocess
import tempfile
import types

import numpy as np
import pytest

import oracle
from paper_1810_00204_amd import workloads as wl
from tests import dense_model as dm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

MAP3 = np.array([0, 1, 0,
                 0, 0, 0,
                 1, 0, 0], dtype=np.uint8)


def _slip4_exact():
    t = np.zeros((4, 9))
    for a, d in enumerate(wl.ACTIONS4):
        t[a, wl.K_OF[d]] += 0.8
        t[a, wl.K_OF[wl.ACTIONS4[(a + 1) % 4]]] += 0.1
        t[a, wl.K_OF[wl.ACTIONS4[(a + 3) % 4]]] += 0.1
    return t


def _slip8_exact():
    t = np.zeros((8, 9))
    for a, d in enumerate(wl.ACTIONS8):
        t[a, wl.K_OF[d]] += 0.7
        t[a, wl.K_OF[wl.ACTIONS8[(a + 1) % 8]]] += 0.1
        t[a, wl.K_OF[wl.ACTIONS8[(a + 7) % 8]]] += 0.1
        t[a, 4] += 0.1
    return t


def _prob3(slip, goal=-1, lm=(), flip=(0.1, 0.1, 0.1, 0.1), lm_p=0.9):
    A = slip.shape[0]
    return types.SimpleNamespace(
        W=3, H=3, occ=MAP3.copy(), slip=slip, flip=np.array(flip),
        lm_cell=np.array(lm, dtype=np.int32), lm_p=lm_p,
        R=np.zeros((9, A)), goal=goal, gamma=0.95, A=A,
        b0=np.full(9, 1 / 7.0) * (1 - MAP3))


# ---------------------------------------------------------------------------
# transition model
# ---------------------------------------------------------------------------

def test_transition_rows_match_hand_worked_fixture():
    rows = 0
    for line in open(os.path.join(GOLDEN, "transition_3x3.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        f = line.split()
        slip = _slip4_exact() if f[0] == "act4" else _slip8_exact()
        goal, s, a = int(f[1]), int(f[2]), int(f[3])
        prob = _prob3(slip, goal=goal)
        expect = np.zeros(9)
        for kv in f[4:]:
            t, p = kv.split(":")
            expect[int(t)] = float(p)
        delta = np.zeros(9)
        delta[s] = 1.0
        row = oracle.predict(prob, delta, a)
        np.testing.assert_allclose(row, expect, atol=1e-15, err_msg=line)
        rows += 1
    assert rows == 9


@pytest.mark.parametrize("seed", range(4))
def test_transition_row_stochastic_and_mass_conserving(seed):
    prob = wl.make_small(seed=seed, W=7, H=6)
    rng = np.random.default_rng(seed)
    free = np.flatnonzero(prob.occ == 0)
    for a in range(prob.A):
        for s in free:
            d = np.zeros(prob.S)
            d[s] = 1.0
            row = oracle.predict(prob, d, a)
            assert row.min() >= 0.0
            assert abs(row.sum() - 1.0) < 1e-6     # fp32 slip rows
            assert np.all(row[prob.occ == 1] == 0.0)
        b = np.zeros(prob.S)
        b[free] = rng.random(free.size)
        bp = oracle.predict(prob, b, a)
        assert abs(bp.sum() - b.sum()) < 1e-6 * b.sum()
        assert np.all(bp[prob.occ == 1] == 0.0)


def test_predict_equals_dense_product():
    prob = wl.make_rect(seed=3, side=12, n_landmarks=4, D=1, n=2)
    T = dm.transition_matrices(prob)
    b = prob.b0.astype(np.float64)
    for a in range(prob.A):
        np.testing.assert_allclose(oracle.predict(prob, b, a), b @ T[a], atol=1e-15)


# ---------------------------------------------------------------------------
# sensor model
# ---------------------------------------------------------------------------

def test_sensor_matches_hand_worked_fixture():
    prob = _prob3(_slip4_exact(), lm=(4,), flip=(0.1, 0.2, 0.3, 0.4))
    w = dm.wall_pattern(prob)
    n = 0
    for line in open(os.path.join(GOLDEN, "sensor_3x3.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        f = line.split()
        if f[0] == "wall":
            assert w[int(f[1])] == int(f[2]), line
            # the wall pattern is the reading that a noiseless sensor makes
            p0 = _prob3(_slip4_exact(), flip=(0, 0, 0, 0))
            assert oracle.obs_prob(p0, int(f[2]), int(f[1])) == 1.0
        else:
            got = oracle.obs_prob(prob, int(f[1]), int(f[2]))
            # lm_p reaches the model as an FP32 value
            assert abs(got - float(f[3])) <= 5e-7 * float(f[3]) + 1e-15, line
        n += 1
    assert n == 15


def test_sensor_rows_sum_to_one():
    prob = wl.make_rect(seed=1, side=10, n_landmarks=5, D=1, n=2)
    O = np.array([[oracle.obs_prob(prob, z, s) for z in range(prob.Z)]
                  for s in range(prob.S)])
    np.testing.assert_allclose(O.sum(axis=1), 1.0, atol=1e-6)
    np.testing.assert_allclose(O, dm.observation_matrix(prob), atol=1e-7)


# ---------------------------------------------------------------------------
# likelihood and Bayes update
# ---------------------------------------------------------------------------

def _bp(prob, a=0):
    return oracle.predict(prob, prob.b0.astype(np.float64), a)


def test_likelihood_is_dense_product_and_normalised():
    prob = wl.make_rect(seed=2, side=16, n_landmarks=6, D=1, n=2)
    O = dm.observation_matrix(prob)
    for a in range(prob.A):
        bp = _bp(prob, a)
        p = oracle.likelihood(prob, bp)
        np.testing.assert_allclose(p, bp @ O, atol=1e-12)
        assert abs(p.sum() - bp.sum()) < 1e-6


def test_likelihood_uninformative_sensor_is_uniform():
    prob = wl.make_small(seed=5)
    prob.flip = np.full(4, 0.5)
    p = oracle.likelihood(prob, _bp(prob))
    np.testing.assert_allclose(p, np.full(16, p.sum() / 16), rtol=1e-13)


def test_likelihood_noiseless_sensor_is_wall_histogram():
    prob = wl.make_small(seed=6)
    prob.flip = np.zeros(4)
    bp = _bp(prob, 2)
    p = oracle.likelihood(prob, bp)
    w = dm.wall_pattern(prob)
    hist = np.bincount(w, weights=bp, minlength=16)
    np.testing.assert_allclose(p, hist, atol=1e-15)


def test_bayes_update_normalised_and_total_probability():
    prob = wl.make_rect(seed=4, side=12, n_landmarks=3, D=1, n=2)
    for a in (0, 3):
        bp = _bp(prob, a)
        p = oracle.likelihood(prob, bp)
        zs = np.flatnonzero(p > 0)
        post, pz, st = oracle.belief_update(prob, np.tile(prob.b0, (zs.size, 1)), a, zs)
        assert st == 0
        np.testing.assert_allclose(pz, p[zs], rtol=1e-14)
        np.testing.assert_allclose(post.sum(axis=1), 1.0, atol=1e-13)
        assert post.min() >= 0.0
        # law of total probability: sum_z P(z) Phi(b,a,z) = b'
        mix = (pz[:, None] * post).sum(axis=0)
        np.testing.assert_allclose(mix, bp, atol=1e-14)


def test_bayes_update_special_cases():
    prob = wl.make_small(seed=7)
    b = prob.b0.astype(np.float64)
    bp = oracle.predict(prob, b, 1)
    prob.flip = np.full(4, 0.5)
    post, pz, st = oracle.belief_update(prob, b, 1, 9)
    np.testing.assert_allclose(post[0], bp / bp.sum(), atol=1e-15)
    prob.flip = np.zeros(4)
    w = dm.wall_pattern(prob)
    zs = [z for z in range(16) if bp[w == z].sum() > 0]
    for z in zs:
        post, pz, st = oracle.belief_update(prob, b, 1, z)
        want = np.where(w == z, bp, 0.0)
        np.testing.assert_allclose(post[0], want / want.sum(), atol=1e-15)
    # an impossible reading is reported, not divided by zero
    bad = [z for z in range(16) if bp[w == z].sum() == 0][0]
    _, pz, st = oracle.belief_update(prob, b, 1, bad)
    assert st == 2 and pz[0] == 0.0


# ---------------------------------------------------------------------------
# observation sampling
# ---------------------------------------------------------------------------

def test_philox_known_answers():
    n = 0
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        v = [int(x, 16) for x in line.split()]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert list(out) == v[6:10]
        n += 1
    assert n == 3


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc (rocRAND headers) not available")
def test_philox_matches_rocrand_header():
    src = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char **argv) {
  for (int i = 1; i + 2 < argc; i += 3) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(strtoull(argv[i], 0, 0), strtoull(argv[i + 1], 0, 0),
                 strtoull(argv[i + 2], 0, 0), &st);
    uint4 r = rocrand4(&st);
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
}
"""
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(64):
        key = rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)
        ctr = rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)
        ctr[1] &= (1 << 29) - 1          # keep 4*offset below 2^64
        cases.append((key, ctr))
    with tempfile.TemporaryDirectory() as td:
        cpp = os.path.join(td, "p.cpp")
        exe = os.path.join(td, "p")
        open(cpp, "w").write(src)
        subprocess.check_call(["hipcc", "-O1", "-o", exe, cpp])
        args = []
        for key, ctr in cases:
            seed = int(key[0]) | (int(key[1]) << 32)
            sub = int(ctr[2]) | (int(ctr[3]) << 32)
            off = 4 * (int(ctr[0]) | (int(ctr[1]) << 32))
            args += [str(seed), str(sub), str(off)]
        out = subprocess.check_output([exe] + args).decode().split("\n")
    for (key, ctr), line in zip(cases, out):
        want = [int(x) for x in line.split()]
        assert list(oracle.philox4x32_10(ctr, key)) == want


def test_uniform_layout_and_range():
    # u has 24 random bits and lies in [0, 1)
    us = [oracle.obs_uniform(12345, 7, d, s, a, 5, k)
          for d in range(2) for s in range(3) for a in range(3) for k in range(5)]
    us = np.array(us)
    assert us.min() >= 0.0 and us.max() < 1.0
    assert np.all(us * 2 ** 24 == np.floor(us * 2 ** 24))
    # word k%4 of counter (a*ceil(n/4) + k/4, slot, level, query)
    out = oracle.philox4x32_10([1 * 2 + 1, 3, 1, 7], [12345, 0])
    assert oracle.obs_uniform(12345, 7, 1, 3, 1, 5, 4) == (out[0] >> 8) / 2 ** 24


def test_inverse_cdf_draw_hand_cases():
    p = [0.2, 0.0, 0.5, 0.3]
    assert oracle.draw_obs(p, 0.0)[0] == 0
    assert oracle.draw_obs(p, 0.1)[0] == 0
    assert oracle.draw_obs(p, 0.2)[0] == 2       # u*P == F_0 is not below it
    assert oracle.draw_obs(p, 0.69)[0] == 2
    assert oracle.draw_obs(p, 0.7)[0] == 3
    assert oracle.draw_obs(p, 1 - 2 ** -24)[0] == 3
    # zero-mass bins are never drawn
    assert oracle.draw_obs([0.0, 0.5, 0.0, 0.5], 0.0)[0] == 1
    assert oracle.draw_obs([0.0, 0.5, 0.0, 0.5, 0.0], 0.75)[0] == 3
    # unnormalised input: u is scaled by the total
    assert oracle.draw_obs([2.0, 2.0], 0.49)[0] == 0
    z, mg = oracle.draw_obs(p, 0.2 + 1e-7)
    assert z == 2 and abs(mg - 1e-7) < 1e-12


def test_alg4_forward_sampling_matches_likelihood():
    """Alg. 4 (x ~ b, x' ~ T, z ~ O) draws from P(z|b,a): chi-square test."""
    from scipy import stats
    prob = wl.make_small(seed=8, W=8, H=8)
    b = prob.b0.astype(np.float64)
    for a in (0, 2):
        p = oracle.likelihood(prob, oracle.predict(prob, b, a))
        zs = oracle.alg4_sample(prob, b, a, 200000, seed=99 + a)
        cnt = np.bincount(zs, minlength=16)
        keep = p > 0
        assert cnt[~keep].sum() == 0
        exp = p[keep] / p.sum() * zs.size
        chi2 = ((cnt[keep] - exp) ** 2 / exp).sum()
        assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-3


# ---------------------------------------------------------------------------
# Q-MDP value iteration
# ---------------------------------------------------------------------------

def corridor(L=40, gamma=0.95):
    occ = np.zeros(L, dtype=np.uint8)
    slip = wl.slip_table_4()
    R = wl.reward_step_goal(occ, L, 1, slip, 0)
    return wl.Problem(name="corridor", W=L, H=1, occ=occ, slip=slip,
                      flip=np.full(4, 0.1, np.float32), lm_cell=np.zeros(0, np.int32),
                      lm_p=0.9, R=R, goal=0, gamma=gamma,
                      b0=np.eye(L, dtype=np.float32)[L - 1])


def test_value_iteration_corridor_closed_form():
    """Goal at x = 0 of a 1 x L corridor; moving west succeeds with
    probability p, otherwise the robot stays (probability s; north and south
    lie outside the map).  With reward -1 per step and R1 = -1 + 100 p for
    the move that can enter the goal:
      V(1) = R1 / (1 - g s),  V(d) = c + (V(1) - c) rho^(d-1),
      c = -1 / (1 - g s - g p),  rho = g p / (1 - g s),
    evaluated with the FP32 inputs widened to FP64."""
    L = 40
    prob = corridor(L)
    Q, res, sw = oracle.value_iterate(prob, tol=1e-14)
    g = float(np.float32(0.95))
    p = float(prob.slip[3, 3])                       # west: intended move
    s_ = float(prob.slip[3, 1]) + float(prob.slip[3, 7])
    R1 = float(prob.R[1, 3])
    V1 = R1 / (1 - g * s_)
    c = -1.0 / (1 - g * s_ - g * p)
    rho = g * p / (1 - g * s_)
    d = np.arange(1, L)
    V = Q.max(axis=1)
    np.testing.assert_allclose(V[1:], c + (V1 - c) * rho ** (d - 1), rtol=1e-11, atol=1e-11)
    assert abs(V[0]) < 1e-12
    assert np.all(Q[1:].argmax(axis=1) == 3)    # west everywhere


def test_value_iteration_corridor_exact_inputs():
    """Same closed form with exactly representable-in-FP64 inputs."""
    L = 30
    prob = corridor(L)
    prob.slip = _slip4_exact()
    prob.R = np.where(np.arange(L)[:, None] == 1, np.array([-1.0, -1.0, -1.0, 79.0]), -1.0)
    prob.R[0] = 0.0
    prob.R[1, 0] = -1.0 + 100 * 0.0
    # entering the goal from cell 1: only the west move (0.8) reaches it
    prob.gamma = 0.95
    m = oracle.Model(prob)
    m.c.gamma = 0.95
    import ctypes as C
    Q = np.zeros((L, 4))
    res, sw = C.c_double(), C.c_int()
    oracle.lib().qvo_value_iterate(m.ref, 1e-14, 100000, Q.ctypes.data_as(C.POINTER(C.c_double)),
                                   C.byref(res), C.byref(sw))
    g = 0.95
    V1 = 79.0 / (1 - 0.2 * g)
    c = -1.0 / (1 - g)
    rho = 0.8 * g / (1 - 0.2 * g)
    V = Q.max(axis=1)
    np.testing.assert_allclose(V[1:], c + (V1 - c) * rho ** (np.arange(1, L) - 1), rtol=1e-12)
    np.testing.assert_allclose(V[1:6], [97.530864, 90.275873, 83.468720, 77.081762, 71.089061],
                               atol=1e-6)


@pytest.mark.parametrize("seed", range(3))
def test_value_iteration_equals_linear_policy_evaluation(seed):
    prob = wl.make_small(seed=seed, W=9, H=7)
    Q, res, sw = oracle.value_iterate(prob, tol=1e-13)
    T = dm.transition_matrices(prob)
    pi = Q.argmax(axis=1)
    S = prob.S
    P = T[pi, np.arange(S), :]
    Rpi = prob.R.astype(np.float64)[np.arange(S), pi]
    g = float(np.float32(prob.gamma))
    V = np.linalg.solve(np.eye(S) - g * P, Rpi)
    free = prob.occ == 0
    np.testing.assert_allclose(Q.max(axis=1)[free], V[free], atol=1e-9)
    # Bellman residual of the returned table
    Vq = Q.max(axis=1)
    for a in range(prob.A):
        back = prob.R[:, a].astype(np.float64) + g * T[a] @ Vq
        np.testing.assert_allclose(Q[free, a], back[free], atol=1e-9)


# ---------------------------------------------------------------------------
# tree search
# ---------------------------------------------------------------------------

def _q(prob):
    Q, _, _ = oracle.value_iterate(prob, tol=1e-13)
    return Q


@pytest.mark.parametrize("seed,D", [(0, 1), (1, 2), (2, 2)])
def test_full_expansion_equals_dense_bellman_recursion(seed, D):
    prob = wl.make_small(seed=seed, W=5, H=5, frac=0.2, D=D)
    Q = _q(prob)
    T = dm.transition_matrices(prob)
    O = dm.observation_matrix(prob)
    R = prob.R.astype(np.float64)
    g = float(np.float32(prob.gamma))
    want = dm.bellman_full(T, O, R, Q, g, prob.b0.astype(np.float64), D)
    got = oracle.plan(prob, Q, D=D, full=True)
    np.testing.assert_allclose(got["rootQ"], want, rtol=1e-12, atol=1e-10)


def test_full_expansion_upper_bound_chain():
    """With Q the Q-MDP fixed point, V_D <= V_{D-1} <= ... <= max_a b.Q."""
    prob = wl.make_small(seed=4, W=6, H=6)
    Q = _q(prob)
    b = prob.b0.astype(np.float64)
    vals = [np.max(b @ Q)]
    for D in (1, 2, 3):
        vals.append(oracle.plan(prob, Q, D=D, full=True)["rootQ"].max())
    assert all(vals[i + 1] <= vals[i] + 1e-9 for i in range(3)), vals


def test_perfect_sensor_reduces_to_mdp():
    """A landmark on every free cell that always reports: the belief after
    one observation is a point mass, so V_D(delta_s) = V_MDP(s) for all D."""
    prob = wl.make_small(seed=3, W=5, H=4, frac=0.15)
    free = np.flatnonzero(prob.occ == 0)
    prob.lm_cell = free.astype(np.int32)
    prob.lm_p = 1.0
    prob.slip = _slip4_exact()        # rows summing to exactly 1
    Q = _q(prob)
    V = Q.max(axis=1)
    for s in free[:6]:
        b = np.zeros(prob.S)
        b[s] = 1.0
        for D in (1, 2):
            got = oracle.plan(prob, Q, b0=b, D=D, full=True)["rootQ"]
            np.testing.assert_allclose(got, Q[s], rtol=1e-9, atol=1e-8)
            np.testing.assert_allclose(got.max(), V[s], rtol=1e-9, atol=1e-8)


def test_sampled_backup_is_unbiased_at_depth_one():
    """Averaged over seeds, the frequency-weighted sampled backup equals the
    full expectation over observations (Alg. 3 and 6 vs the Bellman eq.)."""
    prob = wl.make_small(seed=9, W=6, H=6, D=1, n=3)
    Q = _q(prob)
    full = oracle.plan(prob, Q, D=1, full=True)["rootQ"]
    N = 3000
    est = np.array([oracle.plan(prob, Q, D=1, n=3, seed=1000 + i)["rootQ"] for i in range(N)])
    mean, se = est.mean(axis=0), est.std(axis=0) / np.sqrt(N)
    assert np.all(np.abs(mean - full) <= 4 * se + 1e-9), (mean, full, se)
    assert np.all(se > 0)


def test_sampled_tree_records_are_consistent():
    prob = wl.make_small(seed=1, D=2, n=2)
    Q = _q(prob)
    res = oracle.plan(prob, Q, dump_beliefs=True)
    dp = res["dump"]
    A, n, K = prob.A, prob.n, prob.A * prob.n
    g = float(np.float32(prob.gamma))
    for d in range(prob.D):
        valid = dp.level(dp.valid, d)
        for slot in np.flatnonzero(valid):
            gs = dp.level_off[d] + slot
            for a in range(A):
                kids = [slot * K + a * n + r for r in range(n)]
                cv = dp.level(dp.valid, d + 1)[kids]
                cnt = dp.level(dp.count, d + 1)[kids]
                zz = dp.level(dp.z, d + 1)[kids]
                assert cnt[cv == 1].sum() == n
                assert np.all(np.diff(zz[cv == 1]) > 0)      # distinct, ascending
                # valid children are packed first
                assert list(cv) == sorted(cv, reverse=True)
                v = dp.level(dp.V, d + 1)[kids]
                q = dp.rb[gs * A + a] + g * (cnt[cv == 1] / n * v[cv == 1]).sum()
                assert abs(q - dp.qtree[gs * A + a]) < 1e-9
                for kk in np.array(kids)[cv == 1]:
                    bl = dp.beliefs[(dp.level_off[d + 1] + kk) * prob.S:][:prob.S]
                    assert abs(bl.sum() - 1) < 1e-12 and bl.min() >= 0
            assert dp.V[gs] == max(dp.qtree[gs * A:(gs + 1) * A])
    assert res["action"] == int(np.argmax(res["rootQ"]))
    assert res["expansions"] == 1 + dp.level(dp.valid, 1).sum()


def test_sampled_tree_is_deterministic_in_seed():
    prob = wl.make_small(seed=2)
    Q = _q(prob)
    a = oracle.plan(prob, Q)
    b = oracle.plan(prob, Q)
    c = oracle.plan(prob, Q, seed=prob.seed + 1)
    assert np.array_equal(a["rootQ"], b["rootQ"])
    assert np.array_equal(a["dump"].z, b["dump"].z)
    assert not np.array_equal(a["dump"].z, c["dump"].z)


# ---------------------------------------------------------------------------
# belief filter and its adjoint
# ---------------------------------------------------------------------------

def _filter_case(side=4, ntraj=3, T=4, seed=0):
    ts = wl.make_trajectories(seed=seed, side=side, frac=0.15, ntraj=ntraj, T=T)
    return ts


def test_filter_nll_equals_path_enumeration():
    """HMM identity: exp(-NLL) = sum over all state paths of the joint
    probability of the observations (3x3 grid, 3 steps: 9^4 paths)."""
    ts = _filter_case(side=3, ntraj=2, T=3, seed=1)
    prob = ts.problem
    th = ts.theta.astype(np.float64)
    ph = ts.phi.astype(np.float64)
    slip = np.exp(th - th.max(1, keepdims=True))
    slip /= slip.sum(1, keepdims=True)
    flip = 1 / (1 + np.exp(-ph))
    pr = types.SimpleNamespace(**{k: getattr(prob, k) for k in ("W", "H", "occ", "goal", "lm_cell", "lm_p")})
    pr.slip, pr.flip, pr.A = slip, flip, 8
    T = dm.transition_matrices(pr)
    O = dm.observation_matrix(pr)
    nll, _, _ = oracle.filter_nll_grad(prob, th, ph, ts.acts, ts.obs)
    b0 = prob.b0.astype(np.float64)
    S = prob.S
    import itertools
    for i in range(ts.acts.shape[0]):
        tot = 0.0
        for path in itertools.product(range(S), repeat=4):
            p = b0[path[0]]
            for t in range(3):
                p *= T[ts.acts[i, t], path[t], path[t + 1]] * O[path[t + 1], ts.obs[i, t]]
                if p == 0:
                    break
            tot += p
        assert abs(-np.log(tot) - nll[i]) < 1e-12


@pytest.mark.parametrize("landmarks", [False, True])
def test_filter_gradient_matches_central_differences(landmarks):
    ts = _filter_case(side=5, ntraj=3, T=6, seed=2)
    prob = ts.problem
    if landmarks:
        # landmark cells scale the "no landmark" reading by 1 - lm_p
        prob.lm_cell = np.flatnonzero(prob.occ == 0)[::3].astype(np.int32)
        prob.lm_p = 0.7
    th = ts.theta.astype(np.float64)
    ph = ts.phi.astype(np.float64)
    nll, gt, gp = oracle.filter_nll_grad(prob, th, ph, ts.acts, ts.obs)
    h = 1e-4
    fd_t = np.zeros_like(th)
    for idx in np.ndindex(th.shape):
        tp, tm = th.copy(), th.copy()
        tp[idx] += h
        tm[idx] -= h
        fd_t[idx] = (oracle.filter_nll_grad(prob, tp, ph, ts.acts, ts.obs)[0].sum()
                     - oracle.filter_nll_grad(prob, tm, ph, ts.acts, ts.obs)[0].sum()) / (2 * h)
    fd_p = np.zeros(4)
    for j in range(4):
        pp, pm = ph.copy(), ph.copy()
        pp[j] += h
        pm[j] -= h
        fd_p[j] = (oracle.filter_nll_grad(prob, th, pp, ts.acts, ts.obs)[0].sum()
                   - oracle.filter_nll_grad(prob, th, pm, ts.acts, ts.obs)[0].sum()) / (2 * h)
    scale = max(np.abs(gt).max(), np.abs(gp).max())
    assert np.abs(gt - fd_t).max() <= 1e-6 * scale
    assert np.abs(gp - fd_p).max() <= 1e-6 * scale


def test_filter_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    ts = _filter_case(side=6, ntraj=4, T=8, seed=3)
    prob = ts.problem
    pr = types.SimpleNamespace(**{k: getattr(prob, k) for k in ("W", "H", "occ", "goal", "lm_cell", "lm_p")})
    pr.slip, pr.A = np.zeros((8, 9)), 8
    S = prob.S
    # one-hot "where does outcome k of cell s land" tensor from the map
    Tk = np.zeros((9, S, S))
    for k in range(9):
        sl = np.zeros((8, 9))
        sl[:, k] = 1.0
        pr.slip = sl
        Tk[k] = dm.transition_matrices(pr)[0]
    w = dm.wall_pattern(prob)
    th = torch.tensor(ts.theta.astype(np.float64), requires_grad=True)
    ph = torch.tensor(ts.phi.astype(np.float64), requires_grad=True)
    slip = torch.softmax(th, dim=1)
    f = torch.sigmoid(ph)
    Tt = torch.einsum("ak,kst->ast", slip, torch.tensor(Tk))
    bits_true = torch.tensor([[(w[s] >> j) & 1 for j in range(4)] for s in range(S)])
    total = 0
    for i in range(ts.acts.shape[0]):
        b = torch.tensor(prob.b0.astype(np.float64))
        for t in range(ts.acts.shape[1]):
            c = b @ Tt[ts.acts[i, t]]
            z = int(ts.obs[i, t])
            read = torch.tensor([(z >> j) & 1 for j in range(4)])
            o = torch.prod(torch.where(read[None, :] == bits_true, 1 - f[None, :], f[None, :]), dim=1)
            u = o * c
            eta = u.sum()
            total = total - torch.log(eta)
            b = u / eta
    total.backward()
    nll, gt, gp = oracle.filter_nll_grad(prob, ts.theta, ts.phi, ts.acts, ts.obs)
    assert abs(nll.sum() - total.item()) < 1e-10
    np.testing.assert_allclose(gt, th.grad.numpy(), rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(gp, ph.grad.numpy(), rtol=1e-9, atol=1e-11)


# ---------------------------------------------------------------------------
# single-node expansion and leaf score: the references of the large-grid
# GPU test, tied to the pinned tree search and to the dense model
# ---------------------------------------------------------------------------

def _expansion_cases():
    a = wl.make_small(seed=21, D=2, n=2)
    b = wl.make_rect(seed=22, side=16, n_landmarks=12, D=2, n=3)
    b.lm_p = 0.8
    return [a, b]


@pytest.mark.parametrize("case", [0, 1])
def test_expand_node_equals_plan_records(case):
    """qvo_expand_node at the root and at level-1 slots reproduces the
    records and child beliefs that the depth-first search (pinned above by
    brute force and by its invariants) writes for the same nodes."""
    prob = _expansion_cases()[case]
    Q = _q(prob)
    res = oracle.plan(prob, Q, dump_beliefs=True)
    dp = res["dump"]
    A, n, K, S = prob.A, prob.n, prob.K, prob.S
    checked = 0
    nodes = [(0, 0, prob.b0.astype(np.float64))]
    for s1 in np.flatnonzero(dp.level(dp.valid, 1))[:3]:
        g1 = int(dp.level_off[1] + s1)
        nodes.append((1, int(s1), dp.beliefs[g1 * S:(g1 + 1) * S].copy()))
    for d, slot, b in nodes:
        e = oracle.expand_node(prob, b, d, slot, beliefs=True)
        gs = int(dp.level_off[d] + slot)
        kids = int(dp.level_off[d + 1]) + slot * K + np.arange(K)
        assert np.array_equal(e["valid"], dp.valid[kids].astype(np.int32))
        v = e["valid"] == 1
        assert np.array_equal(e["z"][v], dp.z[kids][v])
        assert np.array_equal(e["count"][v], dp.count[kids][v])
        assert np.array_equal(e["pz"][v], dp.pz[kids][v])
        assert np.array_equal(e["margin"], dp.margin[gs * A * n:(gs + 1) * A * n])
        assert np.array_equal(e["rb"], dp.rb[gs * A:(gs + 1) * A])
        for c in np.flatnonzero(v):
            gc = int(kids[c])
            assert np.array_equal(e["beliefs"][c], dp.beliefs[gc * S:(gc + 1) * S])
        checked += int(v.sum())
    assert checked > 8


@pytest.mark.parametrize("case", [0, 1])
def test_expand_node_equals_dense_model(case):
    """The same expansion from the dense matrices of the model (written
    without the oracle): b' = b T_a, P(z) = b' O, the n draws by inverse CDF
    of P over ascending z with the oracle's Philox uniforms (pinned by the
    known-answer vectors), distinct z with counts, children O(z|.) b' / P(z),
    and R(b,a) = b . R(.,a)."""
    prob = _expansion_cases()[case]
    T = dm.transition_matrices(prob)
    O = dm.observation_matrix(prob)
    rng = np.random.default_rng(case)
    free = np.flatnonzero(prob.occ == 0)
    b = np.zeros(prob.S)
    b[free] = rng.random(free.size) ** 4
    b /= b.sum()
    d, slot = 1, 5
    e = oracle.expand_node(prob, b, d, slot, beliefs=True)
    A, n = prob.A, prob.n
    for a in range(A):
        bp = b @ T[a]
        p = bp @ O
        P = p.sum()
        F = np.cumsum(np.where(p > 0, p, 0.0))
        zs = []
        for k in range(n):
            u = oracle.obs_uniform(prob.seed, prob.query_id, d, slot, a, n, k)
            z = int(np.flatnonzero((F > u * P) & (p > 0))[0])
            zs.append(z)
        zu, cnt = np.unique(zs, return_counts=True)
        U = zu.size
        sl = slice(a * n, (a + 1) * n)
        assert list(e["valid"][sl]) == [1] * U + [0] * (n - U)
        assert np.array_equal(e["z"][sl][:U], zu)
        assert np.array_equal(e["count"][sl][:U], cnt)
        np.testing.assert_allclose(e["pz"][sl][:U], p[zu], rtol=1e-12)
        for r in range(U):
            np.testing.assert_allclose(e["beliefs"][a * n + r], O[:, zu[r]] * bp / p[zu[r]],
                                       rtol=1e-12, atol=1e-15)
        assert abs(e["rb"][a] - b @ prob.R[:, a].astype(np.float64)) < 1e-12


def test_leaf_score_is_best_alpha_vector_product():
    """max_a sum_s b(s) Q(s,a) (Alg. 5 with the Q-MDP vectors): numpy on
    random beliefs, the depth-0 plan's root value, and the leaf values the
    depth-first search stores."""
    prob = wl.make_rect(seed=23, side=16, n_landmarks=5, D=1, n=3)
    rng = np.random.default_rng(7)
    Q = rng.standard_normal((prob.S, prob.A)) * 10
    for _ in range(5):
        b = rng.random(prob.S)
        b /= b.sum()
        assert abs(oracle.leaf_score(prob, Q, b) - np.max(b @ Q)) <= 1e-12 * np.abs(Q).max()
    r0 = oracle.plan(prob, Q, D=0)
    v0 = r0["dump"].V[0]
    assert v0 == oracle.leaf_score(prob, Q, prob.b0)
    np.testing.assert_allclose(r0["rootQ"], prob.b0.astype(np.float64) @ Q, rtol=1e-12)
    res = oracle.plan(prob, Q, dump_beliefs=True)
    dp = res["dump"]
    for c in np.flatnonzero(dp.level(dp.valid, 1)):
        g = int(dp.level_off[1] + c)
        assert dp.V[g] == oracle.leaf_score(prob, Q, dp.beliefs[g * prob.S:(g + 1) * prob.S])


# ---------------------------------------------------------------------------
# the filter with an absorbing goal cell
# ---------------------------------------------------------------------------

def _goal_filter_case(side, ntraj, T, seed):
    ts = _filter_case(side=side, ntraj=ntraj, T=T, seed=seed)
    prob = ts.problem
    free = np.flatnonzero(prob.occ == 0)
    prob.goal = int(free[len(free) // 2])      # absorbing; b0 puts mass on it
    return ts


def test_filter_nll_with_goal_equals_path_enumeration():
    ts = _goal_filter_case(side=3, ntraj=2, T=3, seed=4)
    prob = ts.problem
    th = ts.theta.astype(np.float64)
    ph = ts.phi.astype(np.float64)
    slip = np.exp(th - th.max(1, keepdims=True))
    slip /= slip.sum(1, keepdims=True)
    flip = 1 / (1 + np.exp(-ph))
    pr = types.SimpleNamespace(**{k: getattr(prob, k) for k in ("W", "H", "occ", "goal", "lm_cell", "lm_p")})
    pr.slip, pr.flip, pr.A = slip, flip, 8
    T = dm.transition_matrices(pr)
    assert all(T[a, prob.goal, prob.goal] == 1.0 for a in range(8))
    O = dm.observation_matrix(pr)
    nll, _, _ = oracle.filter_nll_grad(prob, th, ph, ts.acts, ts.obs)
    b0 = prob.b0.astype(np.float64)
    import itertools
    for i in range(ts.acts.shape[0]):
        tot = 0.0
        for path in itertools.product(range(prob.S), repeat=4):
            p = b0[path[0]]
            for t in range(3):
                p *= T[ts.acts[i, t], path[t], path[t + 1]] * O[path[t + 1], ts.obs[i, t]]
                if p == 0:
                    break
            tot += p
        assert abs(-np.log(tot) - nll[i]) < 1e-12


def test_filter_gradient_with_goal_matches_central_differences():
    ts = _goal_filter_case(side=5, ntraj=3, T=6, seed=5)
    prob = ts.problem
    th = ts.theta.astype(np.float64)
    ph = ts.phi.astype(np.float64)
    nll, gt, gp = oracle.filter_nll_grad(prob, th, ph, ts.acts, ts.obs)
    h = 1e-4

    def f(t, p):
        return oracle.filter_nll_grad(prob, t, p, ts.acts, ts.obs)[0].sum()

    fd_t = np.zeros_like(th)
    for idx in np.ndindex(th.shape):
        tp, tm = th.copy(), th.copy()
        tp[idx] += h
        tm[idx] -= h
        fd_t[idx] = (f(tp, ph) - f(tm, ph)) / (2 * h)
    fd_p = np.zeros(4)
    for j in range(4):
        pp, pm = ph.copy(), ph.copy()
        pp[j] += h
        pm[j] -= h
        fd_p[j] = (f(th, pp) - f(th, pm)) / (2 * h)
    scale = max(np.abs(gt).max(), np.abs(gp).max())
    assert np.abs(gt - fd_t).max() <= 1e-6 * scale
    assert np.abs(gp - fd_p).max() <= 1e-6 * scale
    # the goal changes the gradient: the same runs without it differ
    prob.goal = -1
    _, gt0, _ = oracle.filter_nll_grad(prob, th, ph, ts.acts, ts.obs)
    assert np.abs(gt0 - gt).max() > 1e-3 * scale
