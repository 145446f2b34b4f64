"""Pins of the oracle's fast informed bound (Sec. IV-A, the FIB alpha-vector
equation), CPU only.

Each pin ties the oracle to something other than itself:
  * a perfect sensor (every free cell a landmark that always reports) makes
    the max over a' act per successor, so FIB is the Q-MDP fixed point, which
    has its own pins (corridor closed form, linear policy evaluation);
  * a corridor whose wall readings tell every cell apart (noiseless bits)
    gives the corridor closed form directly;
  * an uninformative sensor (every bit flipped with probability 1/2, no
    landmarks) makes O(z|x') = 1/16, and the equation reduces to
    alpha^a = R_a + gamma max_a' T_a alpha^a', evaluated here by a dense
    numpy iteration on matrices built independently of the oracle;
  * the ordering blind-policy value <= V_FIB(delta_x) and alpha_FIB <= Q_MDP
    (FIB bounds the optimal value from above and is below Q-MDP), with the
    blind policies solved by numpy.linalg.solve;
  * monotonicity and contraction of the mapping, as stated for FIB.
A dropped O factor fails the uninformative case, a max taken outside the
sum over z fails the perfect-sensor case, and a wrong discount, reward or
transposed T fails all of them.
"""
import numpy as np
import pytest

import oracle
from paper_1810_00204_amd import workloads as wl
from tests import dense_model as dm
from tests.test_oracle_pins import _slip4_exact, _slip8_exact, corridor


def _vi(prob):
    Q, _, _ = oracle.value_iterate(prob, tol=1e-14)
    return Q


def _fib(prob, **kw):
    al, res, sw = oracle.fib_iterate(prob, tol=1e-14, **kw)
    return al


def _with_landmarks(prob, n, seed):
    rng = np.random.default_rng(seed)
    free = np.flatnonzero(prob.occ == 0)
    free = free[free != prob.goal]
    prob.lm_cell = rng.permutation(free)[:n].astype(np.int32)
    return prob


@pytest.mark.parametrize("seed", range(3))
def test_fib_perfect_sensor_is_qmdp(seed):
    prob = wl.make_small(seed=seed, W=7, H=6, frac=0.15)
    free = np.flatnonzero(prob.occ == 0)
    prob.lm_cell = free.astype(np.int32)
    prob.lm_p = 1.0
    prob.slip = _slip4_exact()
    Q = _vi(prob)
    al = _fib(prob)
    np.testing.assert_allclose(al, Q, rtol=1e-10, atol=1e-9)


def test_fib_perfect_sensor_is_qmdp_eight_actions():
    prob = wl.make_rect(seed=5, side=9, frac=0.2, n_landmarks=0, D=1, n=1)
    free = np.flatnonzero(prob.occ == 0)
    prob.lm_cell = free.astype(np.int32)
    prob.lm_p = 1.0
    prob.slip = _slip8_exact()
    np.testing.assert_allclose(_fib(prob), _vi(prob), rtol=1e-10, atol=1e-9)


def test_fib_corridor_with_distinct_readings_is_closed_form():
    """1 x 3 corridor, goal at x = 0, noiseless wall bits: the left bit reads
    1 only at x = 0 and the right bit only at x = 2, so every reading names
    its cell and FIB equals the corridor closed form V(1) = 79/(1 - 0.2 g),
    V(2) = c + (V(1) - c) rho with c = -1/(1 - g), rho = 0.8 g/(1 - 0.2 g)."""
    prob = corridor(3)
    prob.slip = _slip4_exact()
    prob.flip = np.zeros(4)
    prob.R = np.full((3, 4), -1.0)
    prob.R[0] = 0.0
    prob.R[1, 3] = -1.0 + 100 * 0.8
    m = oracle.Model(prob)
    g = float(np.float32(prob.gamma))
    al = _fib(prob)
    V1 = 79.0 / (1 - 0.2 * g)
    c = -1.0 / (1 - g)
    rho = 0.8 * g / (1 - 0.2 * g)
    np.testing.assert_allclose(al.max(axis=1), [0.0, V1, c + (V1 - c) * rho], rtol=1e-12,
                               atol=1e-12)
    assert m.S == 3


def test_fib_corridor_with_shared_readings_is_still_closed_form():
    """1 x 8 corridor, noiseless bits: cells 1..6 read alike, but moving west
    is the best action at every cell, so the max over a' in the FIB equation
    picks the same vector for every successor and FIB keeps the corridor
    closed form V(d) = c + (V(1) - c) rho^(d-1) of Q-MDP."""
    L = 8
    prob = corridor(L)
    prob.slip = _slip4_exact()
    prob.flip = np.zeros(4)
    prob.R = np.full((L, 4), -1.0)
    prob.R[0] = 0.0
    prob.R[1, 3] = -1.0 + 100 * 0.8
    g = float(np.float32(prob.gamma))
    al = _fib(prob)
    V1 = 79.0 / (1 - 0.2 * g)
    c = -1.0 / (1 - g)
    rho = 0.8 * g / (1 - 0.2 * g)
    d = np.arange(1, L)
    np.testing.assert_allclose(al.max(axis=1)[1:], c + (V1 - c) * rho ** (d - 1), rtol=1e-12)
    assert np.all(al[1:].argmax(axis=1) == 3)


@pytest.mark.parametrize("seed", range(2))
def test_fib_uninformative_sensor_reduces_to_open_loop_recursion(seed):
    prob = _with_landmarks(wl.make_small(seed=seed, W=6, H=6, frac=0.2), 0, seed)
    prob.flip = np.full(4, 0.5)
    prob.slip = _slip4_exact()
    T = dm.transition_matrices(prob)
    R = prob.R.astype(np.float64)
    g = float(np.float32(prob.gamma))
    occ = prob.occ.astype(bool)
    al = np.zeros_like(R)
    for _ in range(3000):
        nxt = np.stack([R[:, a] + g * np.max(np.stack([T[a] @ al[:, ap]
                                                        for ap in range(prob.A)]), axis=0)
                        for a in range(prob.A)], axis=1)
        nxt[occ] = 0.0
        if np.max(np.abs(nxt - al)) < 1e-13:
            al = nxt
            break
        al = nxt
    np.testing.assert_allclose(_fib(prob), al, rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("seed,lms", [(0, 0), (1, 6), (2, 12)])
def test_fib_between_blind_policies_and_qmdp(seed, lms):
    prob = _with_landmarks(wl.make_small(seed=seed, W=8, H=7, frac=0.15), lms, seed)
    Q = _vi(prob)
    al = _fib(prob)
    T = dm.transition_matrices(prob)
    R = prob.R.astype(np.float64)
    g = float(np.float32(prob.gamma))
    free = prob.occ == 0
    assert np.all(al[free] <= Q[free] + 1e-9)
    V = al.max(axis=1)
    for a in range(prob.A):
        blind = np.linalg.solve(np.eye(prob.S) - g * T[a], R[:, a])
        assert np.all(V[free] >= blind[free] - 1e-9), a
    # the sensor carries information here, so the bound is strictly tighter
    assert np.max(Q[free] - al[free]) > 1e-3


def test_fib_mapping_is_monotone_and_contractive():
    prob = _with_landmarks(wl.make_small(seed=7, W=6, H=5, frac=0.15), 4, 7)
    cells = np.arange(prob.S)
    g = float(np.float32(prob.gamma))
    rng = np.random.default_rng(0)
    Q = _vi(prob)
    # starting from Q-MDP every sweep moves down
    a1 = oracle.fib_backup(prob, Q, cells)
    a2 = oracle.fib_backup(prob, a1, cells)
    free = prob.occ == 0
    assert np.all(a1[free] <= Q[free] + 1e-12)
    assert np.all(a2[free] <= a1[free] + 1e-12)
    for _ in range(5):
        x = rng.normal(0, 10, size=(prob.S, prob.A))
        y = x + rng.normal(0, 1, size=x.shape)
        hx = oracle.fib_backup(prob, x, cells)
        hy = oracle.fib_backup(prob, y, cells)
        assert np.max(np.abs(hx - hy)) <= g * np.max(np.abs(x - y)[free]) + 1e-12
        # monotone: y >= x componentwise gives H y >= H x
        yy = x + np.abs(rng.normal(0, 1, size=x.shape))
        assert np.all(oracle.fib_backup(prob, yy, cells) >= hx - 1e-12)


def test_fib_iteration_from_qmdp_converges_to_same_bound():
    prob = _with_landmarks(wl.make_small(seed=2, W=7, H=7, frac=0.2), 5, 2)
    a0 = _fib(prob)
    a1 = _fib(prob, init=_vi(prob))
    np.testing.assert_allclose(a1, a0, rtol=1e-10, atol=1e-9)
    # and its backup reproduces it (fixed point)
    back = oracle.fib_backup(prob, a0, np.arange(prob.S))
    np.testing.assert_allclose(back, a0, rtol=1e-11, atol=1e-10)
