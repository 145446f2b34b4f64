"""Pins of the oracle's point-based value iteration (Sec. IV-B, the PBVI
alpha-vector equation and the belief-set expansion it follows), CPU only.

* the successor gather T_a v equals the dense transition matrices of
  tests/dense_model.py (built independently of the oracle);
* one backup at each point equals the PBVI equation evaluated by brute force
  with the dense T and O matrices: max_a [R(b,a) + gamma sum_z max_alpha
  sum_x sum_x' O(x',z) T(x,a,x') alpha(x') b(x)] (a wrong z sum, a
  transposed T or a missing gamma fails it);
* with every free cell a point (the vertices delta_x) and a perfect sensor,
  the backups are the MDP Bellman operator at the vertices and converge to
  the Q-MDP fixed point;
* the values stay between the blind-policy lower bound (from which they
  start and which they can only raise at the points) and FIB;
* expansion adds posteriors Phi(b,a,z) of existing points, at positive L1
  distance from the set.
"""
import numpy as np
import pytest

import oracle
from paper_1810_00204_amd import workloads as wl
from tests import dense_model as dm


def test_successor_gather_is_the_transition_matrix():
    prob = wl.make_small(seed=3, W=7, H=6)
    T = dm.transition_matrices(prob)
    t = oracle.PBVI(prob, np.zeros((prob.S, 1)), 1)
    v = np.random.default_rng(0).random(prob.S)
    free = prob.occ == 0
    for a in range(prob.A):
        np.testing.assert_allclose(t._apply_T(a, v)[free], (T[a] @ v)[free], rtol=0, atol=1e-15)


@pytest.mark.parametrize("maker", ["small", "landmarks"])
def test_backup_is_the_pbvi_equation(maker):
    if maker == "small":
        prob = wl.make_small(seed=4, W=6, H=5)
    else:
        prob = wl.make_rect(seed=7, side=7, frac=0.2, side_lo=1, side_hi=2, n_landmarks=4,
                            D=1, n=1)
    L, _, _ = oracle.blind_iterate(prob, tol=1e-13)
    t = oracle.PBVI(prob, L, seed=3)
    t.expand()
    t.expand()
    G0 = t.Gamma.copy()
    t.backup()
    T = dm.transition_matrices(prob)
    O = dm.observation_matrix(prob)
    R = np.asarray(prob.R, np.float64)
    g = float(np.float32(prob.gamma))
    for i, b in enumerate(t.B):
        best = -np.inf
        for a in range(prob.A):
            v = b @ R[:, a]
            for z in range(O.shape[1]):
                # sum_x sum_x' O(x',z) T(x,a,x') alpha(x') b(x), for every alpha
                vals = (b @ T[a]) * O[:, z] @ G0
                v += g * vals.max()
            best = max(best, v)
        assert b @ t.Gamma[:, i] == pytest.approx(best, rel=1e-11, abs=1e-9), i


def test_vertices_with_a_perfect_sensor_reach_qmdp():
    prob = wl.make_small(seed=5, W=6, H=5, frac=0.15)
    free = np.flatnonzero(prob.occ == 0)
    prob.lm_cell = free.astype(np.int32)
    prob.lm_p = 1.0
    L, _, _ = oracle.blind_iterate(prob, tol=1e-13)
    t = oracle.PBVI(prob, L, seed=1)
    t.B = [np.eye(prob.S)[x] for x in free]
    for _ in range(400):
        t.backup()
    Q, _, _ = oracle.value_iterate(prob, tol=1e-13)
    V = np.array([t.value(np.eye(prob.S)[x]) for x in free])
    np.testing.assert_allclose(V, Q[free].max(1), rtol=1e-8, atol=1e-6)


@pytest.mark.parametrize("seed", range(2))
def test_values_lie_between_blind_and_fib(seed):
    """Every vector is a policy's value, so V_PBVI <= V* <= V_FIB at any
    belief; the first backup from the blind vectors (which satisfy
    alpha^a = R_a + gamma T_a alpha^a, so a Bellman backup cannot lower them)
    raises or keeps every point's value."""
    prob = wl.make_small(seed=seed, W=8, H=7)
    L, _, _ = oracle.blind_iterate(prob, tol=1e-13)
    U, _, _ = oracle.fib_iterate(prob, tol=1e-13)
    t = oracle.PBVI(prob, L, seed=9)
    t.expand()
    before = [t.value(b) for b in t.B]
    t.backup()
    after = [t.value(b) for b in t.B]
    assert all(x >= y - 1e-9 for x, y in zip(after, before))
    for _ in range(2):
        t.expand()
        t.backup()
    rng = np.random.default_rng(2)
    tests = list(t.B) + [rng.dirichlet(np.ones(prob.S)) * (prob.occ == 0) for _ in range(20)]
    for b in tests:
        b = b / b.sum()
        assert t.value(b) <= float(np.max(b @ U)) + 1e-9
    # at corner beliefs: alpha_j(x) <= V*(e_x) <= max_a U(x, a) for every vector
    free = np.asarray(prob.occ).reshape(-1) == 0
    assert np.all(t.Gamma[free] <= U[free].max(1)[:, None] + 1e-9)


def test_expansion_adds_posteriors_of_points():
    prob = wl.make_small(seed=6, W=8, H=6)
    L, _, _ = oracle.blind_iterate(prob, tol=1e-13)
    t = oracle.PBVI(prob, L, seed=4)
    old = list(t.B)
    added = t.expand()
    assert added == len(t.B) - len(old) and added >= 1
    for nb in t.B[len(old):]:
        found = False
        for b in old:
            for a in range(prob.A):
                bp = oracle.predict(prob, b, a)
                p = oracle.likelihood(prob, bp)
                for z in np.flatnonzero(p > 0):
                    post, pz, st = oracle.belief_update(prob, b, a, z)
                    if np.abs(post[0] - nb).max() < 1e-12:
                        found = True
        assert found
        assert min(np.abs(nb - b).sum() for b in old) > 0
