"""Pins of the oracle's best-first search (Alg. 1, 2, 5, 6, 7 with the
heuristics of Sec. IV-C) and of its blind-policy lower bound, CPU only.

* the blind-policy vectors equal each action's policy value solved densely
  with numpy.linalg.solve (matrices built independently of the oracle);
* after one expansion, the root's upper and lower bounds equal the depth-1
  plan of the oracle with the U and L tables as leaf tables (the plan is
  pinned against brute-force Bellman recursion elsewhere), so the Q-node
  backup (R, gamma, weights f/n) is the plan's;
* E and H at the root equal a brute-force search over every unexpanded node:
  the product of gamma * weight along its path times its U - L, over paths
  that take at each expanded node the action of largest U_Q (the AEMS
  propagation of Sec. IV-C); a wrong weight, a dropped gamma or a max over
  the wrong set fails it;
* U >= L at every node (FIB >= blind at the leaves and both backups are the
  same monotone operator);
* update(a, z) keeps the child's subtree when z was drawn, and otherwise
  roots a new node at the filter's posterior.
"""
import numpy as np
import pytest

import oracle
from paper_1810_00204_amd import workloads as wl
from tests import dense_model as dm


def _bounds(prob):
    U, _, _ = oracle.fib_iterate(prob, tol=1e-12)
    L, _, _ = oracle.blind_iterate(prob, tol=1e-12)
    return U, L


@pytest.mark.parametrize("seed", range(3))
def test_blind_bound_is_each_actions_policy_value(seed):
    prob = wl.make_small(seed=seed, W=7, H=6)
    al, res, sw = oracle.blind_iterate(prob, tol=1e-14)
    T = dm.transition_matrices(prob)
    R = np.asarray(prob.R, np.float64)
    g = float(np.float32(prob.gamma))
    free = prob.occ == 0
    for a in range(prob.A):
        v = np.linalg.solve(np.eye(prob.S) - g * T[a], R[:, a])
        np.testing.assert_allclose(al[free, a], v[free], rtol=1e-9, atol=1e-9)
    Q, _, _ = oracle.value_iterate(prob, tol=1e-14)
    assert np.all(al <= Q + 1e-9)


@pytest.mark.parametrize("maker", ["small", "rect"])
def test_first_expansion_equals_depth_one_plan(maker):
    prob = (wl.make_small(seed=4) if maker == "small"
            else wl.make_rect(seed=5, side=16, n_landmarks=6, D=1, n=3))
    U, L = _bounds(prob)
    t = oracle.search(prob, U, L, 1)
    root = t.nodes[t.root]
    pu = oracle.plan(prob, U, D=1)
    pl = oracle.plan(prob, L, D=1)
    np.testing.assert_allclose(root["q"]["UQ"], pu["rootQ"], rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(root["q"]["LQ"], pl["rootQ"], rtol=1e-12, atol=1e-10)
    assert root["U"] == pytest.approx(pu["rootQ"].max(), abs=1e-10)
    assert root["L"] == pytest.approx(pl["rootQ"].max(), abs=1e-10)


def _brute_force_selection(t):
    """max over unexpanded nodes of H_leaf * prod(gamma * w) along the path
    that follows the action of largest U_Q at each expanded ancestor."""
    best, arg = -np.inf, None
    stack = [(t.root, 1.0)]
    while stack:
        v, f = stack.pop()
        nd = t.nodes[v]
        if nd["q"] is None:
            val = f * nd["H"]
            if val > best + 1e-15 or (abs(val - best) <= 1e-15 and (arg is None or v < arg)):
                best, arg = val, v
            continue
        a = int(np.argmax(nd["q"]["UQ"]))
        for c in nd["kids"][a]:
            stack.append((c, f * t.g * t.nodes[c]["w"]))
    return best, arg


@pytest.mark.parametrize("seed,steps", [(0, 5), (1, 25), (2, 60)])
def test_root_heuristic_is_the_brute_force_best_leaf(seed, steps):
    prob = wl.make_small(seed=seed, D=2, n=3)
    U, L = _bounds(prob)
    t = oracle.search(prob, U, L, steps)
    best, arg = _brute_force_selection(t)
    root = t.nodes[t.root]
    assert root["H"] == pytest.approx(best, rel=1e-12, abs=1e-15)
    assert t.nodes[root["E"]]["q"] is None
    # the node the root points to attains the best value (ties: any of them)
    v = root["E"]
    f = 1.0
    while t.nodes[v]["parent"] is not None:
        p, a = t.nodes[v]["parent"]
        f *= t.g * t.nodes[v]["w"]
        assert a == int(np.argmax(t.nodes[p]["q"]["UQ"]))
        v = p
    assert f * t.nodes[root["E"]]["H"] == pytest.approx(best, rel=1e-12, abs=1e-15)
    for nd in t.nodes.values():
        assert nd["U"] >= nd["L"] - 1e-9
    assert len(t.log) == steps and len(set(t.log)) == steps   # each node expanded once


def test_update_keeps_the_subtree_or_roots_the_posterior():
    prob = wl.make_small(seed=6, D=2, n=2)
    U, L = _bounds(prob)
    t = oracle.search(prob, U, L, 12)
    root = t.nodes[t.root]
    a = int(np.argmax(root["q"]["UQ"]))
    c = root["kids"][a][0]
    z = t.nodes[c]["z"]
    assert t.update(a, z) == c and t.root == c and t.nodes[c]["parent"] is None
    # an observation that was not drawn: a new root at Phi(b, a, z)
    nd = t.nodes[t.root]
    drawn = set()
    if nd["q"] is not None:
        drawn = {t.nodes[k]["z"] for k in nd["kids"][0]}
    bp = nd["b"] @ dm.transition_matrices(prob)[0]
    pz = bp @ dm.observation_matrix(prob)
    z2 = int(next(z for z in np.argsort(-pz) if z not in drawn and pz[z] > 0))
    nid = t.update(0, z2)
    assert nid == t.next - 1 and t.root == nid
    O = dm.observation_matrix(prob)
    post = O[:, z2] * bp / pz[z2]
    np.testing.assert_allclose(t.nodes[nid]["b"], post, atol=1e-14)
    assert t.nodes[nid]["U"] == pytest.approx(float(np.max(post @ U)), rel=1e-12)
