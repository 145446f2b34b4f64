"""GPU parity of the planning path against the FP64 oracle (MI355X).

All calls go through the C ABI of libqvts.so.  Inputs are the seeded
workloads; the oracle and the GPU receive identical values (the oracle
widens the FP32 inputs exactly), and the Q table comes from the oracle's
own FP64 value iteration rounded to FP32."""
import os

import numpy as np
import pytest

import oracle
from paper_1810_00204_amd import binding as B
from paper_1810_00204_amd import workloads as wl
from tests import parity

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _q32(prob):
    Q, _, _ = oracle.value_iterate(prob, tol=1e-10)
    return Q.astype(np.float32)


def _run(prob, Q32, flags=0, D=None, n=None):
    from paper_1810_00204_amd.planner import Planner
    pl = Planner(prob, flags=flags, D=D, n=n)
    Qd = torch.as_tensor(Q32.reshape(-1)).cuda()
    act, rq = pl.plan(Qd)
    torch.cuda.synchronize()
    return pl, int(act.item()), rq.cpu().numpy()


def _check(prob, Q32, flags=0, beliefs=True):
    if prob.D == 0:
        beliefs = False
    pl, act, rq = _run(prob, Q32, flags)
    g = pl.tree(beliefs=beliefs)
    res = oracle.plan(prob, Q32, dump_beliefs=beliefs)
    rep = parity.compare_tree(prob, g, res["dump"], check_beliefs=beliefs)
    assert parity.root_action_ok(act, res["rootQ"], res["action"]), (act, res["action"], res["rootQ"])
    if not rep.excused:
        np.testing.assert_allclose(rq, res["rootQ"], rtol=0,
                                   atol=parity.REL * max(1.0, np.abs(res["rootQ"]).max()))
    return rep


PATHS = {"node": 0, "banded": B.QV_PLAN_TILED}


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("seed", range(100))
def test_plan_matches_oracle_small_grid(seed, path):
    _say(f"plan 10x10 4 actions D=2 n=2 seed={seed} path={path}")
    prob = wl.make_small(seed=seed)
    rep = _check(prob, _q32(prob), flags=PATHS[path])
    assert rep.nodes > 1
    assert len(rep.excused) <= 1


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("seed", range(10))
def test_plan_matches_oracle_rect_grid(seed, path):
    """64x64 rectangles, 8 actions, 32 landmarks, depth 3, 4 samples."""
    _say(f"plan 64x64 8 actions L=32 D=3 n=4 seed={seed} path={path}")
    prob = wl.make_rect(seed=seed)
    rep = _check(prob, _q32(prob), flags=PATHS[path])
    assert rep.nodes > 100
    assert len(rep.excused) <= 3


@pytest.mark.parametrize("side", [78, 82, 84, 88])
def test_plan_near_fused_path_lds_limit(side):
    """Square grids on both sides of the largest one the fused per-Q-node
    path holds in LDS (the path switches to the banded kernels above it)."""
    _say(f"plan {side}x{side} 8 actions L=32 D=2 n=2")
    prob = wl.make_rect(seed=side, side=side, D=2, n=2)
    rep = _check(prob, _q32(prob), beliefs=False)
    assert rep.nodes > 1


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("case", ["depth0", "depth1", "n1", "ragged", "corridor", "goal_in_belief",
                                  "landmark_obs", "deep", "nine_actions", "many_samples"])
def test_plan_edge_cases(case, path):
    _say(f"plan edge case {case} path={path}")
    if case == "depth0":
        prob = wl.make_small(seed=3, D=0)
    elif case == "depth1":
        prob = wl.make_rect(seed=4, side=24, n_landmarks=6, D=1, n=5)
    elif case == "n1":
        prob = wl.make_small(seed=5, D=3, n=1)
    elif case == "ragged":
        # 50 x 97: bands of 20 rows, the last one 17 rows
        prob = wl.make_small(seed=6, W=50, H=97, D=2, n=2)
    elif case == "corridor":
        prob = wl.make_small(seed=7, W=40, H=1, frac=0.0, D=2, n=3)
    elif case == "goal_in_belief":
        prob = wl.make_small(seed=8)
        b = prob.b0.astype(np.float64) * 0.5
        b[prob.goal] += 0.5
        prob.b0 = b.astype(np.float32)
    elif case == "landmark_obs":
        prob = wl.make_rect(seed=9, side=12, n_landmarks=20, D=2, n=3)
        prob.lm_p = 0.6
    elif case == "nine_actions":
        # the 8-neighbour set plus "stay" (A = 9, the action set of Sec. V)
        prob = wl.make_rect(seed=14, side=16, n_landmarks=4, D=2, n=2)
        stay = np.zeros((1, 9), np.float32)
        stay[0, 4] = 1.0
        prob.slip = np.concatenate([prob.slip, stay])
        prob.R = wl.reward_step_goal(prob.occ, prob.W, prob.H, prob.slip, prob.goal)
    elif case == "many_samples":
        prob = wl.make_small(seed=15, W=12, H=9, D=2, n=16)
    else:
        prob = wl.make_small(seed=10, W=6, H=5, D=4, n=1)
    _check(prob, _q32(prob), flags=PATHS[path])


def test_plan_store_leaves_matches_fused_scoring():
    _say("plan stored leaves vs fused leaf scoring")
    prob = wl.make_rect(seed=11, side=32, n_landmarks=8, D=2, n=3)
    Q32 = _q32(prob)
    p1, a1, q1 = _run(prob, Q32, flags=0)
    p2, a2, q2 = _run(prob, Q32, flags=B.QV_PLAN_STORE_LEAVES)
    t1, t2 = p1.tree(beliefs=False), p2.tree()
    assert a1 == a2
    for k in ("valid", "z", "count"):
        assert np.array_equal(t1[k], t2[k])
    # the fused path scores leaves from wall-reading histograms, the stored
    # path cell by cell: the same sums in another order
    v1, v2 = t1["value"][t1["valid"] == 1], t2["value"][t2["valid"] == 1]
    assert np.all(np.abs(v1 - v2) <= parity.REL * np.maximum(1.0, np.abs(v2)))
    # the stored leaves match the oracle's leaf beliefs
    res = oracle.plan(prob, Q32, dump_beliefs=True)
    parity.compare_tree(prob, t2, res["dump"])


@pytest.mark.parametrize("path", list(PATHS))
def test_plan_is_bitwise_deterministic(path):
    _say(f"plan determinism 64x64 path={path}")
    prob = wl.make_rect(seed=12)
    Q32 = _q32(prob)
    p1, a1, q1 = _run(prob, Q32, flags=PATHS[path])
    t1 = p1.tree(beliefs=True)
    p1.plan(torch.as_tensor(Q32.reshape(-1)).cuda())
    t2 = p1.tree(beliefs=True)
    for k in ("valid", "z", "count", "pz", "value", "qvalue", "reward"):
        assert np.array_equal(t1[k], t2[k]), k
    for d in t1["beliefs"]:
        assert np.array_equal(t1["beliefs"][d], t2["beliefs"][d])


def test_plan_with_roctx_ranges_is_unchanged(tmp_path):
    """QVTS_ROCTX=1 brackets the plan and its levels with roctx ranges; the
    plan it makes (in a process of its own, since the switch is read once)
    is the one made without them."""
    _say("plan with roctx ranges")
    import subprocess
    import sys
    prob = wl.make_rect(seed=14, side=40, D=3, n=2)
    Q32 = _q32(prob)
    _, a1, q1 = _run(prob, Q32, flags=0)
    np.save(tmp_path / "q.npy", Q32)
    code = (
        "import numpy as np, torch\n"
        "from paper_1810_00204_amd import workloads as wl\n"
        "from paper_1810_00204_amd.planner import Planner\n"
        "prob = wl.make_rect(seed=14, side=40, D=3, n=2)\n"
        f"Q = np.load({str(tmp_path / 'q.npy')!r})\n"
        "pl = Planner(prob)\n"
        "a, rq = pl.plan(torch.as_tensor(Q.reshape(-1)).cuda())\n"
        "torch.cuda.synchronize()\n"
        f"np.save({str(tmp_path / 'rq.npy')!r}, rq.cpu().numpy())\n"
        "print('action', int(a.item()))\n")
    env = dict(os.environ, QVTS_ROCTX="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    assert f"action {a1}" in r.stdout
    assert np.array_equal(np.load(tmp_path / "rq.npy"), q1)


def test_plan_seed_and_query_id_change_the_draws():
    _say("plan seed/query id")
    prob = wl.make_small(seed=13, D=2, n=3)
    Q32 = _q32(prob)
    from paper_1810_00204_amd.planner import Planner
    pl = Planner(prob)
    Qd = torch.as_tensor(Q32.reshape(-1)).cuda()
    zs = []
    for seed, qid in ((1, 0), (2, 0), (1, 5)):
        pl.plan(Qd, seed=seed, query_id=qid)
        zs.append(pl.tree(beliefs=False)["z"].copy())
        res = oracle.plan(prob, Q32, seed=seed, qid=qid)
        g = pl.tree(beliefs=False)
        parity.compare_tree(prob, g, res["dump"], check_beliefs=False)
    assert not np.array_equal(zs[0], zs[1]) and not np.array_equal(zs[0], zs[2])


def test_plan_large_grid_sampled_nodes():
    """512 x 512 with 256 landmarks, depth 3, 3 samples: sampled nodes are
    checked one by one against the oracle's expansion of its own parent
    belief; every stored belief is checked for the invariants."""
    _say("plan 512x512 8 actions L=256 D=3 n=3")
    prob = wl.make_large(seed=0)
    # Q: a seeded stand-in table (the leaf score is linear in Q; parity does
    # not depend on Q being converged)
    rng = np.random.default_rng(5)
    Q32 = (rng.standard_normal((prob.S, prob.A)) * 10).astype(np.float32)
    Q32[prob.occ == 1] = 0.0
    pl, act, rq = _run(prob, Q32)
    g = pl.tree(beliefs=False)
    lf, K, A, n, S = g["level_first"], prob.K, prob.A, prob.n, prob.S
    # root expansion
    root = oracle.expand_node(prob, prob.b0, 0, 0)
    _match_expansion(g, lf, 0, 0, root, K, A, n)
    # two level-1 nodes and, under one of them, one level-2 node
    valid1 = np.flatnonzero(root["valid"])
    picks = [int(valid1[0]), int(valid1[-1])]
    for s1 in picks:
        gb = pl.belief_of(1, s1).astype(np.float64)
        ob = root["beliefs"][s1]
        _belief_close(gb, ob)
        e1 = oracle.expand_node(prob, ob, 1, s1, beliefs=(s1 == picks[0]))
        _match_expansion(g, lf, 1, s1, e1, K, A, n)
        if s1 == picks[0]:
            v2 = np.flatnonzero(e1["valid"])
            s2loc = int(v2[len(v2) // 2])
            s2 = s1 * K + s2loc
            gb2 = pl.belief_of(2, s2).astype(np.float64)
            _belief_close(gb2, e1["beliefs"][s2loc])
            e2 = oracle.expand_node(prob, e1["beliefs"][s2loc], 2, s2, beliefs=True)
            _match_expansion(g, lf, 2, s2, e2, K, A, n)
            # leaf values of that node's children
            for c in np.flatnonzero(e2["valid"])[:6]:
                v = oracle.leaf_score(prob, Q32, e2["beliefs"][c])
                gv = g["value"][lf[3] + s2 * K + c]
                assert abs(gv - v) <= 1e-5 * max(1.0, abs(v)), (c, gv, v)
    # invariants on every stored belief of level 1
    for s1 in np.flatnonzero(g["valid"][lf[1]:lf[2]]):
        b = pl.belief_of(1, int(s1))
        assert abs(b.sum() - 1) < 1e-4 and b.min() >= 0 and np.all(b[prob.occ == 1] == 0)


def _match_expansion(g, lf, d, slot, e, K, A, n):
    kids = lf[d + 1] + slot * K + np.arange(K)
    for a in range(A):
        sl = slice(a * n, (a + 1) * n)
        same = (np.array_equal(g["valid"][kids][sl], e["valid"][sl])
                and np.array_equal(g["z"][kids][sl][e["valid"][sl] == 1], e["z"][sl][e["valid"][sl] == 1])
                and np.array_equal(g["count"][kids][sl][e["valid"][sl] == 1], e["count"][sl][e["valid"][sl] == 1]))
        if not same:
            assert e["margin"][sl].min() <= parity.DRAW_BAND, (d, slot, a)
            continue
        v = e["valid"][sl] == 1
        np.testing.assert_allclose(g["pz"][kids][sl][v], e["pz"][sl][v], rtol=1e-5)
    gs = lf[d] + slot
    np.testing.assert_allclose(g["reward"][gs * A:(gs + 1) * A], e["rb"], rtol=1e-5,
                               atol=1e-5 * max(1.0, np.abs(e["rb"]).max()))


def _belief_close(gb, ob):
    tol = 1e-5 * np.abs(ob) + 1e-12 * ob.max()
    bad = np.abs(gb - ob) > tol
    assert not bad.any(), (np.flatnonzero(bad)[:5], gb[bad][:5], ob[bad][:5])


@pytest.mark.parametrize("case", ["d3n2", "d4n1", "landmarks_goal"])
def test_plan_basis_inner_levels_match_oracle(case):
    """Grids beyond the one-workgroup-per-Q-node size with D >= 3 take the
    statistics of levels 1..D-2 from the basis pass over the sorted leaf bands
    with the rows of R in place of those of Q, and every child's reward from
    its parent's reward-weighted histograms (the last level then forms no
    R(b,a) of its own).  The whole tree against the oracle: draws, counts,
    P(z), rewards, beliefs, values and the root action."""
    _say(f"basis inner levels {case}")
    prob = {"d3n2": lambda: wl.make_rect(seed=31, side=112, D=3, n=2),
            "d4n1": lambda: wl.make_rect(seed=32, side=104, D=4, n=1),
            "landmarks_goal": lambda: wl.make_rect(seed=33, side=120, n_landmarks=60,
                                                   D=3, n=2, sigma=9.0)}[case]()
    Q32 = _q32(prob)
    rep = _check(prob, Q32, flags=0, beliefs=True)
    assert len(rep.excused) <= 2, rep.excused


@pytest.mark.parametrize("maker", ["rect64_tiled", "large"])
def test_per_parent_items_equal_per_action_items(maker, monkeypatch):
    """The banded inner levels with one workgroup per (parent, band) over all
    actions give bitwise the same tree as one workgroup per (parent, band,
    action): the same sums in the same order.  (QV_PLAN_TILED keeps these
    per-action statistics at every level; without it, levels 1..D-2 of a
    large grid take the basis pass instead, tested against the oracle below.)"""
    _say(f"per-parent vs per-action banded items {maker}")
    from paper_1810_00204_amd.planner import Planner
    if maker == "large":
        prob, flags = wl.make_large(seed=0), B.QV_PLAN_TILED
        rng = np.random.default_rng(5)
        Q32 = (rng.standard_normal((prob.S, prob.A)) * 10).astype(np.float32)
        Q32[prob.occ == 1] = 0.0
    else:
        prob, flags = wl.make_rect(seed=3), B.QV_PLAN_TILED
        Q32 = _q32(prob)
    Qd = torch.as_tensor(Q32.reshape(-1)).cuda()
    trees = []
    for env in ("0", "1"):
        monkeypatch.setenv("QVTS_PER_ACTION_ITEMS", env)
        pl = Planner(prob, flags=flags)
        pl.plan(Qd)
        t = pl.tree(beliefs=maker != "large")
        if maker == "large":
            t["b1"] = [pl.belief_of(1, int(s)) for s in np.flatnonzero(t["valid"][t["level_first"][1]:t["level_first"][2]])[:4]]
        trees.append((t, pl.action.item(), pl.rootQ.cpu().numpy()))
        del pl
    (t1, a1, q1), (t2, a2, q2) = trees
    assert a1 == a2 and np.array_equal(q1, q2)
    ok = t1["valid"] == 1
    assert np.array_equal(t1["valid"], t2["valid"])
    for k in ("z", "count", "pz", "value"):
        assert np.array_equal(t1[k][ok], t2[k][ok]), k
    if maker == "large":
        for x, y in zip(t1["b1"], t2["b1"]):
            assert np.array_equal(x, y)
    else:
        # rows of absent nodes are never written: compare the existing ones
        lf = t1["level_first"]
        for d in t1["beliefs"]:
            live = ok[lf[d]:lf[d] + t1["beliefs"][d].shape[0]]
            assert live.any()
            assert np.array_equal(t1["beliefs"][d][live], t2["beliefs"][d][live])
