"""GPU parity of batched planning (qv_batch_*) through the C ABI: against
single-query plans of the same queries (bit for bit at the default shape),
against the FP64 oracle, across graph replays and after autotuning."""
import numpy as np
import pytest

import oracle
from paper_1810_00204_amd import binding as B
from paper_1810_00204_amd import workloads as wl
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEED = 0x5EED1810


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _q32(prob):
    Q, _, _ = oracle.value_iterate(prob, tol=1e-10)
    return Q.astype(np.float32)


def _gpu_q(prob):
    """Q-MDP table from the library's own value iteration (the batch and the
    single-query plans it is compared with read the same table)."""
    m = B.DeviceModel(prob)
    Q = torch.empty(m.S * m.A, dtype=torch.float32, device="cuda")
    ws = torch.empty(B.qv_vi_workspace_bytes(m, 10000), dtype=torch.uint8, device="cuda")
    st, _, _ = B.qv_value_iterate(m, 1e-6, 10000, Q, ws)
    B.check(st, "qv_value_iterate")
    return Q


def _same_tree(t1, t2):
    """Every record a plan writes: existence, z, counts and P(z) of all
    slots; values of existing nodes; Q-values and rewards of existing
    non-leaf nodes (entries of absent nodes are never written)."""
    for k in ("valid", "z", "count", "pz"):
        assert np.array_equal(t1[k], t2[k]), k
    v = t1["valid"] == 1
    assert np.array_equal(t1["value"][v], t2["value"][v]), "value"
    inner = v.copy()
    inner[t1["level_first"][-2]:] = False
    A = t1["qvalue"].size // v.size
    m = np.repeat(inner, A)
    for k in ("qvalue", "reward"):
        assert np.array_equal(t1[k][m], t2[k][m]), k


def _single(prob, Q, q):
    from paper_1810_00204_amd.planner import Planner
    pl = Planner(prob, flags=B.QV_PLAN_TILED)
    Qd = Q if hasattr(Q, "data_ptr") else torch.as_tensor(Q.reshape(-1)).cuda()
    act, rq = pl.plan(Qd, seed=SEED, query_id=q)
    torch.cuda.synchronize()
    return pl.tree(beliefs=False), int(act.item()), rq.cpu().numpy()


def _mixed_batch():
    """Square and ragged grids, 4 and 8 actions, with and without landmarks,
    depths 1..3."""
    probs = wl.make_batch(seed=3, nq=6, side_lo=8, side_hi=24)
    probs.append(wl.make_small(seed=21, W=31, H=9, D=3, n=3, query_id=len(probs)))
    r = wl.make_rect(seed=22, side=20, n_landmarks=6, D=2, n=3)
    probs.append(r)
    probs.append(wl.make_small(seed=23, W=7, H=13, D=1, n=3))
    return probs


def test_batch_equals_single_query_plans():
    _say("batch of 9 mixed queries vs single-query plans")
    from paper_1810_00204_amd.planner import BatchPlanner
    probs = _mixed_batch()
    Qs = [_q32(p) for p in probs]
    bp = BatchPlanner(probs, Qs, n=3)
    acts, rq = bp.plan(SEED)
    acts = acts.cpu().numpy()
    rq = rq.cpu().numpy()
    for q, p in enumerate(probs):
        t1, a1, r1 = _single(p, Qs[q], q)
        _same_tree(bp.tree(q), t1)
        assert acts[q] == a1
        assert np.array_equal(rq[q, :p.A], r1)
        assert not rq[q, p.A:].any()


def test_batch_matches_oracle():
    _say("batch vs oracle")
    from paper_1810_00204_amd.planner import BatchPlanner
    probs = _mixed_batch()
    Qs = [_q32(p) for p in probs]
    bp = BatchPlanner(probs, Qs, n=3)
    acts, rq = bp.plan(SEED)
    acts = acts.cpu().numpy()
    rq = rq.cpu().numpy()
    for q, p in enumerate(probs):
        p.n = 3
        res = oracle.plan(p, Qs[q], seed=SEED, qid=q)
        rep = parity.compare_tree(p, bp.tree(q), res["dump"], check_beliefs=False)
        assert parity.root_action_ok(int(acts[q]), res["rootQ"], res["action"])
        if not rep.excused:
            np.testing.assert_allclose(rq[q, :p.A], res["rootQ"], rtol=0,
                                       atol=parity.REL * max(1.0, np.abs(res["rootQ"]).max()))


def test_batch_graph_replays_match_eager():
    """Graph replays, with eager work of the program in between, give the
    eager batch's results on every replay."""
    _say("batch graph replays")
    from paper_1810_00204_amd.planner import BatchPlanner
    probs = _mixed_batch()
    Qs = [_q32(p) for p in probs]
    eager = BatchPlanner(probs, Qs, n=3)
    ea, er = eager.plan(SEED)
    ea, er = ea.cpu().numpy().copy(), er.cpu().numpy().copy()
    etrees = [eager.tree(q) for q in range(len(probs))]
    graph = BatchPlanner(probs, Qs, n=3, flags=B.QV_BATCH_GRAPH)
    for rep in range(3):
        ga, gr = graph.plan(SEED)
        torch.cuda.synchronize()
        assert np.array_equal(ga.cpu().numpy(), ea), rep
        assert np.array_equal(gr.cpu().numpy(), er), rep
        for q in range(len(probs)):
            _same_tree(graph.tree(q), etrees[q])
        # eager work between replays: a single-query plan and a batch plan
        _single(probs[rep], Qs[rep], rep)
        eager.plan(SEED + 1)
        torch.cuda.synchronize()


def test_batch_new_inputs_between_graph_replays():
    """A replay reads the start beliefs and Q tables of its own call."""
    _say("batch graph with new beliefs")
    from paper_1810_00204_amd.planner import BatchPlanner
    probs = wl.make_batch(seed=4, nq=5, side_lo=8, side_hi=20)
    Qs = [_q32(p) for p in probs]
    graph = BatchPlanner(probs, Qs, n=3, flags=B.QV_BATCH_GRAPH)
    graph.plan(SEED)
    rng = np.random.default_rng(0)
    for p, b in zip(probs, graph.b0s):
        free = np.flatnonzero(p.occ == 0)
        cells = rng.choice(free, size=3, replace=False)
        nb = wl.belief_uniform_cells(p.W * p.H, cells)
        b.copy_(torch.as_tensor(nb))
        p.b0 = nb
    graph.plan(SEED)
    for q, p in enumerate(probs):
        t1, _, _ = _single(p, Qs[q], q)
        _same_tree(graph.tree(q), t1)


def test_batch_autotune_keeps_parity():
    _say("batch autotune")
    from paper_1810_00204_amd.planner import BatchPlanner
    probs = wl.make_batch(seed=5, nq=8, side_lo=16, side_hi=40)
    Qs = [_q32(p) for p in probs]
    bp = BatchPlanner(probs, Qs, n=3, flags=B.QV_BATCH_GRAPH)
    ms = bp.autotune(SEED, reps=2)
    assert ms > 0
    tc, ch = bp.shape()
    print(f"chosen shape: {tc} cells per band, {ch} items per visit, {ms:.3f} ms")
    acts, _ = bp.plan(SEED)
    acts = acts.cpu().numpy()
    for q, p in enumerate(probs):
        res = oracle.plan(p, Qs[q], seed=SEED, qid=q)
        parity.compare_tree(p, bp.tree(q), res["dump"], check_beliefs=False)
        assert parity.root_action_ok(int(acts[q]), res["rootQ"], res["action"])
    a2, _ = bp.plan(SEED)
    assert np.array_equal(a2.cpu().numpy(), acts)


def test_batch_autotune_shape_cache(tmp_path):
    """A second batch of the same key takes the cached shape without timing
    and plans exactly as the tuned one."""
    _say("batch autotune cache")
    from paper_1810_00204_amd.planner import BatchPlanner
    probs = wl.make_batch(seed=6, nq=6, side_lo=16, side_hi=32)
    Qs = [_q32(p) for p in probs]
    cache = str(tmp_path / "shapes.json")
    bp1 = BatchPlanner(probs, Qs, n=3, flags=B.QV_BATCH_GRAPH)
    ms1 = bp1.autotune(SEED, reps=2, cache=cache)
    assert not bp1.tuned_from_cache and ms1 > 0
    a1, r1 = bp1.plan(SEED)
    a1, r1 = a1.cpu().numpy().copy(), r1.cpu().numpy().copy()
    bp2 = BatchPlanner(probs, Qs, n=3, flags=B.QV_BATCH_GRAPH)
    ms2 = bp2.autotune(SEED, reps=2, cache=cache)
    assert bp2.tuned_from_cache and ms2 == ms1
    assert bp2.shape() == bp1.shape()
    a2, r2 = bp2.plan(SEED)
    assert np.array_equal(a2.cpu().numpy(), a1)
    assert np.array_equal(r2.cpu().numpy(), r1)
    for q in range(len(probs)):
        _same_tree(bp2.tree(q), bp1.tree(q))


@pytest.mark.parametrize("shape", [(256, 1), (4096, 4), (512, 2)])
def test_batch_shapes_match_oracle(shape):
    _say(f"batch shape {shape}")
    from paper_1810_00204_amd.planner import BatchPlanner
    probs = _mixed_batch()
    Qs = [_q32(p) for p in probs]
    bp = BatchPlanner(probs, Qs, n=3)
    bp.set_shape(*shape)
    assert bp.shape() == shape
    acts, _ = bp.plan(SEED)
    acts = acts.cpu().numpy()
    for q, p in enumerate(probs):
        p.n = 3
        res = oracle.plan(p, Qs[q], seed=SEED, qid=q)
        parity.compare_tree(p, bp.tree(q), res["dump"], check_beliefs=False)
        assert parity.root_action_ok(int(acts[q]), res["rootQ"], res["action"])


def test_batch_single_query():
    _say("batch of one")
    from paper_1810_00204_amd.planner import BatchPlanner
    p = wl.make_small(seed=30, W=12, H=12, D=2, n=3)
    Q = _q32(p)
    bp = BatchPlanner([p], [Q], n=3)
    bp.plan(SEED)
    t1, _, _ = _single(p, Q, 0)
    _same_tree(bp.tree(0), t1)


def test_batch_full_size_sampled_queries():
    """256 queries, sides 32..256, depth 2-3, 3 samples: sampled queries
    against single-query plans, bit for bit."""
    _say("batch 256 queries sides 32..256")
    from paper_1810_00204_amd.planner import BatchPlanner
    probs = wl.make_batch(seed=0)
    Qs = [_gpu_q(p) for p in probs]
    bp = BatchPlanner(probs, Qs, n=3, flags=B.QV_BATCH_GRAPH)
    acts, rq = bp.plan(SEED)
    torch.cuda.synchronize()
    sides = np.array([p.W for p in probs])
    picks = sorted({int(np.argmin(sides)), int(np.argmax(sides)), 0, 127, 255})
    acts = acts.cpu().numpy()
    for q in picks:
        t1, a1, _ = _single(probs[q], Qs[q], q)
        _same_tree(bp.tree(q), t1)
        assert acts[q] == a1
    assert np.all((acts >= 0) & (acts < 4))


def test_batch_rejects_bad_arguments():
    _say("batch argument checks")
    p = wl.make_small(seed=31)
    m = B.DeviceModel(p)
    st, _ = B.qv_batch_create([m], [0], 3)
    assert st == B.QV_ERR_INVALID_ARG
    st, _ = B.qv_batch_create([m], [2], 0)
    assert st == B.QV_ERR_INVALID_ARG
    st, h = B.qv_batch_create([m], [2], 3)
    assert st == B.QV_OK
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    Q = torch.zeros(p.W * p.H * 4, device="cuda")
    b0 = torch.as_tensor(p.b0).cuda()
    acts = torch.zeros(1, dtype=torch.int32, device="cuda")
    rq = torch.zeros(B.QV_MAX_ACTIONS, device="cuda")
    assert B.qv_batch_plan(h, [Q], [b0], 1, acts, rq, ws) == B.QV_ERR_WORKSPACE
    assert B.qv_batch_set_shape(h, 1024, 0) == B.QV_ERR_INVALID_ARG
    assert B.qv_batch_destroy(h) == B.QV_OK
