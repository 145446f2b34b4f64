"""Device validation of the problem statement (the tuple of Sec. II: b0 must
lie in B(X), a distribution over the free cells), through the C ABI:
qv_model_check and the QV_PLAN_CHECK flag of qv_plan_step."""
import numpy as np
import pytest

from paper_1810_00204_amd import binding as B
from paper_1810_00204_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _check(prob, b0):
    m = B.DeviceModel(prob)
    ws = torch.empty(B.qv_check_workspace_bytes(), dtype=torch.uint8, device="cuda")
    bt = None if b0 is None else torch.as_tensor(np.ascontiguousarray(b0, np.float32)).cuda()
    return B.qv_model_check(m, bt, ws)


def _bad_beliefs(prob):
    b = prob.b0.astype(np.float32)
    free = np.flatnonzero(b > 0)
    out = {}
    x = b.copy(); x[free[0]] = -x[free[0]]; out["negative"] = x
    x = b.copy(); x[free[0]] = np.nan; out["nan"] = x
    x = b.copy(); x[free[0]] = np.inf; out["inf"] = x
    x = b.copy(); x[np.flatnonzero(prob.occ == 1)[0]] = 1e-3; out["blocked_mass"] = x
    out["sum_1.1"] = b * 1.1
    out["sum_0.99998"] = b * np.float32(0.99998)
    out["zero"] = np.zeros_like(b)
    return out


@pytest.mark.parametrize("maker", ["small", "large"])
def test_model_check_accepts_valid_and_rejects_invalid_beliefs(maker):
    _say(f"model check {maker}")
    prob = wl.make_small(seed=2) if maker == "small" else wl.make_large(seed=0)
    assert _check(prob, prob.b0) == B.QV_OK
    assert _check(prob, None) == B.QV_OK
    # within the 1e-5 tolerance of the total
    assert _check(prob, prob.b0.astype(np.float32) * np.float32(1 + 4e-6)) == B.QV_OK
    for name, b in _bad_beliefs(prob).items():
        assert _check(prob, b) == B.QV_ERR_BELIEF_INVALID, name


def test_model_check_rejects_bad_rewards_and_landmarks():
    _say("model check rewards/landmarks")
    prob = wl.make_rect(seed=3, side=20, n_landmarks=5, D=1, n=1)
    assert _check(prob, prob.b0) == B.QV_OK
    p2 = wl.make_rect(seed=3, side=20, n_landmarks=5, D=1, n=1)
    p2.R = p2.R.copy()
    p2.R[7, 2] = np.inf
    assert _check(p2, p2.b0) == B.QV_ERR_INVALID_ARG
    p3 = wl.make_rect(seed=3, side=20, n_landmarks=5, D=1, n=1)
    p3.lm_cell = p3.lm_cell.copy()
    p3.lm_cell[2] = int(np.flatnonzero(p3.occ == 1)[0])
    assert _check(p3, p3.b0) == B.QV_ERR_INVALID_ARG
    p4 = wl.make_rect(seed=3, side=20, n_landmarks=5, D=1, n=1)
    p4.lm_cell = p4.lm_cell.copy()
    p4.lm_cell[0] = p4.S + 3
    assert _check(p4, p4.b0) == B.QV_ERR_INVALID_ARG


def test_plan_check_flag():
    """With QV_PLAN_CHECK a bad start belief returns QV_ERR_BELIEF_INVALID and
    leaves the outputs untouched; a good one plans exactly as without it."""
    _say("plan with QV_PLAN_CHECK")
    from paper_1810_00204_amd.planner import Planner
    prob = wl.make_small(seed=4)
    Q = torch.as_tensor(np.zeros(prob.S * prob.A, np.float32)).cuda()
    ref = Planner(prob)
    ref.plan(Q)
    t_ref = ref.tree(beliefs=False)
    a_ref, q_ref = int(ref.action.item()), ref.rootQ.cpu().numpy().copy()
    pl = Planner(prob, flags=B.QV_PLAN_CHECK)
    pl.plan(Q)
    t = pl.tree(beliefs=False)
    assert int(pl.action.item()) == a_ref and np.array_equal(pl.rootQ.cpu().numpy(), q_ref)
    # records of absent slots are not written: compare the present ones
    ok = t_ref["valid"] == 1
    assert np.array_equal(t["valid"], t_ref["valid"])
    for k in ("z", "count", "value"):
        assert np.array_equal(t[k][ok], t_ref[k][ok]), k
    inner = ok.copy()
    inner[t_ref["level_first"][prob.D]:] = False
    qa, qb = t["qvalue"].reshape(-1, prob.A), t_ref["qvalue"].reshape(-1, prob.A)
    assert np.array_equal(qa[inner], qb[inner])
    for name, b in _bad_beliefs(prob).items():
        pl.action.fill_(-7)
        pl.rootQ.fill_(123.0)
        bt = torch.as_tensor(np.ascontiguousarray(b, np.float32)).cuda()
        st = B.qv_plan_step(pl.m, Q, bt, prob.D, prob.n, prob.seed, 0, B.QV_PLAN_CHECK,
                            pl.action, pl.rootQ, pl.ws)
        assert st == B.QV_ERR_BELIEF_INVALID, name
        torch.cuda.synchronize()
        assert int(pl.action.item()) == -7 and np.all(pl.rootQ.cpu().numpy() == 123.0), name
