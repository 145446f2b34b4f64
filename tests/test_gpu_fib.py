"""GPU parity of the fast informed bound (Sec. IV-A, the FIB alpha-vector
equation) and of the one-launch sweep driver, through the C ABI.

* small grids: the GPU fixed point (FP32 sweeps, FP64 residual) against the
  oracle's FP64 fixed point, within the error bound of FP32 sweeps;
* any size: one FP64 backup of the GPU's own alpha vectors by the oracle at
  every (or sampled) cell must give back the vectors to within the last
  sweep's residual plus FP32 rounding (a fixed point of the equation);
* a perfect sensor makes FIB the Q-MDP fixed point; FIB lies below Q-MDP;
* the one-launch and per-sweep forms give bitwise equal results;
* the alpha vectors score the leaves of a plan as the Q table does, and the
  plan then matches the oracle's plan with the same table."""

import numpy as np
import pytest

import oracle
from paper_1810_00204_amd import binding as B
from paper_1810_00204_amd import workloads as wl
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _fib(prob, tol=1e-6, max_sweeps=20000):
    m = B.DeviceModel(prob)
    al = torch.empty(m.S * m.A, dtype=torch.float32, device="cuda")
    ws = torch.empty(B.qv_fib_workspace_bytes(m, max_sweeps), dtype=torch.uint8, device="cuda")
    st, res, sw = B.qv_fib_iterate(m, tol, max_sweeps, al, ws)
    B.check(st, "qv_fib_iterate")
    return al.cpu().numpy().reshape(m.S, m.A), res, sw


def _vi(prob, tol=1e-6, max_sweeps=20000):
    m = B.DeviceModel(prob)
    Q = torch.empty(m.S * m.A, dtype=torch.float32, device="cuda")
    ws = torch.empty(B.qv_vi_workspace_bytes(m, max_sweeps), dtype=torch.uint8, device="cuda")
    st, res, sw = B.qv_value_iterate(m, tol, max_sweeps, Q, ws)
    B.check(st, "qv_value_iterate")
    return Q.cpu().numpy().reshape(m.S, m.A), res, sw


def _blind(prob, tol=1e-6, max_sweeps=20000):
    m = B.DeviceModel(prob)
    al = torch.empty(m.S * m.A, dtype=torch.float32, device="cuda")
    ws = torch.empty(B.qv_blind_workspace_bytes(m, max_sweeps), dtype=torch.uint8, device="cuda")
    st, res, sw = B.qv_blind_iterate(m, tol, max_sweeps, al, ws)
    B.check(st, "qv_blind_iterate")
    return al.cpu().numpy().reshape(m.S, m.A), res, sw


def _problem(maker):
    return {"small": lambda: wl.make_small(seed=1),
            "rect32": lambda: wl.make_rect(seed=2, side=32, n_landmarks=8, D=2, n=2),
            "ragged": lambda: wl.make_small(seed=4, W=50, H=21),
            "nine": lambda: _nine_actions(wl.make_rect(seed=3, side=20, n_landmarks=5, D=1, n=1)),
            }[maker]()


def _nine_actions(prob):
    stay = np.zeros((1, 9), np.float32)
    stay[0, 4] = 1.0
    prob.slip = np.concatenate([prob.slip, stay])
    prob.R = wl.reward_step_goal(prob.occ, prob.W, prob.H, prob.slip, prob.goal)
    return prob


@pytest.mark.parametrize("maker", ["small", "rect32", "ragged", "nine"])
def test_fib_matches_fp64(maker):
    _say(f"FIB vs FP64 {maker}")
    prob = _problem(maker)
    al32, res, sw = _fib(prob)
    al64, res64, sw64 = oracle.fib_iterate(prob, tol=1e-12)
    err = np.abs(al32.astype(np.float64) - al64).max()
    amax = np.abs(al64).max()
    print(f"max |alpha32 - alpha64| = {err:.3g} (|alpha|max {amax:.3g}), sweeps {sw} "
          f"(fp64 {sw64}), residual {res:.3g}")
    # the FP32 fixed point: stopping error tol*|a|/(1-g) plus rounding of a
    # few ulp per sweep, damped by 1/(1-g)
    g = float(prob.gamma)
    assert err <= (1e-6 + 20 * U32) * max(1.0, amax) / (1 - g)
    assert np.all(al32[prob.occ == 1] == 0)
    assert sw < 20000


def test_fib_perfect_sensor_is_qmdp():
    """Every free cell a landmark that always reports: the observation names
    the successor, and FIB is the Q-MDP fixed point."""
    _say("FIB perfect sensor = Q-MDP")
    prob = wl.make_small(seed=5, W=9, H=8, frac=0.15)
    prob.lm_cell = np.flatnonzero(prob.occ == 0).astype(np.int32)
    prob.lm_p = 1.0
    al, _, _ = _fib(prob, tol=0.0, max_sweeps=600)
    Q, _, _ = _vi(prob, tol=0.0, max_sweeps=600)
    vmax = max(1.0, np.abs(Q).max())
    assert np.abs(al - Q).max() <= 40 * U32 * vmax / (1 - float(prob.gamma))


@pytest.mark.parametrize("maker", ["rect64", "large"])
def test_fib_is_a_fixed_point_at_full_size(maker):
    """One FP64 backup of the GPU's alpha vectors (every cell of 64 x 64, or
    2000 sampled cells of 512 x 512, near walls and landmarks included) gives
    the vectors back to within gamma times the last residual plus rounding;
    and FIB lies below the Q-MDP vectors."""
    _say(f"FIB fixed point {maker}")
    prob = wl.make_rect(seed=0) if maker == "rect64" else wl.make_large(seed=0)
    al, res, sw = _fib(prob)
    Q, _, _ = _vi(prob)
    free = np.flatnonzero(prob.occ == 0)
    if maker == "rect64":
        cells = np.arange(prob.S, dtype=np.int32)
    else:
        rng = np.random.default_rng(7)
        lm = np.asarray(prob.lm_cell, np.int64)
        near = np.unique(np.concatenate([lm + d for d in (-prob.W - 1, -1, 0, 1, prob.W + 1)]))
        near = near[(near >= 0) & (near < prob.S)]
        cells = np.unique(np.concatenate([rng.choice(free, 1500, replace=False),
                                          rng.choice(near, 500, replace=False),
                                          [prob.goal]])).astype(np.int32)
    h = oracle.fib_backup(prob, al.astype(np.float64), cells)
    amax = max(1.0, np.abs(al).max())
    dev = np.abs(h - al[cells]).max()
    print(f"{maker}: sweeps {sw}, residual {res:.3g}, max |H(alpha) - alpha| = {dev:.3g}")
    assert dev <= float(prob.gamma) * res + 64 * U32 * amax
    # Q-MDP bounds FIB from above (both FP32 fixed points)
    assert np.all(al[free] <= Q[free] + 40 * U32 * amax / (1 - float(prob.gamma)))


@pytest.mark.parametrize("solver", ["fib", "vi", "blind"])
def test_one_launch_equals_per_sweep_launches(solver, monkeypatch):
    """The cooperative one-launch driver and the per-sweep launches do the
    same arithmetic: bitwise equal results, same sweep count and residual."""
    _say(f"{solver}: one launch vs per-sweep launches")
    prob = wl.make_rect(seed=6, side=40, n_landmarks=6, D=1, n=1)
    run = {"fib": _fib, "vi": _vi, "blind": _blind}[solver]
    monkeypatch.setenv("QVTS_SWEEP_COOP", "1")
    a1, r1, s1 = run(prob)
    monkeypatch.setenv("QVTS_SWEEP_LAUNCHES", "1")
    a2, r2, s2 = run(prob)
    assert s1 == s2 and r1 == r2
    assert np.array_equal(a1, a2)
    # a capped run stops at the cap in both forms
    monkeypatch.delenv("QVTS_SWEEP_LAUNCHES")
    monkeypatch.setenv("QVTS_SWEEP_COOP", "1")
    a3, r3, s3 = run(prob, tol=0.0, max_sweeps=5)
    monkeypatch.setenv("QVTS_SWEEP_LAUNCHES", "1")
    a4, r4, s4 = run(prob, tol=0.0, max_sweeps=5)
    assert s3 == s4 == 5 and np.array_equal(a3, a4)


@pytest.mark.parametrize("maker", ["small", "rect24"])
def test_plan_with_fib_leaves_matches_oracle(maker):
    """Leaves scored with the FIB vectors (U_V = V_FIB of Alg. 5): the GPU plan
    with the FIB table equals the oracle's plan with the same table."""
    _say(f"plan with FIB leaves {maker}")
    from paper_1810_00204_amd.planner import Planner
    prob = (wl.make_small(seed=11) if maker == "small"
            else wl.make_rect(seed=12, side=24, n_landmarks=6, D=2, n=3))
    pl = Planner(prob)
    al, _, _ = pl.fib_iterate(tol=1e-6)
    act, rq = pl.plan(al)
    torch.cuda.synchronize()
    al32 = al.cpu().numpy().reshape(prob.S, prob.A)
    g = pl.tree(beliefs=True)
    ref = oracle.plan(prob, al32, dump_beliefs=True)
    rep = parity.compare_tree(prob, g, ref["dump"])
    assert rep.nodes > 1
    assert parity.root_action_ok(int(act.item()), ref["rootQ"], ref["action"])
    # FIB leaves are never above the Q-MDP leaves of the same tree draws
    Q, _, _ = pl.value_iterate(tol=1e-6)
    pl.plan(Q)
    gq = pl.tree(beliefs=False)
    lf = g["level_first"]
    leaf = slice(lf[prob.D], lf[prob.D + 1])
    ok = g["valid"][leaf] == 1
    assert np.array_equal(gq["valid"][leaf], g["valid"][leaf])
    vq, vf = gq["value"][leaf][ok], g["value"][leaf][ok]
    assert np.all(vf <= vq + 1e-5 * np.maximum(1.0, np.abs(vq)))


def test_fib_rejects_bad_arguments():
    _say("FIB argument checks")
    prob = wl.make_small(seed=2)
    m = B.DeviceModel(prob)
    al = torch.empty(m.S * m.A, dtype=torch.float32, device="cuda")
    ws = torch.empty(B.qv_fib_workspace_bytes(m, 10), dtype=torch.uint8, device="cuda")
    assert B.qv_fib_iterate(m, 1e-6, 0, al, ws)[0] == B.QV_ERR_INVALID_ARG
    assert B.qv_fib_iterate(m, -1.0, 10, al, ws)[0] == B.QV_ERR_INVALID_ARG
    assert B.qv_fib_iterate(m, 1e-6, 100, al, ws)[0] == B.QV_ERR_WORKSPACE
    assert B.qv_fib_workspace_bytes(m, 0) == 0
