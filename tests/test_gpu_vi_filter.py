"""GPU parity of value iteration and of the batched Bayes filter step against
the FP64 oracle (MI355X, through the C ABI)."""
import numpy as np
import pytest

import oracle
from paper_1810_00204_amd import binding as B
from paper_1810_00204_amd import workloads as wl
from tests.test_oracle_pins import corridor

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _vi(prob, tol, max_sweeps=20000):
    m = B.DeviceModel(prob)
    Q = torch.empty(m.S * m.A, dtype=torch.float32, device="cuda")
    ws = torch.empty(B.qv_vi_workspace_bytes(m, max_sweeps), dtype=torch.uint8, device="cuda")
    st, res, sw = B.qv_value_iterate(m, tol, max_sweeps, Q, ws)
    B.check(st, "qv_value_iterate")
    return Q.cpu().numpy().reshape(m.S, m.A).astype(np.float64), res, sw


def test_value_iteration_corridor_closed_form():
    _say("VI corridor 1x40")
    L = 40
    prob = corridor(L)
    Q, res, sw = _vi(prob, 1e-7)
    g = float(np.float32(0.95))
    p = float(prob.slip[3, 3])
    s_ = float(prob.slip[3, 1]) + float(prob.slip[3, 7])
    R1 = float(prob.R[1, 3])
    V1 = R1 / (1 - g * s_)
    c = -1.0 / (1 - g * s_ - g * p)
    rho = g * p / (1 - g * s_)
    V = Q.max(axis=1)
    want = c + (V1 - c) * rho ** (np.arange(1, L) - 1)
    # FP32 fixed point: a few ULPs of |V| <= 100 per sweep, damped by 1/(1-g)
    assert np.abs(V[1:] - want).max() <= 2e-4, np.abs(V[1:] - want).max()
    assert np.all(Q[1:].argmax(axis=1) == 3)
    assert res <= 1e-7 * max(1.0, np.abs(V).max()) or res == 0.0


@pytest.mark.parametrize("maker", ["small", "rect", "ragged", "large"])
def test_value_iteration_matches_fp64(maker):
    _say(f"VI vs FP64 {maker}")
    prob = {"small": lambda: wl.make_small(seed=1),
            "rect": lambda: wl.make_rect(seed=0),
            "ragged": lambda: wl.make_small(seed=2, W=50, H=100),
            "large": lambda: wl.make_large(seed=0)}[maker]()
    Q32, res, sw = _vi(prob, 1e-6)
    Q64, res64, sw64 = oracle.value_iterate(prob, tol=1e-12)
    err = np.abs(Q32 - Q64).max()
    vmax = np.abs(Q64).max()
    print(f"max |Q32 - Q64| = {err:.3g} (|V|max {vmax:.3g}), sweeps {sw} (fp64 {sw64})")
    # the stopping rule leaves |V_k - V*| <= r_k gamma / (1 - gamma) with
    # r_k <= tol * |V|, plus FP32 rounding of a few ulp per sweep, damped by
    # 1 / (1 - gamma): (tol + 8u) |V| / (1 - gamma), about 1.6 times the
    # largest error measured on these maps (1.8e-3 on the 50 x 100 one)
    assert err <= (1e-6 + 8 * 2 ** -24) * max(1.0, vmax) / (1 - 0.95)
    assert np.all(Q32[prob.occ == 1] == 0)
    # the FP32 run stopped by its own rule
    assert sw < 20000
    # greedy actions agree wherever the FP64 gap is clear
    gap = np.sort(Q64, axis=1)[:, -1] - np.sort(Q64, axis=1)[:, -2]
    clear = (prob.occ == 0) & (gap > 1e-3)
    assert np.array_equal(Q32[clear].argmax(1), Q64[clear].argmax(1))


def test_value_iteration_tolerance_and_cap():
    _say("VI cap")
    prob = wl.make_small(seed=3)
    Q, res, sw = _vi(prob, 0.0, max_sweeps=7)
    assert sw == 7
    Q64, _, sw64 = oracle.value_iterate(prob, tol=0.0, max_sweeps=7)
    assert sw64 == 7
    np.testing.assert_allclose(Q, Q64, rtol=1e-5, atol=1e-4)


def _bu(prob, b, a, z, check=True):
    from paper_1810_00204_amd.planner import belief_update
    m = B.DeviceModel(prob)
    bt = torch.as_tensor(np.ascontiguousarray(b, np.float32)).cuda()
    at = torch.as_tensor(np.asarray(a, np.int32)).cuda()
    zt = torch.as_tensor(np.asarray(z, np.int32)).cuda()
    bo, po, st = belief_update(m, bt, at, zt, check=check)
    torch.cuda.synchronize()
    return bo.cpu().numpy().astype(np.float64), po.cpu().numpy().astype(np.float64), st


@pytest.mark.parametrize("maker", ["small", "rect", "ragged", "large"])
def test_belief_update_matches_oracle(maker):
    _say(f"belief update {maker}")
    prob = {"small": lambda: wl.make_small(seed=4),
            "rect": lambda: wl.make_rect(seed=1),
            "ragged": lambda: wl.make_small(seed=5, W=50, H=100),
            "large": lambda: wl.make_large(seed=1)}[maker]()
    rng = np.random.default_rng(0)
    free = np.flatnonzero(prob.occ == 0)
    nb = 3 if maker == "large" else 12
    bs, acts, zs = [], [], []
    for i in range(nb):
        if i == 0:
            b = prob.b0.astype(np.float64)
        else:
            b = np.zeros(prob.S)
            cells = rng.choice(free, size=min(free.size, 1 + rng.integers(1, 200)), replace=False)
            b[cells] = rng.random(cells.size)
            b /= b.sum()
        b = b.astype(np.float32)
        a = int(rng.integers(0, prob.A))
        p = oracle.likelihood(prob, oracle.predict(prob, b.astype(np.float64), a))
        cand = np.flatnonzero(p > 0)
        z = int(rng.choice(cand))
        bs.append(b)
        acts.append(a)
        zs.append(z)
    b = np.stack(bs)
    out, p, st = _bu(prob, b, acts, zs)
    assert st == B.QV_OK
    ref, pref, st2 = oracle.belief_update(prob, b, np.array(acts), np.array(zs))
    assert st2 == 0
    np.testing.assert_allclose(p, pref, rtol=1e-5)
    tol = 1e-5 * np.abs(ref) + 1e-12 * ref.max(axis=1, keepdims=True)
    assert np.all(np.abs(out - ref) <= tol)


def test_belief_update_zero_likelihood_and_bad_index():
    _say("belief update zero likelihood")
    prob = wl.make_small(seed=6)
    prob.flip = np.zeros(4, np.float32)
    b = prob.b0.astype(np.float64)
    from tests.dense_model import wall_pattern
    bp = oracle.predict(prob, b, 0)
    w = wall_pattern(prob)
    bad = [z for z in range(16) if bp[w == z].sum() == 0][0]
    good = [z for z in range(16) if bp[w == z].sum() > 0][0]
    bb = np.stack([b, b]).astype(np.float32)
    out, p, st = _bu(prob, bb, [0, 0], [good, bad])
    assert st == B.QV_ERR_ZERO_LIKELIHOOD
    assert p[1] == 0.0 and p[0] > 0
    assert np.all(out[1] == 0.0)          # untouched (zero-initialised) row
    out, p, st = _bu(prob, bb, [0, 9], [good, good])   # action out of range
    assert st == B.QV_ERR_ZERO_LIKELIHOOD and p[1] == 0.0
    out, p, st = _bu(prob, bb, [0, 0], [good, 16])     # z out of range (|Z| = 16)
    assert st == B.QV_ERR_ZERO_LIKELIHOOD and p[1] == 0.0
