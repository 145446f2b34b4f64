"""The allocation-free belief update (qv_belief_update_noalloc) against the
workspace form (qv_belief_update), through the C ABI: two calls in a row on
the library's own scratch region, the second with a smaller input, each
bitwise equal to the workspace form on the same inputs (the same kernels
run on either scratch space); and sizes over the stated limit are refused
before anything is enqueued."""
import numpy as np
import pytest

from paper_1810_00204_amd import binding as B
from paper_1810_00204_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _inputs(prob, batch, seed):
    rng = np.random.default_rng(seed)
    free = np.flatnonzero(prob.occ == 0)
    b = np.zeros((batch, prob.S), np.float32)
    for i in range(batch):
        cells = rng.choice(free, size=min(40, free.size), replace=False)
        w = rng.random(cells.size)
        b[i, cells] = w / w.sum()
    a = rng.integers(0, prob.A, size=batch).astype(np.int32)
    # observations drawn from the cell each belief is most sure of, so that
    # P(z|b,a) > 0 (wall reading of that cell, no landmark)
    z = rng.integers(0, 16, size=batch).astype(np.int32)
    return b, a, z


def _workspace_form(m, batch, bt, at, zt):
    bo = torch.zeros_like(bt)
    po = torch.zeros(batch, dtype=torch.float32, device="cuda")
    ws = torch.empty(max(B.qv_belief_update_workspace_bytes(m, batch), 1), dtype=torch.uint8,
                     device="cuda")
    st = B.qv_belief_update(m, batch, bt, at, zt, bo, po, 1, ws)
    return st, bo, po


def _noalloc_form(m, batch, bt, at, zt):
    bo = torch.zeros_like(bt)
    po = torch.zeros(batch, dtype=torch.float32, device="cuda")
    st = B.qv_belief_update_noalloc(m, batch, bt, at, zt, bo, po, 1)
    return st, bo, po


def test_noalloc_belief_update_matches_workspace_form():
    cases = [(wl.make_large(seed=2), 6, 1), (wl.make_rect(seed=3, side=40, n_landmarks=8), 3, 2)]
    for prob, batch, seed in cases:
        _say(f"noalloc belief update {prob.W}x{prob.H} batch {batch}")
        m = B.DeviceModel(prob)
        b, a, z = _inputs(prob, batch, seed)
        bt = torch.as_tensor(b).cuda()
        at = torch.as_tensor(a).cuda()
        zt = torch.as_tensor(z).cuda()
        st1, bo1, po1 = _workspace_form(m, batch, bt, at, zt)
        st2, bo2, po2 = _noalloc_form(m, batch, bt, at, zt)
        torch.cuda.synchronize()
        assert st1 == st2 == B.QV_OK, (st1, st2)
        assert np.array_equal(po1.cpu().numpy(), po2.cpu().numpy())
        assert np.array_equal(bo1.cpu().numpy(), bo2.cpu().numpy())
        assert np.all(po2.cpu().numpy() > 0)


def test_noalloc_belief_update_reports_like_workspace_form():
    _say("noalloc belief update statuses")
    prob = wl.make_small(seed=4)
    m = B.DeviceModel(prob)
    b, a, z = _inputs(prob, 2, 3)
    a[1] = 99   # out of range
    bt, at, zt = (torch.as_tensor(x).cuda() for x in (b, a, z))
    st1, bo1, po1 = _workspace_form(m, 2, bt, at, zt)
    st2, bo2, po2 = _noalloc_form(m, 2, bt, at, zt)
    assert st1 == st2 != B.QV_OK
    assert np.array_equal(bo1[0].cpu().numpy(), bo2[0].cpu().numpy())


def test_noalloc_belief_update_refuses_sizes_over_the_limit():
    _say("noalloc belief update limits")
    prob = wl.make_small(seed=5, W=1100, H=1000, frac=0.1)   # 1.1 M cells
    m = B.DeviceModel(prob)
    bt = torch.zeros(prob.S, dtype=torch.float32, device="cuda")
    at = torch.zeros(1, dtype=torch.int32, device="cuda")
    zt = torch.zeros(1, dtype=torch.int32, device="cuda")
    bo = torch.zeros_like(bt)
    po = torch.full((1,), -3.0, dtype=torch.float32, device="cuda")
    assert B.qv_belief_update_noalloc(m, 1, bt, at, zt, bo, po, 0) == B.QV_ERR_UNSUPPORTED
    assert po.item() == -3.0
    prob2 = wl.make_small(seed=6, W=512, H=512, frac=0.1)   # 256 bands per belief
    m2 = B.DeviceModel(prob2)
    n = 65   # 65 * 256 bands > 16384
    bt2 = torch.zeros(n * prob2.S, dtype=torch.float32, device="cuda")
    at2 = torch.zeros(n, dtype=torch.int32, device="cuda")
    bo2 = torch.zeros_like(bt2)
    po2 = torch.zeros(n, dtype=torch.float32, device="cuda")
    assert B.qv_belief_update_noalloc(m2, n, bt2, at2, at2, bo2, po2, 0) == B.QV_ERR_UNSUPPORTED
