"""GPU parity of the differentiable filter (NLL and hand adjoint) against the
FP64 oracle, through the C ABI, plus properties that hold at any size."""
import numpy as np
import pytest

import oracle
from paper_1810_00204_amd import binding as B
from paper_1810_00204_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _problem(ts, sub=None, ckpt=10):
    from paper_1810_00204_amd.filter import FilterProblem
    acts, obs = ts.acts, ts.obs
    if sub is not None:
        acts, obs = acts[sub], obs[sub]
    return FilterProblem(ts.problem, acts, obs, ckpt_every=ckpt)


def _grad_close(g32, g64, rel=1e-4, entry=1e-4):
    """The slip-logit part (the first A*9 entries) and the flip-logit part
    (the last 4) are compared separately, each by its relative L2 error, so
    the small flip part cannot hide behind the slip part; then every entry
    against the largest magnitude of its own part: |g32 - g64| <=
    entry * max|g64 part| + 1e-7 (a sign or scale error in a single entry
    fails this)."""
    g32 = np.asarray(g32, np.float64).reshape(-1)
    g64 = np.asarray(g64, np.float64).reshape(-1)
    errs = []
    for part in (slice(0, g64.size - 4), slice(g64.size - 4, g64.size)):
        a, b = g32[part], g64[part]
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert err <= rel, (part, err)
        bound = entry * np.abs(b).max() + 1e-7
        bad = np.abs(a - b) > bound
        assert not bad.any(), (part, np.flatnonzero(bad), a[bad], b[bad], bound)
        errs.append(err)
    return max(errs)


@pytest.mark.parametrize("case", ["small", "landmarks", "goal", "ragged_segments"])
def test_filter_matches_oracle(case):
    _say(f"filter {case}")
    if case == "small":
        ts = wl.make_trajectories(seed=1, side=16, ntraj=6, T=12)
        ckpt = 5
    elif case == "landmarks":
        ts = wl.make_trajectories(seed=2, side=12, ntraj=6, T=9, n_landmarks=30, lm_p=0.8)
        assert (ts.obs >= 16).any()
        ckpt = 4
    elif case == "goal":
        ts = wl.make_trajectories(seed=3, side=10, ntraj=3, T=8)
        ts.problem.goal = int(np.flatnonzero(ts.problem.occ == 0)[7])
        ckpt = 3
    else:
        ts = wl.make_trajectories(seed=4, side=20, ntraj=5, T=13)
        ckpt = 13
    fp = _problem(ts, ckpt=ckpt)
    th = torch.as_tensor(ts.theta)
    ph = torch.as_tensor(ts.phi)
    nll, gs, gf = fp.run(th, ph)
    torch.cuda.synchronize()
    onll, ogt, ogp = oracle.filter_nll_grad(ts.problem, ts.theta, ts.phi, ts.acts, ts.obs)
    np.testing.assert_allclose(nll.cpu().numpy(), onll, rtol=2e-5)
    err = _grad_close(np.concatenate([gs.cpu().numpy().ravel(), gf.cpu().numpy()]),
                      np.concatenate([ogt.ravel(), ogp]))
    print(f"relative gradient error {err:.2e}")


def test_filter_checkpoint_interval_does_not_change_results():
    _say("filter checkpoint k=1 vs k=10")
    ts = wl.make_trajectories(seed=5, side=24, ntraj=8, T=20)
    th, ph = torch.as_tensor(ts.theta), torch.as_tensor(ts.phi)
    outs = []
    for k in (1, 10, 20):
        nll, gs, gf = _problem(ts, ckpt=k).run(th, ph)
        torch.cuda.synchronize()
        outs.append((nll.cpu().numpy(), gs.cpu().numpy(), gf.cpu().numpy()))
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert np.array_equal(x, y)


def test_filter_full_size_sampled_runs():
    """1024 runs of 50 steps on 128 x 128: sampled runs against the oracle,
    and the gradient of the whole set equals the sum over two halves."""
    _say("filter 128x128 1024x50")
    ts = wl.make_trajectories(seed=0)
    th, ph = torch.as_tensor(ts.theta), torch.as_tensor(ts.phi)
    fp = _problem(ts)
    nll, gs, gf = fp.run(th, ph)
    torch.cuda.synchronize()
    nll = nll.cpu().numpy()
    assert np.all(np.isfinite(nll))
    pick = [0, 511, 1023]
    onll, ogt, ogp = oracle.filter_nll_grad(ts.problem, ts.theta, ts.phi, ts.acts[pick], ts.obs[pick])
    np.testing.assert_allclose(nll[pick], onll, rtol=2e-5)
    n1, g1s, g1f = _problem(ts, sub=slice(0, 512)).run(th, ph)
    n2, g2s, g2f = _problem(ts, sub=slice(512, 1024)).run(th, ph)
    s3, g3s, g3f = _problem(ts, sub=pick).run(th, ph)
    torch.cuda.synchronize()
    _grad_close(np.concatenate([g3s.cpu().numpy().ravel(), g3f.cpu().numpy()]),
                np.concatenate([ogt.ravel(), ogp]))
    whole = np.concatenate([gs.cpu().numpy().ravel(), gf.cpu().numpy()]).astype(np.float64)
    halves = (np.concatenate([g1s.cpu().numpy().ravel(), g1f.cpu().numpy()]).astype(np.float64)
              + np.concatenate([g2s.cpu().numpy().ravel(), g2f.cpu().numpy()]))
    assert np.linalg.norm(whole - halves) <= 1e-5 * np.linalg.norm(whole)
    np.testing.assert_array_equal(np.concatenate([n1.cpu().numpy(), n2.cpu().numpy()]), nll)


def test_filter_autograd_function():
    _say("filter autograd")
    from paper_1810_00204_amd.filter import FilterNLL
    ts = wl.make_trajectories(seed=6, side=12, ntraj=4, T=10)
    fp = _problem(ts, ckpt=3)
    onll, ogt, ogp = oracle.filter_nll_grad(ts.problem, ts.theta, ts.phi, ts.acts, ts.obs)
    # leaf tensors on the GPU, and on the host (the gradients come back on
    # the device and dtype of the parameters)
    for dev, dt in (("cuda", torch.float32), ("cpu", torch.float32), ("cpu", torch.float64)):
        th = torch.tensor(ts.theta, device=dev, dtype=dt, requires_grad=True)
        ph = torch.tensor(ts.phi, device=dev, dtype=dt, requires_grad=True)
        loss = 2.0 * FilterNLL.apply(th, ph, fp)
        loss.backward()
        assert th.grad.device == th.device and th.grad.dtype == dt
        assert ph.grad.device == ph.device and ph.grad.dtype == dt
        assert abs(loss.item() - 2 * onll.sum()) <= 2e-5 * abs(2 * onll.sum())
        _grad_close(np.concatenate([th.grad.cpu().numpy().ravel(), ph.grad.cpu().numpy()]),
                    2 * np.concatenate([ogt.ravel(), ogp]))


def test_filter_reports_bad_inputs():
    _say("filter bad inputs")
    ts = wl.make_trajectories(seed=7, side=10, ntraj=3, T=5)
    acts = ts.acts.copy()
    acts[1, 2] = 99
    from paper_1810_00204_amd.filter import FilterProblem
    fp = FilterProblem(ts.problem, acts, ts.obs, ckpt_every=2)
    th, ph = torch.as_tensor(ts.theta), torch.as_tensor(ts.phi)
    with pytest.raises(B.QvError) as ei:
        fp.run(th, ph)
    assert ei.value.status == B.QV_ERR_INVALID_ARG


def test_filter_no_runs_gives_zero_gradient():
    _say("filter zero runs")
    ts = wl.make_trajectories(seed=8, side=10, ntraj=2, T=4)
    from paper_1810_00204_amd.filter import FilterProblem
    fp = FilterProblem(ts.problem, ts.acts[:0], ts.obs[:0], ckpt_every=2)
    th, ph = torch.as_tensor(ts.theta), torch.as_tensor(ts.phi)
    nll, gs, gf = fp.run(th, ph)
    torch.cuda.synchronize()
    assert nll.numel() == 0
    assert not gs.abs().sum().item() and not gf.abs().sum().item()


def test_filter_long_runs_stay_finite():
    """200 steps on a map with many blocked cells: every output is finite
    and the adjoint still matches the oracle."""
    _say("filter long runs")
    ts = wl.make_trajectories(seed=9, side=16, frac=0.3, ntraj=3, T=200)
    fp = _problem(ts, ckpt=16)
    th, ph = torch.as_tensor(ts.theta), torch.as_tensor(ts.phi)
    nll, gs, gf = fp.run(th, ph)
    torch.cuda.synchronize()
    g = np.concatenate([gs.cpu().numpy().ravel(), gf.cpu().numpy()])
    assert np.all(np.isfinite(nll.cpu().numpy())) and np.all(np.isfinite(g))
    onll, ogt, ogp = oracle.filter_nll_grad(ts.problem, ts.theta, ts.phi, ts.acts, ts.obs)
    np.testing.assert_allclose(nll.cpu().numpy(), onll, rtol=1e-4)
    _grad_close(g, np.concatenate([ogt.ravel(), ogp]), rel=5e-4, entry=5e-4)
