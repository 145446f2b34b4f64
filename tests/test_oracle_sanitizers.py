"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

``qvo.c`` is built a second time with ``-fsanitize=address,undefined`` and
driven, in a child process that preloads gcc's sanitizer runtimes, through
every entry point the parity tests use: the model pieces, the plan with its
node expansion and leaf score, value iteration, the filter and its adjoint
(with an absorbing goal), the fast informed bound, the blind-policy bound,
best-first search and point-based value iteration.  Any out-of-bounds access,
use after free or undefined operation aborts the child with a report.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
import numpy as np
import oracle
from paper_1810_00204_amd import workloads as wl

prob = wl.make_small(seed=7, W=9, H=7, D=2, n=3)
Q, _, _ = oracle.value_iterate(prob, tol=1e-10)
res = oracle.plan(prob, Q.astype(np.float32), seed=11, qid=1)
e = oracle.expand_node(prob, prob.b0, 0, 0, beliefs=True)
v = oracle.leaf_score(prob, Q, prob.b0)
bp = oracle.predict(prob, prob.b0, 1)
lk = oracle.likelihood(prob, bp)
b1, pz, st = oracle.belief_update(prob, np.stack([prob.b0, prob.b0]), np.array([1, 2]),
                                  np.array([3, 0]))
draws = oracle.alg4_sample(prob, prob.b0, 0, 16, 5)

lm = wl.make_rect(seed=8, side=16, n_landmarks=6, D=2, n=2)
Ql, _, _ = oracle.value_iterate(lm, tol=1e-10)
oracle.plan(lm, Ql.astype(np.float32), seed=3, qid=0)

ts = wl.make_trajectories(seed=2, side=8, ntraj=2, T=5, n_landmarks=4, lm_p=0.8)
tp = ts.problem
free = np.flatnonzero(tp.occ == 0)
tp.goal = int(free[len(free) // 2])
nll, gt, gp = oracle.filter_nll_grad(tp, ts.theta, ts.phi, ts.acts, ts.obs)

U, _, _ = oracle.fib_iterate(prob, tol=1e-10)
oracle.fib_backup(prob, U, np.arange(prob.S))
L, _, _ = oracle.blind_iterate(prob, tol=1e-10)
t = oracle.search(prob, U.astype(np.float32), L.astype(np.float32), 12, seed=4, qid=0)
pb = oracle.pbvi(prob, L, 2, 2, seed=6, qid=0)
assert np.isfinite(res["rootQ"]).all() and np.isfinite(nll).all()
maps = open("/proc/self/maps").read()
assert "liboracle_san.so" in maps and "libasan" in maps and "libubsan" in maps
print("sanitized oracle ok")
"""


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.timeout(300)
def test_oracle_entry_points_under_sanitizers():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc's sanitizer runtimes are not installed")
    oracle.build(force=True, sanitize=True)
    env = dict(os.environ)
    env.update({
        "QVO_SANITIZED": "1",
        "LD_PRELOAD": f"{asan}:{ubsan}",
        # the interpreter's own allocations outlive it by design
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "PYTHONPATH": ROOT,
        "OMP_NUM_THREADS": "1",
    })
    r = subprocess.run([sys.executable, "-c", DRIVER], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=280)
    report = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "sanitized oracle ok" in r.stdout, report
    assert "AddressSanitizer" not in r.stderr, report
    assert "runtime error" not in r.stderr, report
