"""Host-side checks of libqvts.so that need no GPU: the library loads, it
exports every function include/qvts.h declares, and the host logic
(status strings, workspace layouts, argument validation) behaves as the
header documents.  No call here reaches a kernel."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1810_00204_amd import binding as B
from paper_1810_00204_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "qvts.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qv_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = header_functions()
    assert len(names) >= 9
    lib = C.CDLL(B.LIB_PATH)
    for nm in names:
        assert hasattr(lib, nm), nm
    assert sorted(B.EXPORTS) == names


def test_status_strings():
    for s in range(8):
        assert B.qv_status_string(s) != "unknown status"
    assert B.qv_status_string(99) == "unknown status"


class FakeModel:
    """qv_model whose device pointers are dummies: only host logic may run."""

    def __init__(self, prob, **kw):
        sl = np.zeros(81, np.float32)
        src = np.asarray(kw.get("slip", prob.slip), np.float32).reshape(-1)
        sl[:src.size] = src
        fl = np.asarray(kw.get("flip", prob.flip), np.float32)
        self.c = B.qv_model(kw.get("W", prob.W), kw.get("H", prob.H), 0x1000, src.size // 9,
                            (C.c_float * 81)(*sl.tolist()), (C.c_float * 4)(*fl.tolist()),
                            kw.get("L", len(prob.lm_cell)), 0x2000 if kw.get("L", len(prob.lm_cell)) else 0,
                            kw.get("lm_p", prob.lm_p), 0x3000, kw.get("goal", prob.goal),
                            kw.get("gamma", prob.gamma))


@pytest.mark.parametrize("D,n", [(0, 1), (1, 2), (2, 2), (3, 4)])
def test_plan_layout_is_consistent(D, n):
    prob = wl.make_rect(seed=0, side=64, n_landmarks=32, D=D, n=n)
    m = FakeModel(prob)
    nb = B.qv_plan_workspace_bytes(m, D, n, 0)
    st, L = B.qv_plan_layout(m, D, n, 0)
    assert st == 0 and nb == L.total_bytes > 0
    K = prob.A * n
    assert [L.level_slots[d] for d in range(D + 1)] == [K ** d for d in range(D + 1)]
    assert L.level_first[D + 1] == sum(K ** d for d in range(D + 1))
    assert L.tile_rows * L.tiles >= prob.H > (L.tiles - 1) * L.tile_rows
    for off in (L.valid, L.z, L.count, L.pz, L.value, L.qvalue, L.reward):
        assert off % 256 == 0 and off < L.total_bytes
    # beliefs are stored for levels 1..D-1 only (leaves are scored on the fly)
    for d in range(1, D + 1):
        assert (L.belief_offset[d] != 0) == (d < D)
    st2, L2 = B.qv_plan_layout(m, D, n, B.QV_PLAN_STORE_LEAVES)
    if D >= 1:
        assert L2.belief_offset[D] != 0 and L2.total_bytes > L.total_bytes


def test_validation_errors_return_before_any_launch():
    prob = wl.make_small(seed=0)
    bad_slip = prob.slip.copy()
    bad_slip[0, 4] += 0.5
    cases = [
        (FakeModel(prob, slip=bad_slip), B.QV_ERR_NOT_STOCHASTIC),
        (FakeModel(prob, gamma=1.0), B.QV_ERR_INVALID_ARG),
        (FakeModel(prob, goal=prob.S), B.QV_ERR_INVALID_ARG),
        (FakeModel(prob, W=0), B.QV_ERR_INVALID_ARG),
        (FakeModel(prob, W=4096), B.QV_ERR_INVALID_ARG),
        (FakeModel(prob, lm_p=1.5), B.QV_ERR_INVALID_ARG),
        (FakeModel(prob, flip=[0.1, 0.1, -0.1, 0.1]), B.QV_ERR_INVALID_ARG),
        (FakeModel(prob, L=600), B.QV_ERR_INVALID_ARG),
    ]
    for m, want in cases:
        st = B.lib().qv_plan_step(C.byref(m.c), 0x10, 0x20, 2, 2, 1, 0, 0, 0x30, 0x40, 0x100,
                                  1 << 20, None)
        assert st == want
        assert B.qv_plan_workspace_bytes(m, 2, 2, 0) == 0
    m = FakeModel(prob)
    # bad depth / samples / flags / null outputs / workspace
    assert B.lib().qv_plan_step(C.byref(m.c), 0x10, 0x20, 7, 2, 1, 0, 0, 0x30, 0x40, 0x100, 1 << 20, None) == B.QV_ERR_INVALID_ARG
    assert B.lib().qv_plan_step(C.byref(m.c), 0x10, 0x20, 2, 17, 1, 0, 0, 0x30, 0x40, 0x100, 1 << 20, None) == B.QV_ERR_INVALID_ARG
    assert B.lib().qv_plan_step(C.byref(m.c), 0x10, 0x20, 2, 2, 1, 0, 8, 0x30, 0x40, 0x100, 1 << 20, None) == B.QV_ERR_INVALID_ARG
    assert B.lib().qv_plan_step(C.byref(m.c), 0x10, 0x20, 2, 2, 1, 0, 0, None, 0x40, 0x100, 1 << 20, None) == B.QV_ERR_INVALID_ARG
    need = B.qv_plan_workspace_bytes(m, 2, 2, 0)
    assert B.lib().qv_plan_step(C.byref(m.c), 0x10, 0x20, 2, 2, 1, 0, 0, 0x30, 0x40, 0x100, need - 1, None) == B.QV_ERR_WORKSPACE
    assert B.lib().qv_plan_step(C.byref(m.c), 0x10, 0x20, 2, 2, 1, 0, 0, 0x30, 0x40, 0x104, need, None) == B.QV_ERR_WORKSPACE
    assert B.lib().qv_plan_step(C.byref(m.c), 0x10, 0x20, 2, 2, 1, 0, 0, 0x30, 0x40, None, need, None) == B.QV_ERR_WORKSPACE
    # value iteration and the filter step check their arguments the same way
    vneed = B.qv_vi_workspace_bytes(m, 100)
    assert vneed > 0
    r, k = C.c_double(), C.c_int32()
    assert B.lib().qv_value_iterate(C.byref(m.c), 1e-6, 0, 0x10, C.byref(r), C.byref(k), 0x100, vneed, None) == B.QV_ERR_INVALID_ARG
    assert B.lib().qv_value_iterate(C.byref(m.c), 1e-6, 100, 0x10, C.byref(r), C.byref(k), 0x100, vneed - 1, None) == B.QV_ERR_WORKSPACE
    bneed = B.qv_belief_update_workspace_bytes(m, 4)
    assert bneed > 0
    assert B.lib().qv_belief_update(C.byref(m.c), -1, 0x10, 0x20, 0x30, 0x40, 0x50, 0, 0x100, bneed, None) == B.QV_ERR_INVALID_ARG
    assert B.lib().qv_belief_update(C.byref(m.c), 4, 0x1000, 0x20, 0x30, 0x1100, 0x50, 0, 0x100, bneed, None) == B.QV_ERR_INVALID_ARG   # b and b_out overlap
    assert B.lib().qv_belief_update(C.byref(m.c), 4, 0x10, 0x20, 0x30, 0x100000, 0x50, 0, 0x100, bneed - 1, None) == B.QV_ERR_WORKSPACE


def test_tree_capacity_limit_is_reported():
    prob = wl.make_rect(seed=0, side=64, n_landmarks=32, D=6, n=16)
    m = FakeModel(prob)
    assert B.qv_plan_workspace_bytes(m, 6, 16, 0) == 0
    st, _ = B.qv_plan_layout(m, 6, 16, 0)
    assert st == B.QV_ERR_UNSUPPORTED


def test_fib_and_check_arguments_are_checked_on_the_host():
    prob = wl.make_small(seed=1)
    m = FakeModel(prob)
    r, k = C.c_double(), C.c_int32()
    fneed = B.qv_fib_workspace_bytes(m, 50)
    assert fneed > B.qv_vi_workspace_bytes(m, 50) > 0   # A values per cell, not one
    lib = B.lib()
    assert lib.qv_fib_iterate(C.byref(m.c), 1e-6, 0, 0x10, C.byref(r), C.byref(k), 0x100, fneed, None) == B.QV_ERR_INVALID_ARG
    assert lib.qv_fib_iterate(C.byref(m.c), 1e-6, 50, None, C.byref(r), C.byref(k), 0x100, fneed, None) == B.QV_ERR_INVALID_ARG
    assert lib.qv_fib_iterate(C.byref(m.c), 1e-6, 50, 0x10, C.byref(r), C.byref(k), 0x100, fneed - 1, None) == B.QV_ERR_WORKSPACE
    bad = FakeModel(prob, gamma=0.0)
    assert lib.qv_fib_iterate(C.byref(bad.c), 1e-6, 50, 0x10, C.byref(r), C.byref(k), 0x100, fneed, None) == B.QV_ERR_INVALID_ARG
    assert B.qv_check_workspace_bytes() == 256
    assert lib.qv_model_check(C.byref(bad.c), 0x10, 0x100, 256, None) == B.QV_ERR_INVALID_ARG
    assert lib.qv_model_check(C.byref(m.c), 0x10, 0x100, 255, None) == B.QV_ERR_WORKSPACE
    assert lib.qv_model_check(C.byref(m.c), 0x10, 0x104, 256, None) == B.QV_ERR_WORKSPACE
    # the check flag is accepted by the plan call's flag test (bad depth still wins)
    assert lib.qv_plan_step(C.byref(m.c), 0x10, 0x20, 7, 2, 1, 0, B.QV_PLAN_CHECK, 0x30, 0x40, 0x100, 1 << 20, None) == B.QV_ERR_INVALID_ARG
    assert lib.qv_plan_step(C.byref(m.c), 0x10, 0x20, 2, 2, 1, 0, 16, 0x30, 0x40, 0x100, 1 << 20, None) == B.QV_ERR_INVALID_ARG


def test_pbvi_layout_and_arguments_are_checked_on_the_host():
    prob = wl.make_small(seed=1)
    m = FakeModel(prob)
    P, k = 16, prob.A
    need = B.qv_pbvi_workspace_bytes(m, P, k)
    st, L = B.qv_pbvi_layout_of(m, P, k)
    assert st == 0 and need == L.total_bytes > 0
    assert L.ZC == 16 * (len(prob.lm_cell) + 1) and L.ld == max(P, k) and L.max_points == P
    # regions in order, 256-byte aligned, inside the workspace
    offs = [getattr(L, f) for f, _ in B.qv_pbvi_layout._fields_[5:-1]]
    assert offs == sorted(offs) and all(o % 256 == 0 for o in offs) and offs[-1] < need
    assert L.gamma1 - L.gamma0 >= prob.S * L.ld * 4
    assert L.pred - L.points >= P * prob.S * 4
    # capacity and column limits
    assert B.qv_pbvi_workspace_bytes(m, 0, k) == 0
    assert B.qv_pbvi_workspace_bytes(m, B.QV_PBVI_MAX_POINTS + 1, k) == 0
    assert B.qv_pbvi_workspace_bytes(m, P, 0) == 0
    assert B.qv_pbvi_workspace_bytes(FakeModel(prob, W=400, H=400), P, k) == 0
    lib = B.lib()
    assert lib.qv_pbvi_init(C.byref(m.c), None, 0x10, k, P, 0x100, need, None) == B.QV_ERR_INVALID_ARG
    assert lib.qv_pbvi_init(C.byref(m.c), 0x10, 0x20, k, P, 0x100, need - 1, None) == B.QV_ERR_WORKSPACE
    assert lib.qv_pbvi_init(C.byref(m.c), 0x10, 0x20, k, 0, 0x100, need, None) == B.QV_ERR_INVALID_ARG
    added = C.c_int32()
    assert lib.qv_pbvi_expand(C.byref(m.c), k, P, 1, 0, None, 0x100, need, None) == B.QV_ERR_INVALID_ARG
    assert lib.qv_pbvi_backup(C.byref(m.c), k, P, -1, 0x100, need, None) == B.QV_ERR_INVALID_ARG
    assert lib.qv_pbvi_backup(C.byref(m.c), k, P, 0, 0x100, need, None) == 0   # nothing to do
    assert lib.qv_pbvi_result(C.byref(m.c), k, P, 0x10, 0, C.byref(added), 0x100, need, None) == B.QV_ERR_INVALID_ARG
    assert lib.qv_pbvi_result(C.byref(m.c), k, P, None, P, C.byref(added), 0x100, need, None) == B.QV_ERR_INVALID_ARG
