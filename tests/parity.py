"""Comparison of a GPU planning tree with the FP64 oracle's tree.

Protocol (both sides get the same seeded inputs and the same FP32 Q table,
the oracle widening it exactly to FP64):

* discrete results -- which child slots exist, their observation z and
  frequency, the root action -- must match exactly;
* a mismatch is excused only where the oracle's own decision margin lies
  inside the FP32 error band: an observation draw whose target u*P lies
  within DRAW_BAND*P of a running total, or a root action whose two best
  Q-values differ by at most ACTION_BAND*max(1,|Q|).  The subtree under an
  excused Q-node, and the values of its ancestors, are left out;
* continuous results (P(z|b,a), beliefs, R(b,a), Q-node and node values)
  must agree to a relative 1e-5, beliefs with an absolute floor of
  1e-12 * max(b_ref) for values near zero.
"""
import numpy as np

DRAW_BAND = 3e-5
ACTION_BAND = 1e-5
REL = 1e-5

# Session totals, printed at the end of the pytest run (tests/conftest.py):
# compared trees, nodes and beliefs, and every excused draw or root action
# with its oracle margin.
TOTALS = {"trees": 0, "nodes": 0, "beliefs": 0, "draws_excused": [], "actions_excused": []}


class Report:
    def __init__(self):
        self.nodes = 0
        self.beliefs = 0
        self.excused = []


def compare_tree(prob, g, o, check_beliefs=True, rel=REL):
    """g: Planner.tree() dict; o: oracle TreeDump.  Returns a Report."""
    A, n, D = prob.A, prob.n, prob.D
    K = A * n
    rep = Report()
    lf = g["level_first"]
    skip = np.zeros(int(lf[D + 1]), dtype=bool)       # excluded subtrees
    tainted = np.zeros(int(lf[D + 1]), dtype=bool)    # values not comparable
    # discrete structure, top-down
    for d in range(D):
        for slot in range(K ** d):
            gs = lf[d] + slot
            if skip[gs] or not o.valid[gs]:
                continue
            for a in range(A):
                kids = lf[d + 1] + slot * K + a * n + np.arange(n)
                same = (np.array_equal(g["valid"][kids], o.valid[kids].astype(np.int32))
                        and np.array_equal(g["z"][kids][o.valid[kids] == 1],
                                           o.z[kids][o.valid[kids] == 1])
                        and np.array_equal(g["count"][kids][o.valid[kids] == 1],
                                           o.count[kids][o.valid[kids] == 1]))
                if not same:
                    mg = o.margin[(gs * A + a) * n:(gs * A + a + 1) * n].min()
                    assert mg <= DRAW_BAND, (
                        f"level {d} slot {slot} action {a}: z {g['z'][kids]} vs {o.z[kids]}, "
                        f"counts {g['count'][kids]} vs {o.count[kids]}, margin {mg:.3g}")
                    rep.excused.append((d, slot, a, float(mg)))
                    skip[kids] = True
                    # ancestors' values depend on this Q-node
                    p = gs
                    for dd in range(d, -1, -1):
                        tainted[p] = True
                        if dd > 0:
                            p = lf[dd - 1] + (p - lf[dd]) // K
                    _skip_subtree(skip, lf, kids, K, d + 1, D)
    # continuous values, node by node
    for d in range(D + 1):
        for slot in range(K ** d):
            gs = lf[d] + slot
            if skip[gs] or not o.valid[gs]:
                continue
            rep.nodes += 1
            if d >= 1:
                assert abs(g["pz"][gs] - o.pz[gs]) <= rel * abs(o.pz[gs]), (d, slot, g["pz"][gs], o.pz[gs])
            if not tainted[gs]:
                V = o.V[gs]
                assert abs(g["value"][gs] - V) <= rel * max(1.0, abs(V)), (d, slot, g["value"][gs], V)
            if d < D:
                rb = o.rb[gs * A:(gs + 1) * A]
                np.testing.assert_allclose(g["reward"][gs * A:(gs + 1) * A], rb,
                                           rtol=rel, atol=rel * max(1.0, np.abs(rb).max()))
                if not tainted[gs]:
                    qt = o.qtree[gs * A:(gs + 1) * A]
                    np.testing.assert_allclose(g["qvalue"][gs * A:(gs + 1) * A], qt, rtol=0,
                                               atol=rel * max(1.0, np.abs(qt).max()))
            if check_beliefs and d >= 1 and d in g.get("beliefs", {}) and o.beliefs is not None:
                gb = g["beliefs"][d][slot].astype(np.float64)
                ob = o.beliefs[gs * prob.S:(gs + 1) * prob.S]
                tol = rel * np.abs(ob) + 1e-12 * ob.max()
                bad = np.abs(gb - ob) > tol
                assert not bad.any(), (d, slot, np.flatnonzero(bad)[:5], gb[bad][:5], ob[bad][:5])
                rep.beliefs += 1
    TOTALS["trees"] += 1
    TOTALS["nodes"] += rep.nodes
    TOTALS["beliefs"] += rep.beliefs
    TOTALS["draws_excused"].extend((prob.name,) + e for e in rep.excused)
    return rep


def _skip_subtree(skip, lf, kids, K, d, D):
    cur = [int(k) for k in kids]
    while d < D:
        nxt = []
        for gs in cur:
            slot = gs - lf[d]
            ch = lf[d + 1] + slot * K + np.arange(K)
            skip[ch] = True
            nxt.extend(int(c) for c in ch)
        cur = nxt
        d += 1


def root_action_ok(g_action, o_rootQ, o_action):
    """True if the actions agree or the oracle's top two are within the band."""
    if g_action == o_action:
        return True
    q = np.sort(o_rootQ)[::-1]
    ok = (q[0] - q[1]) <= ACTION_BAND * max(1.0, abs(q[0]))
    if ok:
        TOTALS["actions_excused"].append((int(g_action), int(o_action), float(q[0] - q[1])))
    return ok


def summary() -> str:
    t = TOTALS
    if not t["trees"]:
        return ""
    lines = [f"parity: {t['trees']} trees, {t['nodes']} nodes, {t['beliefs']} beliefs compared "
             f"with the oracle; {len(t['draws_excused'])} draws and "
             f"{len(t['actions_excused'])} root actions excused as near ties"]
    for e in t["draws_excused"]:
        lines.append(f"  excused draw: {e[0]} level {e[1]} slot {e[2]} action {e[3]}, "
                     f"oracle margin {e[4]:.3g} (band {DRAW_BAND:g})")
    for e in t["actions_excused"]:
        lines.append(f"  excused root action: gpu {e[0]} oracle {e[1]}, top-two gap {e[2]:.3g}")
    return "\n".join(lines)
