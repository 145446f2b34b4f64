"""FP64 CPU oracle for the QV-tree search hot path -- TEST INFRASTRUCTURE.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never does, and the two share no code: the oracle is the plain C
file ``qvo.c`` compiled with gcc, driven from here through ctypes.

Every function takes a ``workloads.Problem``-like object; FP32 inputs are
widened exactly to FP64 and all arithmetic is FP64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qvo.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source built with AddressSanitizer and UndefinedBehaviorSanitizer;
# loaded instead of the plain build when QVO_SANITIZED=1 (the process must
# preload gcc's libasan and libubsan)
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-g"]


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile ``qvo.c`` with gcc (strict IEEE FP64: no fast-math, no FMA
    contraction) into ``liboracle.so`` (``liboracle_san.so`` with the
    sanitizers)."""
    out = _LIB_SAN if sanitize else _LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math",
                               "-Wall", "-Wextra"] + (SAN_FLAGS if sanitize else []) +
                              ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


class _Model(C.Structure):
    _fields_ = [("W", C.c_int), ("H", C.c_int),
                ("occ", C.POINTER(C.c_ubyte)),
                ("A", C.c_int),
                ("slip", C.POINTER(C.c_double)),
                ("flip", C.POINTER(C.c_double)),
                ("L", C.c_int),
                ("lm_cell", C.POINTER(C.c_int)),
                ("lm_p", C.c_double),
                ("R", C.POINTER(C.c_double)),
                ("goal", C.c_int),
                ("gamma", C.c_double)]


class _Dump(C.Structure):
    _fields_ = [("valid", C.POINTER(C.c_ubyte)),
                ("z", C.POINTER(C.c_int)),
                ("count", C.POINTER(C.c_int)),
                ("pz", C.POINTER(C.c_double)),
                ("V", C.POINTER(C.c_double)),
                ("qtree", C.POINTER(C.c_double)),
                ("rb", C.POINTER(C.c_double)),
                ("margin", C.POINTER(C.c_double)),
                ("beliefs", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        san = os.environ.get("QVO_SANITIZED") == "1"
        path = _LIB_SAN if san else _LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build(force=True, sanitize=san)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        mp = C.POINTER(_Model)
        L.qvo_predict.argtypes = [mp, dp, C.c_int, dp]
        L.qvo_predict.restype = None
        L.qvo_likelihood.argtypes = [mp, dp, dp]
        L.qvo_obs_prob.argtypes = [mp, C.c_int, C.c_int]
        L.qvo_obs_prob.restype = C.c_double
        L.qvo_belief_update.argtypes = [mp, C.c_int, dp, ip, ip, dp, dp]
        L.qvo_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                       C.POINTER(C.c_uint32)]
        L.qvo_philox4x32_10.restype = None
        L.qvo_obs_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_uint32,
                                     C.c_int, C.c_int, C.c_int]
        L.qvo_obs_uniform.restype = C.c_double
        L.qvo_draw_obs.argtypes = [dp, C.c_int, C.c_double, dp]
        L.qvo_alg4_sample.argtypes = [mp, dp, C.c_int, C.c_int, C.c_uint64, ip]
        L.qvo_value_iterate.argtypes = [mp, C.c_double, C.c_int, dp, dp, ip]
        L.qvo_tree_slots.argtypes = [C.c_int, C.c_int, C.c_int]
        L.qvo_tree_slots.restype = C.c_long
        L.qvo_plan.argtypes = [mp, dp, dp, C.c_int, C.c_int, C.c_uint64, C.c_uint32,
                              C.c_int, ip, dp, C.POINTER(_Dump), C.POINTER(C.c_long)]
        L.qvo_expand_node.argtypes = [mp, dp, C.c_int, C.c_long, C.c_int, C.c_uint64,
                                      C.c_uint32, ip, ip, ip, dp, dp, dp, dp]
        L.qvo_leaf_score.argtypes = [mp, dp, dp]
        L.qvo_leaf_score.restype = C.c_double
        L.qvo_filter_nll_grad.argtypes = [mp, dp, dp, C.c_int, C.c_int, dp, ip, ip,
                                         dp, dp, dp]
        L.qvo_fib_iterate.argtypes = [mp, dp, C.c_double, C.c_int, dp, dp, ip]
        L.qvo_blind_iterate.argtypes = [mp, C.c_double, C.c_int, dp, dp, ip]
        L.qvo_fib_backup_cells.argtypes = [mp, dp, C.c_int, ip, dp]
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Model:
    """FP64 copy of a problem's model arrays, kept alive for the C calls."""

    def __init__(self, prob, slip=None, flip=None):
        self.W, self.H = int(prob.W), int(prob.H)
        self.occ = np.ascontiguousarray(prob.occ, dtype=np.uint8)
        self.slip = np.ascontiguousarray(prob.slip if slip is None else slip,
                                         dtype=np.float64).reshape(-1)
        self.A = self.slip.size // 9
        self.flip = np.ascontiguousarray(prob.flip if flip is None else flip,
                                         dtype=np.float64)
        self.lm = np.ascontiguousarray(prob.lm_cell, dtype=np.int32)
        self.R = np.ascontiguousarray(prob.R, dtype=np.float64).reshape(-1)
        self.c = _Model(self.W, self.H, _ptr(self.occ, C.c_ubyte), self.A,
                        _ptr(self.slip, C.c_double), _ptr(self.flip, C.c_double),
                        int(self.lm.size), _ptr(self.lm, C.c_int),
                        float(np.float32(prob.lm_p)), _ptr(self.R, C.c_double),
                        int(prob.goal), float(np.float32(prob.gamma)))
        self.S = self.W * self.H
        self.Z = 16 * (int(self.lm.size) + 1)

    @property
    def ref(self):
        return C.byref(self.c)


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def predict(prob, b, a) -> np.ndarray:
    m = Model(prob)
    b = _f64(b)
    out = np.zeros(m.S)
    lib().qvo_predict(m.ref, _ptr(b, C.c_double), int(a), _ptr(out, C.c_double))
    return out


def likelihood(prob, bp) -> np.ndarray:
    m = Model(prob)
    bp = _f64(bp)
    p = np.zeros(m.Z)
    st = lib().qvo_likelihood(m.ref, _ptr(bp, C.c_double), _ptr(p, C.c_double))
    assert st == 0
    return p


def obs_prob(prob, z, s) -> float:
    m = Model(prob)
    return float(lib().qvo_obs_prob(m.ref, int(z), int(s)))


def belief_update(prob, b, a, z):
    """Batched filter step; returns (posterior [batch, S], p [batch], status)."""
    m = Model(prob)
    b = _f64(b).reshape(-1, m.S)
    bt = b.shape[0]
    a = np.ascontiguousarray(np.broadcast_to(a, (bt,)), dtype=np.int32)
    z = np.ascontiguousarray(np.broadcast_to(z, (bt,)), dtype=np.int32)
    out = np.zeros_like(b)
    p = np.zeros(bt)
    st = lib().qvo_belief_update(m.ref, bt, _ptr(b, C.c_double), _ptr(a, C.c_int),
                                 _ptr(z, C.c_int), _ptr(out, C.c_double),
                                 _ptr(p, C.c_double))
    return out, p, int(st)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().qvo_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return o


def obs_uniform(seed, qid, level, slot, a, n, k) -> float:
    return float(lib().qvo_obs_uniform(C.c_uint64(seed), qid, level, slot, a, n, k))


def draw_obs(p, u):
    """Inverse-CDF observation draw; returns (z, margin)."""
    p = _f64(p)
    mg = C.c_double(0.0)
    z = lib().qvo_draw_obs(_ptr(p, C.c_double), int(p.size), float(u), C.byref(mg))
    return int(z), mg.value


def alg4_sample(prob, b, a, nsamp, seed) -> np.ndarray:
    m = Model(prob)
    b = _f64(b)
    out = np.zeros(nsamp, dtype=np.int32)
    st = lib().qvo_alg4_sample(m.ref, _ptr(b, C.c_double), int(a), int(nsamp),
                               C.c_uint64(seed), _ptr(out, C.c_int))
    assert st == 0
    return out


def value_iterate(prob, tol=1e-12, max_sweeps=100000):
    """Returns (Q [S, A] FP64, residual, sweeps)."""
    m = Model(prob)
    Q = np.zeros((m.S, m.A))
    res = C.c_double(0.0)
    sw = C.c_int(0)
    st = lib().qvo_value_iterate(m.ref, float(tol), int(max_sweeps),
                                 _ptr(Q, C.c_double), C.byref(res), C.byref(sw))
    assert st == 0
    return Q, res.value, sw.value


class TreeDump:
    """Capacity-slot tree records of one plan (see ``qvo.c``)."""

    def __init__(self, A, n, D, S, beliefs=False):
        self.A, self.n, self.D, self.S, self.K = A, n, D, S, A * n
        self.level_size = [self.K ** d for d in range(D + 1)]
        self.level_off = np.concatenate([[0], np.cumsum(self.level_size)]).astype(np.int64)
        tot = int(self.level_off[-1])
        self.valid = np.zeros(tot, dtype=np.uint8)
        self.z = np.full(tot, -1, dtype=np.int32)
        self.count = np.zeros(tot, dtype=np.int32)
        self.pz = np.zeros(tot)
        self.V = np.full(tot, np.nan)
        self.qtree = np.full(tot * A, np.nan)
        self.rb = np.full(tot * A, np.nan)
        self.margin = np.full(tot * A * n, np.inf)
        self.beliefs = np.zeros(tot * S) if beliefs else None
        self.c = _Dump(_ptr(self.valid, C.c_ubyte), _ptr(self.z, C.c_int),
                       _ptr(self.count, C.c_int), _ptr(self.pz, C.c_double),
                       _ptr(self.V, C.c_double), _ptr(self.qtree, C.c_double),
                       _ptr(self.rb, C.c_double), _ptr(self.margin, C.c_double),
                       _ptr(self.beliefs, C.c_double) if beliefs else None)

    def level(self, arr, d, width=1):
        o, n = int(self.level_off[d]), self.level_size[d]
        return arr[o * width:(o + n) * width]


def plan(prob, Q, b0=None, D=None, n=None, seed=None, qid=None, full=False,
         dump: Optional[TreeDump] = None, dump_beliefs=False):
    """One planning step; returns dict(action, rootQ, expansions, dump)."""
    m = Model(prob)
    D = prob.D if D is None else D
    n = prob.n if n is None else n
    seed = prob.seed if seed is None else seed
    qid = prob.query_id if qid is None else qid
    Qd = _f64(Q).reshape(-1)
    b0 = _f64(prob.b0 if b0 is None else b0)
    if dump is None and not full:
        dump = TreeDump(m.A, n, D, m.S, beliefs=dump_beliefs)
    act = C.c_int(-1)
    rq = np.zeros(m.A)
    ex = C.c_long(0)
    st = lib().qvo_plan(m.ref, _ptr(Qd, C.c_double), _ptr(b0, C.c_double), int(D), int(n),
                        C.c_uint64(seed), int(qid), 1 if full else 0, C.byref(act),
                        _ptr(rq, C.c_double), C.byref(dump.c) if dump is not None else None,
                        C.byref(ex))
    assert st == 0, st
    return dict(action=act.value, rootQ=rq, expansions=ex.value, dump=dump)


def expand_node(prob, b, d, slot, n=None, seed=None, qid=None, beliefs=True):
    """One V-node expansion of belief b at (level d, capacity slot); returns a
    dict of per-(action, rank) child records, child beliefs and R(b, a)."""
    m = Model(prob)
    n = prob.n if n is None else n
    seed = prob.seed if seed is None else seed
    qid = prob.query_id if qid is None else qid
    b = _f64(b)
    K = m.A * n
    valid = np.zeros(K, np.int32)
    z = np.zeros(K, np.int32)
    cnt = np.zeros(K, np.int32)
    pz = np.zeros(K)
    mg = np.zeros(K)
    bel = np.zeros(K * m.S) if beliefs else None
    rb = np.zeros(m.A)
    st = lib().qvo_expand_node(m.ref, _ptr(b, C.c_double), int(d), int(slot), int(n),
                               C.c_uint64(seed), int(qid), _ptr(valid, C.c_int), _ptr(z, C.c_int),
                               _ptr(cnt, C.c_int), _ptr(pz, C.c_double), _ptr(mg, C.c_double),
                               _ptr(bel, C.c_double) if beliefs else None, _ptr(rb, C.c_double))
    assert st == 0, st
    return dict(valid=valid, z=z, count=cnt, pz=pz, margin=mg, rb=rb,
                beliefs=bel.reshape(K, m.S) if beliefs else None)


def leaf_score(prob, Q, b) -> float:
    m = Model(prob)
    Qd = _f64(Q).reshape(-1)
    b = _f64(b)
    return float(lib().qvo_leaf_score(m.ref, _ptr(Qd, C.c_double), _ptr(b, C.c_double)))


def filter_nll_grad(prob, theta, phi, acts, obs, b0=None):
    """Returns (nll per trajectory [ntraj], g_theta [A, 9], g_phi [4])."""
    m = Model(prob)
    theta = _f64(theta).reshape(-1)
    phi = _f64(phi)
    acts = np.ascontiguousarray(acts, dtype=np.int32)
    obs = np.ascontiguousarray(obs, dtype=np.int32)
    ntraj, T = acts.shape
    b0 = _f64(prob.b0 if b0 is None else b0)
    if b0.ndim == 1:
        b0 = np.ascontiguousarray(np.broadcast_to(b0, (ntraj, m.S)))
    nll = np.zeros(ntraj)
    gt = np.zeros(theta.size)
    gp = np.zeros(4)
    m.c.A = theta.size // 9
    st = lib().qvo_filter_nll_grad(m.ref, _ptr(theta, C.c_double), _ptr(phi, C.c_double),
                                   int(ntraj), int(T), _ptr(b0, C.c_double),
                                   _ptr(acts, C.c_int), _ptr(obs, C.c_int),
                                   _ptr(nll, C.c_double), _ptr(gt, C.c_double),
                                   _ptr(gp, C.c_double))
    assert st == 0, st
    return nll, gt.reshape(-1, 9), gp


def fib_iterate(prob, tol=1e-12, max_sweeps=100000, init=None):
    """Fast informed bound by Jacobi sweeps of its alpha-vector equation
    (Sec. IV-A); returns (alpha [S, A] FP64, residual, sweeps)."""
    m = Model(prob)
    al = np.zeros((m.S, m.A))
    ini = None if init is None else _f64(init).reshape(-1)
    res = C.c_double(0.0)
    sw = C.c_int(0)
    st = lib().qvo_fib_iterate(m.ref, _ptr(ini, C.c_double) if ini is not None else None,
                               float(tol), int(max_sweeps), _ptr(al, C.c_double),
                               C.byref(res), C.byref(sw))
    assert st == 0, st
    return al, res.value, sw.value


def fib_backup(prob, alpha, cells):
    """Right-hand side of the FIB equation at the listed cells, given the
    vectors alpha [S, A]; returns [len(cells), A]."""
    m = Model(prob)
    al = _f64(alpha).reshape(-1)
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    out = np.zeros((cells.size, m.A))
    st = lib().qvo_fib_backup_cells(m.ref, _ptr(al, C.c_double), int(cells.size),
                                    _ptr(cells, C.c_int), _ptr(out, C.c_double))
    assert st == 0, st
    return out


def blind_iterate(prob, tol=1e-12, max_sweeps=100000):
    """Blind-policy vectors (the value of taking one action forever), the
    lower bound of the search; returns (alpha [S, A] FP64, residual, sweeps)."""
    m = Model(prob)
    al = np.zeros((m.S, m.A))
    res = C.c_double(0.0)
    sw = C.c_int(0)
    st = lib().qvo_blind_iterate(m.ref, float(tol), int(max_sweeps), _ptr(al, C.c_double),
                                 C.byref(res), C.byref(sw))
    assert st == 0, st
    return al, res.value, sw.value


class SearchTree:
    """Best-first QV-tree (Alg. 1, 2, 5, 6, 7 with the heuristics of Sec. IV-C),
    FP64.  Node ids follow the allocation rule of the search: the root is
    node 0; each expansion reserves K = |A| n consecutive ids, child (a, r)
    of the expansion taking id base + a n + r; a new root made by update(a, z)
    takes one id.  Each node keeps its belief, parent (node, action), weight
    f/n, observation, depth, bounds U, L, heuristic H and node to expand E;
    each expanded node keeps per action R(b,a), U_Q, L_Q, H_Q and E_Q."""

    def __init__(self, prob, Ut, Lt, n, seed, qid, b0, tie=1e-9):
        self.prob, self.n, self.seed, self.qid = prob, n, seed, qid
        self.Ut = _f64(Ut).reshape(prob.S, prob.A)
        # V_L(b) = max over the lower table's columns (A blind vectors, or
        # one vector per point of a point-based bound)
        self.Lt = _f64(Lt).reshape(prob.S, -1)
        # gamma as the model carries it (an FP32 input, widened exactly)
        self.A, self.K, self.g = prob.A, prob.A * n, float(np.float32(prob.gamma))
        self.nodes = {}
        self.next = 0
        self.log = []          # expanded node per expansion
        self.margins = []      # closest decision of the update that set E[root]
        self.root = self._new(_f64(b0), None, 1.0, -1, 0)

    # Alg. 5: a new V-node takes U_V = V_U(b), L_V = V_L(b), H = U - L, E = itself
    def _new(self, b, parent, w, z, depth, nid=None):
        if nid is None:
            nid = self.next
            self.next += 1
        U = float(np.max(b @ self.Ut))
        L = float(np.max(b @ self.Lt))
        self.nodes[nid] = dict(b=b, parent=parent, w=w, z=z, depth=depth, U=U, L=L, H=U - L,
                               E=nid, q=None, kids=None)
        return nid

    def expand(self):
        """findVNodeToExpand, expand, then update every ancestor (Alg. 1)."""
        v = self.nodes[self.root]["E"]
        nd = self.nodes[v]
        if nd["q"] is not None:
            return False
        ex = expand_node(self.prob, nd["b"], nd["depth"], v, n=self.n, seed=self.seed,
                         qid=self.qid, beliefs=True)
        base = self.next
        self.next += self.K
        kids = []
        for a in range(self.A):
            row = []
            for r in range(self.n):
                c = a * self.n + r
                if ex["valid"][c]:
                    row.append(self._new(ex["beliefs"][c], (v, a), ex["count"][c] / self.n,
                                         int(ex["z"][c]), nd["depth"] + 1, nid=base + c))
            kids.append(row)
        nd["kids"] = kids
        nd["rb"] = ex["rb"].copy()
        self.log.append(v)
        margin = np.inf
        p = v
        while p is not None:
            margin = min(margin, self._update(p))
            par = self.nodes[p]["parent"]
            p = None if par is None else par[0]
        self.margins.append(margin)
        return True

    def _update(self, v):
        """Alg. 6 for every action of v, then Alg. 7 (with gamma in the
        Q-node backup and H(b,a) = 1 for the action of largest U_Q only);
        returns the smallest relative gap among the argmax decisions taken."""
        nd, g = self.nodes[v], self.g
        UQ, LQ, HQ, EQ = [], [], [], []
        gap = np.inf
        for a in range(self.A):
            kids = nd["kids"][a]
            u = nd["rb"][a] + g * sum(self.nodes[c]["w"] * self.nodes[c]["U"] for c in kids)
            l = nd["rb"][a] + g * sum(self.nodes[c]["w"] * self.nodes[c]["L"] for c in kids)
            h = [g * self.nodes[c]["w"] * self.nodes[c]["H"] for c in kids]
            j = int(np.argmax(h))
            if len(h) > 1:
                srt = np.sort(h)[::-1]
                gap = min(gap, (srt[0] - srt[1]) / max(abs(srt[0]), 1e-30))
            UQ.append(u)
            LQ.append(l)
            HQ.append(h[j])
            EQ.append(self.nodes[kids[j]]["E"])
        a_star = int(np.argmax(UQ))
        srt = np.sort(UQ)[::-1]
        if self.A > 1:
            gap = min(gap, (srt[0] - srt[1]) / max(1.0, abs(srt[0])))
        nd.update(q=dict(UQ=np.array(UQ), LQ=np.array(LQ), HQ=np.array(HQ), EQ=np.array(EQ)),
                  U=float(max(UQ)), L=float(max(LQ)), H=float(HQ[a_star]), E=int(EQ[a_star]))
        return gap

    def action(self, tie=1e-9):
        """getOptimalAction: the lowest action whose lower bound L_Q at the
        root is within 1e-9 of the largest."""
        q = self.nodes[self.root]["q"]
        lq = q["LQ"]
        return int(np.flatnonzero(lq >= lq.max() - tie)[0])

    def update(self, a, z):
        """update(a, z): the root moves to its child under (a, z), keeping that
        subtree; if z was not drawn there, a new root is formed from Phi(b, a, z)."""
        nd = self.nodes[self.root]
        if nd["q"] is not None:
            for c in nd["kids"][a]:
                if self.nodes[c]["z"] == z:
                    self.root = c
                    self.nodes[c]["parent"] = None
                    return c
        b, p, st = belief_update(self.prob, nd["b"], a, z)
        assert st == 0 and p[0] > 0
        self.root = self._new(b[0], None, 1.0, z, nd["depth"] + 1)
        return self.root


def search(prob, Ut, Lt, expansions, n=None, seed=None, qid=None, b0=None):
    """A best-first search of `expansions` expansions from b0 (default: the
    problem's); returns the SearchTree."""
    t = SearchTree(prob, Ut, Lt, prob.n if n is None else n,
                   prob.seed if seed is None else seed,
                   prob.query_id if qid is None else qid,
                   prob.b0 if b0 is None else b0)
    for _ in range(expansions):
        if not t.expand():
            break
    return t


# ---------------------------------------------------------------------------
# Point-based value iteration (Sec. IV-B), FP64, numpy on the oracle's own
# model pieces (prediction, likelihood, observation probabilities, draws).
# ---------------------------------------------------------------------------

def _successor_table(prob):
    """dest[x, k]: the cell that neighbour move k leads to from x (the cell
    itself when the target is blocked or off the grid; the goal and blocked
    cells keep every move at themselves)."""
    W, H = prob.W, prob.H
    occ = np.asarray(prob.occ).reshape(-1)
    dest = np.zeros((W * H, 9), dtype=np.int64)
    for x in range(W * H):
        y0, x0 = divmod(x, W)
        for k in range(9):
            dy, dx = k // 3 - 1, k % 3 - 1
            yy, xx = y0 + dy, x0 + dx
            t = yy * W + xx
            ok = 0 <= yy < H and 0 <= xx < W and not occ[t]
            dest[x, k] = t if ok and not occ[x] and x != prob.goal else x
    return dest


def _obs_table(prob):
    """O[x, z] = P(z | x) for every cell and observation."""
    m = Model(prob)
    O = np.zeros((m.S, m.Z))
    for x in range(m.S):
        if prob.occ[x]:
            continue
        for z in range(m.Z):
            O[x, z] = lib().qvo_obs_prob(m.ref, int(z), int(x))
    return O


class PBVI:
    """Point-based value iteration of Sec. IV-B: a set of belief points, one
    alpha vector per point, backed up with the PBVI Bellman equation:
      for every action a and observation z, the vector of Gamma best at the
      point's predicted belief weighted by O(z|.) (first maximum on ties);
      alpha_a = R_a + gamma sum_z T_a (O_z * alpha_{a,z});
      the point's new vector is the alpha_a of largest b.alpha_a.
    The set grows by the expansion the paper follows (Pineau et al.): every
    point draws one observation per action (inverse CDF on P(z|b,a), uniform
    from the Philox stream with counter (a, point, 64 + round, query)) and
    adds the posterior farthest in L1 from the current set (first maximum;
    not added at distance 0).  Gamma starts from `init` [S, k] (a lower
    bound, e.g. the blind-policy vectors); every backed-up vector is a
    policy's value, so V(b) = max_alpha b.alpha stays a lower bound."""

    def __init__(self, prob, init, seed, qid=0):
        self.prob, self.seed, self.qid = prob, seed, qid
        self.g = float(np.float32(prob.gamma))
        self.R = _f64(prob.R).reshape(prob.S, prob.A)
        self.dest = _successor_table(prob)
        self.slip = _f64(prob.slip).reshape(prob.A, 9)
        self.O = _obs_table(prob)
        self.free = np.asarray(prob.occ).reshape(-1) == 0
        self.B = [_f64(prob.b0)]
        self.Gamma = _f64(init).reshape(prob.S, -1).copy()
        self.rounds = 0
        self.draw_margins = []
        self.pick_gaps = []

    def _apply_T(self, a, v):
        """(T_a v)(x) = sum_x' T(x, a, x') v(x'); the goal is absorbing."""
        out = (v[self.dest] * self.slip[a][None, :]).sum(1)
        if self.prob.goal >= 0:
            out[self.prob.goal] = v[self.prob.goal]
        return out

    def expand(self):
        prob, A = self.prob, self.prob.A
        cur = np.array(self.B)
        new = []
        for i, b in enumerate(self.B):
            best, bd = None, 0.0
            for a in range(A):
                bp = predict(prob, b, a)
                p = likelihood(prob, bp)
                u = obs_uniform(self.seed, self.qid, 64 + self.rounds, i, a, 1, 0)
                z, mg = draw_obs(p, u)
                self.draw_margins.append(mg)
                post = self.O[:, z] * bp / p[z]
                d = float(np.abs(cur - post[None, :]).sum(1).min())
                if d > bd:
                    best, bd = post, d
            if best is not None:
                new.append(best)
        self.B.extend(new)
        self.rounds += 1
        return len(new)

    def backup(self):
        prob, A, g = self.prob, self.prob.A, self.g
        G = self.Gamma
        out = np.zeros((prob.S, len(self.B)))
        for i, b in enumerate(self.B):
            vals, cands = np.zeros(A), []
            for a in range(A):
                bp = predict(prob, b, a)
                # values of every vector at every observation: (O_z * b') . alpha
                V = (self.O * bp[:, None]).T @ G          # [Z, |Gamma|]
                idx = V.argmax(1)
                srt = np.sort(V, axis=1)
                if V.shape[1] > 1:
                    top = srt[:, -1]
                    self.pick_gaps.append(float(((top - srt[:, -2]) / np.maximum(np.abs(top), 1e-300)).min()))
                # sum_z T_a (O_z * alpha_{a,z}) = T_a (sum_z O_z * alpha_{a,z})
                acc = self._apply_T(a, (self.O * G[:, idx]).sum(1))
                al = np.where(self.free, self.R[:, a] + g * acc, 0.0)
                vals[a] = b @ al
                cands.append(al)
            out[:, i] = cands[int(np.argmax(vals))]
        self.Gamma = out
        return out

    def value(self, b):
        return float(np.max(_f64(b) @ self.Gamma))


def pbvi(prob, init, expansions, sweeps, seed, qid=0):
    """`expansions` rounds of (expand the point set, then `sweeps` backups)."""
    t = PBVI(prob, init, seed, qid)
    for _ in range(expansions):
        t.expand()
        for _ in range(sweeps):
            t.backup()
    return t
