"""Convenience layer over the C ABI: device buffers and workspaces for one
problem, and readers for the tree records the library leaves in its
workspace.  All computation happens in libqvts.so."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import binding as B


class Planner:
    def __init__(self, prob, device="cuda", flags: int = 0, D=None, n=None):
        import torch
        self.torch = torch
        self.prob = prob
        self.device = device
        self.flags = flags
        self.D = prob.D if D is None else D
        self.n = prob.n if n is None else n
        self.m = B.DeviceModel(prob, device)
        nb = B.qv_plan_workspace_bytes(self.m, self.D, self.n, flags)
        if nb == 0:
            raise B.QvError(B.QV_ERR_UNSUPPORTED, "qv_plan_workspace_bytes")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        st, self.layout = B.qv_plan_layout(self.m, self.D, self.n, flags)
        B.check(st, "qv_plan_layout")
        self.action = torch.zeros(1, dtype=torch.int32, device=device)
        self.rootQ = torch.zeros(self.m.A, dtype=torch.float32, device=device)
        self.b0 = torch.as_tensor(np.ascontiguousarray(prob.b0, np.float32)).to(device)

    # -- offline Q-MDP values ---------------------------------------------
    def value_iterate(self, tol=1e-6, max_sweeps=10000):
        torch = self.torch
        Q = torch.empty(self.m.S * self.m.A, dtype=torch.float32, device=self.device)
        ws = torch.empty(B.qv_vi_workspace_bytes(self.m, max_sweeps), dtype=torch.uint8,
                         device=self.device)
        st, res, sw = B.qv_value_iterate(self.m, tol, max_sweeps, Q, ws)
        B.check(st, "qv_value_iterate")
        return Q, res, sw

    # -- offline fast informed bound (its alpha vectors score leaves as a Q table)
    def fib_iterate(self, tol=1e-6, max_sweeps=10000):
        torch = self.torch
        al = torch.empty(self.m.S * self.m.A, dtype=torch.float32, device=self.device)
        ws = torch.empty(B.qv_fib_workspace_bytes(self.m, max_sweeps), dtype=torch.uint8,
                         device=self.device)
        st, res, sw = B.qv_fib_iterate(self.m, tol, max_sweeps, al, ws)
        B.check(st, "qv_fib_iterate")
        return al, res, sw

    # -- offline blind-policy vectors (a lower-bound table)
    def blind_iterate(self, tol=1e-6, max_sweeps=10000):
        torch = self.torch
        al = torch.empty(self.m.S * self.m.A, dtype=torch.float32, device=self.device)
        ws = torch.empty(B.qv_blind_workspace_bytes(self.m, max_sweeps), dtype=torch.uint8,
                         device=self.device)
        st, res, sw = B.qv_blind_iterate(self.m, tol, max_sweeps, al, ws)
        B.check(st, "qv_blind_iterate")
        return al, res, sw

    # -- one planning step ------------------------------------------------
    def plan(self, Q, b0=None, seed=None, query_id=None, stream=None):
        prob = self.prob
        st = B.qv_plan_step(self.m, Q, self.b0 if b0 is None else b0, self.D, self.n,
                            prob.seed if seed is None else seed,
                            prob.query_id if query_id is None else query_id, self.flags,
                            self.action, self.rootQ, self.ws, stream)
        B.check(st, "qv_plan_step")
        return self.action, self.rootQ

    # -- tree records -----------------------------------------------------
    def tree(self, beliefs: bool = True) -> dict:
        """Copies the tree records out of the workspace (after a sync)."""
        self.torch.cuda.synchronize()
        return read_tree(self.ws, self.layout, beliefs)

    def belief_of(self, d: int, slot: int):
        """One stored belief of level d as a float32 numpy array."""
        L = self.layout
        off = int(L.belief_offset[d])
        if not off:
            raise ValueError(f"level {d} beliefs are not stored")
        S = L.S
        start = off + slot * S * 4
        return self.ws[start:start + S * 4].cpu().numpy().view(np.float32).copy()


def read_tree(raw, L, beliefs: bool = True) -> dict:
    """Tree records described by layout L from the uint8 device tensor raw
    (a workspace, or the slice of one that holds a batch query)."""
    tot = int(L.level_first[L.D + 1])
    A, S = L.A, L.S

    def arr(off, count, dt):
        nbytes = count * np.dtype(dt).itemsize
        return raw[off:off + nbytes].cpu().numpy().view(dt).copy()

    out = dict(valid=arr(L.valid, tot, np.int32), z=arr(L.z, tot, np.int32),
               count=arr(L.count, tot, np.int32), pz=arr(L.pz, tot, np.float32),
               value=arr(L.value, tot, np.float32),
               qvalue=arr(L.qvalue, tot * A, np.float32),
               reward=arr(L.reward, tot * A, np.float32),
               level_first=[int(L.level_first[d]) for d in range(L.D + 2)],
               level_slots=[int(L.level_slots[d]) for d in range(L.D + 1)],
               tiles=int(L.tiles), tile_rows=int(L.tile_rows))
    if beliefs:
        out["beliefs"] = {}
        for d in range(1, L.D + 1):
            off = int(L.belief_offset[d])
            if off:
                out["beliefs"][d] = arr(off, int(L.level_slots[d]) * S, np.float32).reshape(-1, S)
    return out


def batch_key(probs, n: int, flags: int, device_name: str, lib_hash: str) -> str:
    """Key of a batch in the shape cache: what the batched launches' work
    depends on (every query's grid, actions, landmarks and depth; n; the
    flags), the device and the library build."""
    h = hashlib.sha256()
    h.update(json.dumps([int(n), int(flags), device_name, lib_hash]).encode())
    for p in probs:
        h.update(json.dumps([int(p.W), int(p.H), int(p.A), int(len(p.lm_cell)),
                             int(p.D)]).encode())
    return h.hexdigest()[:24]


class ShapeCache:
    """The batch shapes that autotuning chose, in a JSON file: {key:
    {"tile_cells", "chunk", "ms_per_batch"}}.  Entries are merged into the
    file and written through a temporary file, so concurrent writers lose at
    most their own entry."""

    def __init__(self, path: str):
        self.path = path

    def _read(self) -> dict:
        try:
            with open(self.path) as f:
                d = json.load(f)
            return d if isinstance(d, dict) else {}
        except (OSError, ValueError):
            return {}

    def get(self, key: str):
        e = self._read().get(key)
        if not isinstance(e, dict):
            return None
        try:
            return int(e["tile_cells"]), int(e["chunk"]), float(e["ms_per_batch"])
        except (KeyError, TypeError, ValueError):
            return None

    def put(self, key: str, tile_cells: int, chunk: int, ms: float):
        d = self._read()
        d[key] = {"tile_cells": int(tile_cells), "chunk": int(chunk), "ms_per_batch": float(ms)}
        tmp = f"{self.path}.{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


class BatchPlanner:
    """Many planning queries planned together (qv_batch_*): the problems'
    device arrays, their Q tables and start beliefs, one workspace."""

    def __init__(self, probs, Qs, device="cuda", n=None, flags: int = 0, b0s=None):
        import torch
        self.torch = torch
        self.probs = probs
        self.device = device
        self.n = probs[0].n if n is None else n
        self.models = [B.DeviceModel(p, device) for p in probs]
        self.Qs = [torch.as_tensor(np.ascontiguousarray(q, np.float32).reshape(-1)).to(device)
                   if not hasattr(q, "data_ptr") else q for q in Qs]
        b0s = [p.b0 for p in probs] if b0s is None else b0s
        self.b0s = [torch.as_tensor(np.ascontiguousarray(b, np.float32)).to(device)
                    if not hasattr(b, "data_ptr") else b for b in b0s]
        self.flags = flags
        st, self.h = B.qv_batch_create(self.models, [p.D for p in probs], self.n, flags)
        B.check(st, "qv_batch_create")
        nb = B.qv_batch_workspace_bytes(self.h)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        nq = len(probs)
        self.actions = torch.zeros(nq, dtype=torch.int32, device=device)
        self.rootQ = torch.zeros(nq * B.QV_MAX_ACTIONS, dtype=torch.float32, device=device)

    def close(self):
        if self.h is not None and self.h.value:
            B.check(B.qv_batch_destroy(self.h), "qv_batch_destroy")
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_shape(self, tile_cells: int, chunk: int):
        B.check(B.qv_batch_set_shape(self.h, tile_cells, chunk), "qv_batch_set_shape")

    def shape(self):
        st, tc, ch = B.qv_batch_get_shape(self.h)
        B.check(st, "qv_batch_get_shape")
        return tc, ch

    def plan(self, seed: int, stream=None):
        st = B.qv_batch_plan(self.h, self.Qs, self.b0s, seed, self.actions, self.rootQ,
                             self.ws, stream)
        B.check(st, "qv_batch_plan")
        return self.actions, self.rootQ.view(-1, B.QV_MAX_ACTIONS)

    def autotune(self, seed: int, reps: int = 3, stream=None, cache: str = None) -> float:
        """Time the candidate shapes (qv_batch_autotune) and keep the fastest;
        returns its ms per batch.  With `cache` (a JSON file path; default
        $QVTS_TUNE_CACHE), a batch of the same key takes the stored shape
        without timing, and a new choice is stored."""
        cache = cache or os.environ.get("QVTS_TUNE_CACHE")
        self.tuned_from_cache = False
        if cache:
            from .build import source_hash
            key = batch_key(self.probs, self.n, self.flags,
                            self.torch.cuda.get_device_name(self.device), source_hash())
            hit = ShapeCache(cache).get(key)
            if hit is not None:
                self.set_shape(hit[0], hit[1])
                self.tuned_from_cache = True
                return hit[2]
        st, ms = B.qv_batch_autotune(self.h, self.Qs, self.b0s, seed, self.actions, self.rootQ,
                                     reps, self.ws, stream)
        B.check(st, "qv_batch_autotune")
        if cache:
            tc, ch = self.shape()
            ShapeCache(cache).put(key, tc, ch, ms)
        return ms

    def tree(self, q: int, beliefs: bool = False) -> dict:
        self.torch.cuda.synchronize()
        st, L, off = B.qv_batch_layout(self.h, q)
        B.check(st, "qv_batch_layout")
        return read_tree(self.ws[off:off + int(L.total_bytes)], L, beliefs)


def belief_update(m: B.DeviceModel, b, a, z, check: bool = True, stream=None):
    """Batched filter step on device tensors; returns (b_out, p_out, status)."""
    import torch
    batch = int(a.numel())
    b_out = torch.zeros_like(b)
    p_out = torch.zeros(batch, dtype=torch.float32, device=b.device)
    ws = torch.empty(max(B.qv_belief_update_workspace_bytes(m, batch), 1), dtype=torch.uint8,
                     device=b.device)
    st = B.qv_belief_update(m, batch, b, a, z, b_out, p_out, 1 if check else 0, ws, stream)
    return b_out, p_out, st


class SearchPlanner:
    """Best-first (anytime) search over one problem (qv_search_*): the node
    pool's workspace, the two bound tables and readers of the node records."""

    def __init__(self, prob, Ut, Lt, max_nodes: int, device="cuda", n=None):
        import torch
        self.torch = torch
        self.prob = prob
        self.device = device
        self.n = prob.n if n is None else n
        self.max_nodes = int(max_nodes)
        self.m = B.DeviceModel(prob, device)

        def dev(t):
            return t if hasattr(t, "data_ptr") else torch.as_tensor(
                np.ascontiguousarray(t, np.float32).reshape(-1)).to(device)
        self.Ut, self.Lt = dev(Ut), dev(Lt)
        # columns of the lower-bound table (blind: A; PBVI: its point capacity)
        self.lcols = int(self.Lt.numel()) // prob.S
        nb = B.qv_search_workspace_bytes(self.m, self.n, self.max_nodes)
        if nb == 0:
            raise B.QvError(B.QV_ERR_UNSUPPORTED, "qv_search_workspace_bytes")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        st, self.layout = B.qv_search_layout_of(self.m, self.n, self.max_nodes)
        B.check(st, "qv_search_layout_of")
        self.action = torch.zeros(1, dtype=torch.int32, device=device)
        self.rootU = torch.zeros(self.m.A, dtype=torch.float32, device=device)
        self.rootL = torch.zeros(self.m.A, dtype=torch.float32, device=device)

    def init(self, b0=None, stream=None):
        b0 = self.prob.b0 if b0 is None else b0
        bt = b0 if hasattr(b0, "data_ptr") else self.torch.as_tensor(
            np.ascontiguousarray(b0, np.float32)).to(self.device)
        self._b0 = bt
        B.check(B.qv_search_init(self.m, self.Ut, self.Lt, self.lcols, bt, self.n, self.max_nodes,
                                 self.ws, stream), "qv_search_init")

    def expand(self, expansions: int, seed=None, query_id=None, stream=None):
        p = self.prob
        B.check(B.qv_search_expand(self.m, self.Ut, self.Lt, self.lcols, self.n, self.max_nodes,
                                   p.seed if seed is None else seed,
                                   p.query_id if query_id is None else query_id,
                                   int(expansions), self.ws, stream), "qv_search_expand")

    def result(self, stream=None):
        B.check(B.qv_search_result(self.m, self.n, self.max_nodes, self.action, self.rootU,
                                   self.rootL, self.ws, stream), "qv_search_result")
        return self.action, self.rootU, self.rootL

    def update(self, a: int, z: int, stream=None) -> int:
        return B.qv_search_update(self.m, self.Ut, self.Lt, self.lcols, self.n, self.max_nodes,
                                  int(a), int(z), self.ws, stream)

    def records(self, beliefs: bool = False) -> dict:
        """Copies the node records (and optionally the beliefs) out of the
        workspace (after a sync)."""
        self.torch.cuda.synchronize()
        L, raw, NV, A, S = self.layout, self.ws, self.max_nodes, self.prob.A, self.prob.S

        def arr(off, count, dt):
            nbytes = count * np.dtype(dt).itemsize
            return raw[off:off + nbytes].cpu().numpy().view(dt).copy()
        out = {k: arr(getattr(L, k), NV, np.int32) for k in
               ("valid", "z", "count", "parent", "depth", "E", "expanded", "child_base")}
        out.update({k: arr(getattr(L, k), NV, np.float32) for k in ("pz", "weight", "U", "L", "H")})
        out.update({k: arr(getattr(L, k), NV * A, np.float32).reshape(NV, A)
                    for k in ("rb", "UQ", "LQ", "HQ")})
        out["EQ"] = arr(L.EQ, NV * A, np.int32).reshape(NV, A)
        ctl = arr(L.ctl, 6, np.int32)
        out.update(root=int(ctl[0]), select=int(ctl[1]), next=int(ctl[2]),
                   expansions=int(ctl[3]), flags=int(ctl[4]), err=int(ctl[5]))
        out["log"] = arr(L.log, NV, np.int32)[:out["expansions"]]
        if beliefs:
            out["belief"] = arr(L.belief, NV * S, np.float32).reshape(NV, S)
        return out


class PbviPlanner:
    """Point-based value iteration over one problem (qv_pbvi_*): the
    workspace holding the point set and the vector tables, and readers of
    the state for tests and callers.  `init` is the starting vector table
    [S, init_cols] (e.g. the blind-policy vectors)."""

    def __init__(self, prob, init, max_points: int, device="cuda"):
        import torch
        self.torch = torch
        self.prob = prob
        self.device = device
        self.max_points = int(max_points)
        self.m = B.DeviceModel(prob, device)
        self.init_t = init if hasattr(init, "data_ptr") else torch.as_tensor(
            np.ascontiguousarray(init, np.float32).reshape(-1)).to(device)
        self.init_cols = int(self.init_t.numel()) // prob.S
        nb = B.qv_pbvi_workspace_bytes(self.m, self.max_points, self.init_cols)
        if nb == 0:
            raise B.QvError(B.QV_ERR_UNSUPPORTED, "qv_pbvi_workspace_bytes")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        st, self.layout = B.qv_pbvi_layout_of(self.m, self.max_points, self.init_cols)
        B.check(st, "qv_pbvi_layout_of")

    def init(self, b0=None, stream=None):
        b0 = self.prob.b0 if b0 is None else b0
        bt = b0 if hasattr(b0, "data_ptr") else self.torch.as_tensor(
            np.ascontiguousarray(b0, np.float32)).to(self.device)
        self._b0 = bt
        B.check(B.qv_pbvi_init(self.m, bt, self.init_t, self.init_cols, self.max_points, self.ws,
                               stream), "qv_pbvi_init")

    def expand(self, seed=None, query_id=0, stream=None) -> int:
        st, added = B.qv_pbvi_expand(self.m, self.init_cols, self.max_points,
                                     self.prob.seed if seed is None else seed, query_id, self.ws,
                                     stream)
        B.check(st, "qv_pbvi_expand")
        return added

    def backup(self, sweeps: int = 1, stream=None):
        B.check(B.qv_pbvi_backup(self.m, self.init_cols, self.max_points, int(sweeps), self.ws,
                                 stream), "qv_pbvi_backup")

    def table(self, ld=None, stream=None):
        """The vectors as a bound table [S * ld] (device; ld defaults to the
        point capacity) and the number of points."""
        ld = self.max_points if ld is None else int(ld)
        out = self.torch.empty(self.prob.S * ld, dtype=self.torch.float32, device=self.device)
        st, npts = B.qv_pbvi_result(self.m, self.init_cols, self.max_points, out, ld, self.ws,
                                    stream)
        B.check(st, "qv_pbvi_result")
        return out, npts

    def state(self) -> dict:
        """Copies the point set, the current vectors and the last expansion's
        and backup's records out of the workspace (after a sync)."""
        self.torch.cuda.synchronize()
        L, raw = self.layout, self.ws
        P, A, S, ZC, ld = self.max_points, self.prob.A, self.prob.S, L.ZC, L.ld

        def arr(off, count, dt):
            nbytes = count * np.dtype(dt).itemsize
            return raw[off:off + nbytes].cpu().numpy().view(dt).copy()
        ctl = arr(L.ctl, 5, np.int32)
        npts, rnd, cur, cols, added = (int(v) for v in ctl)
        G = arr(L.gamma1 if cur else L.gamma0, S * ld, np.float32).reshape(S, ld)[:, :cols]
        out = {"points": arr(L.points, P * S, np.float32).reshape(P, S)[:npts],
               "gamma": G, "round": rnd, "added": added, "cols": cols,
               "idx": arr(L.idx, P * A * ZC, np.int32).reshape(P, A, ZC)[:npts],
               "vals": arr(L.vals, P * A, np.float32).reshape(P, A)[:npts],
               "pick": arr(L.pick, P, np.int32)[:npts],
               "alpha": arr(L.cand, P * A * S, np.float32).reshape(P, A, S)[:npts],
               "dist": arr(L.dist, P * A, np.float32).reshape(P, A),
               "draw_valid": arr(L.dvalid, P * A, np.int32).reshape(P, A),
               "draw_z": arr(L.dz, P * A, np.int32).reshape(P, A),
               "src": arr(L.src, P, np.int32)}
        return out
