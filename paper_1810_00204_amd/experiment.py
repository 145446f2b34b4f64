"""Closed-loop runs of the planner (the outer loop of Alg. 1) on the GPU:
plan from the current belief (qv_plan_step), execute the chosen action in
the true world (workloads.Environment), receive the observation and move
the belief to Phi(b, a, z) (qv_belief_update), until the robot takes the
stay action (it declares that it has arrived) or a step cap is reached.
Per run it records the quantities of the paper's comparison table (Sec. V):
the discounted reward, collisions, steps, whether the run failed, and the
planning time per step.

The belief never leaves the GPU; per step the host reads back the chosen
action (4 bytes) and sends the observation (4 bytes).  A run's return is
sum_t gamma^t R(x_t, a_t) over the executed steps plus the tail of the
final stay, R(x_T, stay) / (1 - gamma) discounted by gamma^T (zero at the
target, -2 / (1 - gamma) elsewhere): after stopping, the robot stays put.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding as B
from . import workloads as wl


class ClosedLoop:
    """One problem's device arrays, a leaf table and the buffers of a
    closed-loop run."""

    def __init__(self, prob, Q, device="cuda", D=None, n=None, flags: int = 0):
        import torch
        self.torch = torch
        self.prob = prob
        self.device = device
        self.D = prob.D if D is None else D
        self.n = prob.n if n is None else n
        self.flags = flags
        self.m = B.DeviceModel(prob, device)
        self.Q = Q if hasattr(Q, "data_ptr") else torch.as_tensor(
            np.ascontiguousarray(Q, np.float32).reshape(-1)).to(device)
        nb = B.qv_plan_workspace_bytes(self.m, self.D, self.n, flags)
        if nb == 0:
            raise B.QvError(B.QV_ERR_UNSUPPORTED, "qv_plan_workspace_bytes")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        self.bws = torch.empty(max(B.qv_belief_update_workspace_bytes(self.m, 1), 256),
                               dtype=torch.uint8, device=device)
        self.b = [torch.empty(prob.S, dtype=torch.float32, device=device) for _ in range(2)]
        self.action = torch.zeros(1, dtype=torch.int32, device=device)
        self.rootQ = torch.zeros(self.m.A, dtype=torch.float32, device=device)
        self.z = torch.zeros(1, dtype=torch.int32, device=device)
        self.p = torch.zeros(1, dtype=torch.float32, device=device)
        self.z_host = torch.zeros(1, dtype=torch.int32).pin_memory()

    def run(self, env: wl.Environment, seed: int, max_steps: int = 400, b0=None) -> dict:
        """One closed-loop run from the problem's start belief (or b0).
        Query id t draws step t's observations, so a run is reproducible
        from (seed, env seed)."""
        torch = self.torch
        prob = self.prob
        stop = int(prob.meta.get("stop_action", -1))
        target = int(prob.meta.get("target", prob.goal))
        b0 = prob.b0 if b0 is None else b0
        self.b[0].copy_(torch.as_tensor(np.ascontiguousarray(b0, np.float32)))
        cur = 0
        ret, disc, collisions = 0.0, 1.0, 0
        actions, observations, states, plan_ms = [], [], [env.s], []
        success, lost = False, False
        steps = 0
        for t in range(max_steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.check(B.qv_plan_step(self.m, self.Q, self.b[cur], self.D, self.n, seed, t,
                                   self.flags, self.action, self.rootQ, self.ws),
                    "qv_plan_step")
            a = int(self.action.item())
            plan_ms.append((time.perf_counter() - t0) * 1e3)
            actions.append(a)
            x = env.s
            ret += disc * float(prob.R[x, a])
            if a == stop:
                # the robot declares arrival and stays put from here on
                tail = float(prob.R[x, a]) * prob.gamma / (1.0 - prob.gamma)
                ret += disc * tail
                success = x == target
                break
            z, hit = env.step(a)
            collisions += int(hit)
            steps += 1
            observations.append(z)
            states.append(env.s)
            disc *= prob.gamma
            self.z_host[0] = z
            self.z.copy_(self.z_host, non_blocking=True)
            st = B.qv_belief_update(self.m, 1, self.b[cur], self.action, self.z, self.b[1 - cur],
                                    self.p, 1, self.bws)
            if st == B.QV_ERR_ZERO_LIKELIHOOD:
                lost = True   # the belief no longer covers the true cell (FP32 underflow)
                break
            B.check(st, "qv_belief_update")
            cur = 1 - cur
        torch.cuda.synchronize()
        return {"return": ret, "collisions": collisions, "steps": steps, "success": success,
                "stopped": bool(actions) and actions[-1] == stop, "lost": lost,
                "plan_ms": plan_ms, "actions": actions, "observations": observations,
                "states": states, "belief": self.b[cur].cpu().numpy()}


class SearchLoop:
    """The same closed loop with the anytime planner of Alg. 1: each step
    runs a budget of best-first expansions (qv_search_expand), takes
    getOptimalAction (qv_search_result), and after the world's answer calls
    update(a, z) (qv_search_update), which keeps the drawn child's subtree or
    roots the posterior; the root's belief is the filter's belief.  When the
    node pool is more than half used the tree restarts from the root belief."""

    def __init__(self, prob, Ut, Lt, expansions: int, max_nodes=None, device="cuda", n=None):
        import torch
        from .planner import SearchPlanner
        self.torch = torch
        self.prob = prob
        self.expansions = int(expansions)
        n = prob.n if n is None else n
        K = prob.A * n
        max_nodes = max_nodes or (1 + 4 * self.expansions * K)
        self.sp = SearchPlanner(prob, Ut, Lt, max_nodes, device=device, n=n)
        self.S = prob.S

    def _root_belief(self):
        g = self.sp.records()
        L = self.sp.layout
        off = int(L.belief) + g["root"] * self.S * 4
        return self.sp.ws[off:off + self.S * 4].view(self.torch.float32).clone(), g

    def run(self, env: wl.Environment, seed: int, max_steps: int = 400, b0=None) -> dict:
        torch = self.torch
        prob, sp = self.prob, self.sp
        stop = int(prob.meta.get("stop_action", -1))
        target = int(prob.meta.get("target", prob.goal))
        sp.init(prob.b0 if b0 is None else b0)
        ret, disc, collisions, steps = 0.0, 1.0, 0, 0
        actions, observations, states, plan_ms, restarts = [], [], [env.s], [], 0
        success, lost = False, False
        for t in range(max_steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sp.expand(self.expansions, seed=seed, query_id=t)
            act, _, _ = sp.result()
            a = int(act.item())
            plan_ms.append((time.perf_counter() - t0) * 1e3)
            actions.append(a)
            x = env.s
            ret += disc * float(prob.R[x, a])
            if a == stop:
                ret += disc * float(prob.R[x, a]) * prob.gamma / (1.0 - prob.gamma)
                success = x == target
                break
            z, hit = env.step(a)
            collisions += int(hit)
            steps += 1
            observations.append(z)
            states.append(env.s)
            disc *= prob.gamma
            st = sp.update(a, z)
            if st == B.QV_ERR_UNSUPPORTED:      # the pool is full: restart at the root
                b, _ = self._root_belief()
                sp.init(b)
                restarts += 1
                st = sp.update(a, z)
            if st == B.QV_ERR_ZERO_LIKELIHOOD:
                lost = True
                break
            B.check(st, "qv_search_update")
            b, g = self._root_belief()
            if g["next"] > sp.max_nodes // 2:
                sp.init(b)
                restarts += 1
        torch.cuda.synchronize()
        b, _ = self._root_belief()
        return {"return": ret, "collisions": collisions, "steps": steps, "success": success,
                "stopped": bool(actions) and actions[-1] == stop, "lost": lost,
                "plan_ms": plan_ms, "actions": actions, "observations": observations,
                "states": states, "belief": b.cpu().numpy(), "restarts": restarts}


def summarize(runs) -> dict:
    """Mean and standard deviation over runs, as in the paper's comparison
    table: discounted reward, collisions, steps (of the successful runs),
    failure rate and planning time per step."""
    def ms(xs):
        xs = np.asarray(xs, dtype=np.float64)
        if xs.size == 0:
            return {"mean": None, "std": None}
        return {"mean": float(xs.mean()), "std": float(xs.std())}
    ok = [r for r in runs if r["success"]]
    plan = [m for r in runs for m in r["plan_ms"]]
    return {"runs": len(runs), "reward": ms([r["return"] for r in runs]),
            "collisions": ms([r["collisions"] for r in runs]),
            "steps": ms([r["steps"] for r in ok]),
            "failure_rate": 1.0 - len(ok) / max(1, len(runs)),
            "stopped": sum(1 for r in runs if r["stopped"]),
            "stopped_off_target": sum(1 for r in runs if r["stopped"] and not r["success"]),
            "lost": sum(1 for r in runs if r["lost"]),
            "steps_all_runs": ms([r["steps"] for r in runs]),
            "planning_ms_per_step": ms(plan)}

