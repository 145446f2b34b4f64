"""Seeded synthetic problem instances for the five workloads of this project.

This module builds *inputs* only: occupancy grids, slip tables, sensor
parameters, landmark cells, reward tables, start beliefs and logged
trajectories.  It computes no step of the planning method (no prediction,
likelihood, Bayes update, value iteration, leaf score or backup), so that the
HIP path and the FP64 oracle, which both consume these inputs, share no
arithmetic of the method.  Everything is deterministic in the seed.

Conventions shared by every consumer (they define the problem, Sec. II and
Sec. V of the paper):

* cell index ``s = y * W + x``; ``y = 0`` is the top row, "north" is ``y - 1``;
* neighbour index ``k = (dy + 1) * 3 + (dx + 1)`` for ``dy, dx in {-1, 0, 1}``,
  so ``k = 4`` is the cell itself, as in the 3x3 neighbour numbering of Sec. V;
* ``occ[s] = 1`` marks a blocked cell (the map m of Sec. II);
* the slip table ``slip[a, k]`` is T'(a, k), the free-space transition
  probability of moving to neighbour k under action a (Sec. V);
* observation ``z = zw + 16 * zl``: ``zw`` holds the four wall bits (bit 0 up,
  bit 1 left, bit 2 right, bit 3 down, the neighbours N1, N3, N5, N7 of
  Sec. V), ``zl`` is 0 or the id (1..L) of a landmark that reported itself.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 1810002040

# neighbour offsets (dy, dx) for k = 0..8
NEIGHBOURS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
K_OF = {d: k for k, d in enumerate(NEIGHBOURS)}

# action sets --------------------------------------------------------------
# four actions N, E, S, W: intended move 0.8, each perpendicular move 0.1
ACTIONS4 = [(-1, 0), (0, 1), (1, 0), (0, -1)]
# eight actions in clockwise ring order N, NE, E, SE, S, SW, W, NW
ACTIONS8 = [(-1, 0), (-1, 1), (0, 1), (1, 1), (1, 0), (1, -1), (0, -1), (-1, -1)]


def slip_table_4(p_main: float = 0.8, p_side: float = 0.1) -> np.ndarray:
    """T'(a, k) for N/E/S/W with perpendicular slip and no stay mass."""
    t = np.zeros((4, 9), dtype=np.float64)
    for a, d in enumerate(ACTIONS4):
        t[a, K_OF[d]] += p_main
        t[a, K_OF[ACTIONS4[(a + 1) % 4]]] += p_side
        t[a, K_OF[ACTIONS4[(a + 3) % 4]]] += p_side
    return t.astype(np.float32)


def slip_table_8(p_main: float = 0.7, p_adj: float = 0.1,
                 p_stay: float = 0.1) -> np.ndarray:
    """T'(a, k) for the 8-neighbour ring: the intended move, the two
    directions 45 degrees either side, and staying put."""
    t = np.zeros((8, 9), dtype=np.float64)
    for a, d in enumerate(ACTIONS8):
        t[a, K_OF[d]] += p_main
        t[a, K_OF[ACTIONS8[(a + 1) % 8]]] += p_adj
        t[a, K_OF[ACTIONS8[(a + 7) % 8]]] += p_adj
        t[a, 4] += p_stay
    return t.astype(np.float32)


def slip_table_9(p_main: float = 0.8, p_adj: float = 0.05,
                 p_stay: float = 0.1) -> np.ndarray:
    """T'(a, k) for the nine actions of Sec. V: action a aims at neighbour
    N_a (a = 4 is the robot's own cell, "stay").  A move lands on its target
    with p_main, on each of the two ring neighbours 45 degrees either side
    with p_adj, and stays with p_stay; the stay action stays surely.  (The
    paper gives T' only in a figure; these values are this project's.)"""
    t = np.zeros((9, 9), dtype=np.float64)
    for a in range(9):
        if a == 4:
            t[4, 4] = 1.0
            continue
        i = ACTIONS8.index(NEIGHBOURS[a])
        t[a, a] += p_main
        t[a, K_OF[ACTIONS8[(i + 1) % 8]]] += p_adj
        t[a, K_OF[ACTIONS8[(i + 7) % 8]]] += p_adj
        t[a, 4] += p_stay
    return t.astype(np.float32)


@dataclass
class Problem:
    """One planning (or filtering) problem: the tuple (X, A, Z, T, O, R, b0,
    gamma) of Sec. II, with T given by the map and the slip table, O by the
    wall-bit flip probabilities and the landmarks, plus the tree depth D and
    samples per action n of the online search."""

    name: str
    W: int
    H: int
    occ: np.ndarray                 # uint8 [H*W]
    slip: np.ndarray                # float32 [A, 9]
    flip: np.ndarray                # float32 [4]
    lm_cell: np.ndarray             # int32 [L], cell of landmark id l+1
    lm_p: float
    R: np.ndarray                   # float32 [S, A]
    goal: int                       # absorbing goal cell, -1 if none
    gamma: float
    b0: np.ndarray                  # float32 [S]
    D: int = 2
    n: int = 2
    seed: int = 0                   # Philox key for the observation draws
    query_id: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def S(self) -> int:
        return self.W * self.H

    @property
    def A(self) -> int:
        return int(self.slip.shape[0])

    @property
    def L(self) -> int:
        return int(self.lm_cell.shape[0])

    @property
    def Z(self) -> int:
        return 16 * (self.L + 1)

    @property
    def K(self) -> int:
        return self.A * self.n


# ---------------------------------------------------------------------------
# maps
# ---------------------------------------------------------------------------

def occ_exact_count(rng: np.random.Generator, W: int, H: int,
                    frac: float) -> np.ndarray:
    """Exactly round(frac * W * H) blocked cells chosen by a seeded permutation."""
    S = W * H
    nb = int(round(frac * S))
    occ = np.zeros(S, dtype=np.uint8)
    occ[rng.permutation(S)[:nb]] = 1
    return occ


def occ_rectangles(rng: np.random.Generator, W: int, H: int, frac: float,
                   side_lo: int, side_hi: int,
                   walls: Optional[tuple] = None) -> np.ndarray:
    """Axis-aligned rectangles with sides U{side_lo..side_hi} at uniform
    positions until the blocked fraction reaches ``frac``.  With ``walls =
    (len_lo, len_hi)`` rectangles alternate with one-cell-thick horizontal or
    vertical wall segments of length U{len_lo..len_hi}."""
    g = np.zeros((H, W), dtype=np.uint8)
    target = frac * W * H
    i = 0
    while g.sum() < target:
        if walls is not None and i % 2 == 1:
            ln = int(rng.integers(walls[0], walls[1] + 1))
            if rng.random() < 0.5:
                y = int(rng.integers(0, H))
                x = int(rng.integers(0, W))
                g[y, x:x + ln] = 1
            else:
                y = int(rng.integers(0, H))
                x = int(rng.integers(0, W))
                g[y:y + ln, x] = 1
        else:
            h = int(rng.integers(side_lo, side_hi + 1))
            w = int(rng.integers(side_lo, side_hi + 1))
            y = int(rng.integers(0, H - h + 1))
            x = int(rng.integers(0, W - w + 1))
            g[y:y + h, x:x + w] = 1
        i += 1
    return g.reshape(-1)


def largest_free_component(occ: np.ndarray, W: int, H: int) -> np.ndarray:
    """Cells of the largest 8-connected component of free cells."""
    from scipy import ndimage
    free = (occ.reshape(H, W) == 0)
    lab, nlab = ndimage.label(free, structure=np.ones((3, 3), dtype=int))
    if nlab == 0:
        raise ValueError("map has no free cell")
    sizes = np.bincount(lab.reshape(-1))
    sizes[0] = 0
    best = int(np.argmax(sizes))
    return np.flatnonzero(lab.reshape(-1) == best)


# ---------------------------------------------------------------------------
# reward table
# ---------------------------------------------------------------------------

def reward_step_goal(occ: np.ndarray, W: int, H: int, slip: np.ndarray,
                     goal: int, step: float = -1.0,
                     bonus: float = 100.0) -> np.ndarray:
    """R(s, a) = step + bonus * (probability that action a enters the goal
    from s) for a free non-goal cell s; 0 on blocked cells and at the goal.

    Only moves whose target is the goal cell itself contribute, and the goal
    is free, so the probability of entering it is the slip mass aimed at it.
    """
    S = W * H
    A = slip.shape[0]
    R = np.zeros((S, A), dtype=np.float64)
    gy, gx = (goal // W, goal % W) if goal >= 0 else (-10, -10)
    for s in range(S):
        if occ[s] or s == goal:
            continue
        y, x = divmod(s, W)
        for a in range(A):
            hit = 0.0
            for k, (dy, dx) in enumerate(NEIGHBOURS):
                if k != 4 and y + dy == gy and x + dx == gx:
                    hit += float(slip[a, k])
            R[s, a] = step + bonus * hit
    return R.astype(np.float32)


def reward_paper(occ: np.ndarray, W: int, H: int, slip: np.ndarray, target: int,
                 stop_action: int = 4) -> np.ndarray:
    """The stage reward of Sec. V: with r(y) = -2 on a blocked cell (off the
    grid counts as blocked), 0 at the target, -1 on any other free cell,
    R(x, a) = -2 for the stay action away from the target, and otherwise
    sum_y r(y) T'(x, a, y), with the free-space T' (so an action aimed at an
    obstacle pays for it).  Blocked x (never occupied): 0."""
    S = W * H
    A = slip.shape[0]
    R = np.zeros((S, A), dtype=np.float64)
    for s in range(S):
        if occ[s]:
            continue
        y, x = divmod(s, W)
        for a in range(A):
            if a == stop_action and s != target:
                R[s, a] = -2.0
                continue
            v = 0.0
            for k, (dy, dx) in enumerate(NEIGHBOURS):
                p = float(slip[a, k])
                if p == 0.0:
                    continue
                ny, nx = y + dy, x + dx
                t = ny * W + nx
                if not (0 <= ny < H and 0 <= nx < W) or occ[t]:
                    r = -2.0
                elif t == target:
                    r = 0.0
                else:
                    r = -1.0
                v += p * r
            R[s, a] = v
    return R.astype(np.float32)


# ---------------------------------------------------------------------------
# start beliefs
# ---------------------------------------------------------------------------

def _normalise32(w: np.ndarray) -> np.ndarray:
    w = np.asarray(w, dtype=np.float64)
    return (w / w.sum()).astype(np.float32)


def belief_uniform_cells(S: int, cells) -> np.ndarray:
    w = np.zeros(S, dtype=np.float64)
    w[np.asarray(cells)] = 1.0
    return _normalise32(w)


def belief_gaussian(occ: np.ndarray, W: int, H: int, centre: int,
                    sigma: float) -> np.ndarray:
    """b0(s) proportional to exp(-|s - c|^2 / (2 sigma^2)) on free cells."""
    ys, xs = np.divmod(np.arange(W * H), W)
    cy, cx = divmod(centre, W)
    w = np.exp(-((ys - cy) ** 2 + (xs - cx) ** 2) / (2.0 * sigma * sigma))
    w[occ != 0] = 0.0
    return _normalise32(w)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def _rng(k: int, seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_BASE + k, seed]))


def make_small(seed: int = 0, W: int = 10, H: int = 10, frac: float = 0.15,
               D: int = 2, n: int = 2, flip: float = 0.1,
               gamma: float = 0.95, n_start: int = 5,
               query_id: int = 0, cfg_index: int = 0) -> Problem:
    """Plain-method workload, small enough for the FP64 oracle: a W x H grid
    with exactly round(frac*W*H) seeded blocked cells, N/E/S/W actions (0.8
    intended, 0.1 on each perpendicular), four wall bits each flipped with
    probability ``flip``, reward -1 per step and +100 on entering the goal,
    discount 0.95, start belief uniform over ``n_start`` seeded free cells."""
    rng = _rng(cfg_index, seed)
    occ = occ_exact_count(rng, W, H, frac)
    free = np.flatnonzero(occ == 0)
    perm = rng.permutation(free)
    goal = int(perm[0])
    starts = perm[1:1 + n_start]
    slip = slip_table_4()
    R = reward_step_goal(occ, W, H, slip, goal)
    b0 = belief_uniform_cells(W * H, starts)
    return Problem(name=f"grid{W}x{H}-4act-D{D}n{n}", W=W, H=H, occ=occ,
                   slip=slip, flip=np.full(4, flip, dtype=np.float32),
                   lm_cell=np.zeros(0, dtype=np.int32), lm_p=0.9, R=R,
                   goal=goal, gamma=gamma, b0=b0, D=D, n=n,
                   seed=int(rng.integers(0, 2 ** 63)), query_id=query_id)


def make_rect(seed: int = 0, side: int = 64, frac: float = 0.20,
              side_lo: int = 2, side_hi: int = 8, n_landmarks: int = 32,
              D: int = 3, n: int = 4, sigma: float = 5.0,
              walls: Optional[tuple] = None, patches: int = 0,
              cfg_index: int = 1) -> Problem:
    """Plain-method GPU workload: a side x side grid of seeded random
    rectangles (optionally alternating with wall segments), 8 actions with
    8-neighbour slip (0.7 intended, 0.1 on each adjacent direction, 0.1
    stay), wall bits flipped with probability 0.1 plus ``n_landmarks``
    landmark cells that report their id with probability 0.9.  The start
    belief is a Gaussian blob (``sigma`` cells) or, with ``patches > 0``, an
    equal mixture of that many disjoint 20 x 20 patches."""
    rng = _rng(cfg_index, seed)
    W = H = side
    occ = occ_rectangles(rng, W, H, frac, side_lo, side_hi, walls)
    comp = largest_free_component(occ, W, H)
    comp_perm = rng.permutation(comp)
    goal = int(comp_perm[0])
    free = np.flatnonzero(occ == 0)
    free_ng = free[free != goal]
    lm = rng.permutation(free_ng)[:n_landmarks].astype(np.int32)
    slip = slip_table_8()
    R = reward_step_goal(occ, W, H, slip, goal)
    if patches:
        b0 = _patch_mixture(rng, occ, W, H, patches, 20)
    else:
        centre = int(comp_perm[1])
        b0 = belief_gaussian(occ, W, H, centre, sigma)
    return Problem(name=f"rect{W}x{H}-8act-L{n_landmarks}-D{D}n{n}", W=W,
                   H=H, occ=occ, slip=slip,
                   flip=np.full(4, 0.1, dtype=np.float32), lm_cell=lm,
                   lm_p=0.9, R=R, goal=goal, gamma=0.95, b0=b0, D=D, n=n,
                   seed=int(rng.integers(0, 2 ** 63)))


def _patch_mixture(rng, occ, W, H, npatch, size):
    """Equal mixture of ``npatch`` disjoint size x size patches, each uniform
    over its free cells (patches with no free cell are redrawn)."""
    w = np.zeros(W * H, dtype=np.float64)
    taken = np.zeros((H, W), dtype=bool)
    got = 0
    while got < npatch:
        y = int(rng.integers(0, H - size + 1))
        x = int(rng.integers(0, W - size + 1))
        if taken[y:y + size, x:x + size].any():
            continue
        cells = (np.arange(y, y + size)[:, None] * W
                 + np.arange(x, x + size)[None, :]).reshape(-1)
        fc = cells[occ[cells] == 0]
        if fc.size == 0:
            continue
        taken[y:y + size, x:x + size] = True
        w[fc] += 1.0 / (npatch * fc.size)
        got += 1
    return _normalise32(w)


def make_large(seed: int = 0) -> Problem:
    """Large plain-method workload: 512 x 512 rectangles (sides 4..32) and
    corridor walls (length 32..256), 25% blocked, 8 actions, wall bits plus
    256 landmarks, depth 3, 3 samples per action, start belief a mixture of
    four disjoint 20 x 20 patches."""
    return make_rect(seed=seed, side=512, frac=0.25, side_lo=4, side_hi=32,
                     n_landmarks=256, D=3, n=3, walls=(32, 256), patches=4,
                     cfg_index=4)


def make_batch(seed: int = 0, nq: int = 256, side_lo: int = 32,
               side_hi: int = 256, n: int = 3) -> List[Problem]:
    """Batched workload: ``nq`` independent small-method queries with square
    sides U{side_lo..side_hi}, blocked fraction U[0.1, 0.3], depth U{2, 3},
    ``n`` samples per action, N/E/S/W actions and the wall-bit sensor."""
    rng = _rng(2, seed)
    out = []
    for q in range(nq):
        side = int(rng.integers(side_lo, side_hi + 1))
        frac = float(rng.uniform(0.1, 0.3))
        D = int(rng.integers(2, 4))
        p = make_small(seed=int(rng.integers(0, 2 ** 31)), W=side, H=side,
                       frac=frac, D=D, n=n, query_id=q, cfg_index=2)
        p.name = f"batch-q{q}-{side}x{side}-D{D}n{n}"
        out.append(p)
    return out


def make_paper(seed: int = 0, W: int = 100, H: int = 40, frac: float = 0.15,
               side_lo: int = 2, side_hi: int = 6, walls: Optional[tuple] = (8, 30),
               D: int = 2, n: int = 3, cfg_index: int = 5) -> Problem:
    """The experiment model of Sec. V on a synthetic map: a W x H grid of
    seeded rectangles and wall segments, the nine actions of slip_table_9,
    four wall bits each read correctly with probability 0.95, no landmarks,
    the stage reward of reward_paper towards a seeded target cell in the
    largest free component, discount 0.95, and the start belief uniform over
    the free cells.  The target is not absorbing (the paper's model has no
    absorbing state): ``goal`` is -1 and the target is ``meta["target"]``;
    the stay action (``meta["stop_action"]`` = 4) ends a closed-loop run."""
    rng = _rng(cfg_index, seed)
    occ = occ_rectangles(rng, W, H, frac, side_lo, side_hi, walls)
    comp = largest_free_component(occ, W, H)
    target = int(rng.permutation(comp)[0])
    slip = slip_table_9()
    R = reward_paper(occ, W, H, slip, target)
    b0 = belief_uniform_cells(W * H, np.flatnonzero(occ == 0))
    return Problem(name=f"paper{W}x{H}-9act-D{D}n{n}", W=W, H=H, occ=occ, slip=slip,
                   flip=np.full(4, 0.05, dtype=np.float32),
                   lm_cell=np.zeros(0, dtype=np.int32), lm_p=0.9, R=R, goal=-1,
                   gamma=0.95, b0=b0, D=D, n=n, seed=int(rng.integers(0, 2 ** 63)),
                   meta={"target": target, "stop_action": 4, "component": comp})


class Environment:
    """The true world of one closed-loop run (the generative model of Sec. V):
    the robot's cell, moved by a seeded draw of the slip outcome of each
    executed action, and the observation of each new cell, drawn with the
    sensor's flip probabilities (and landmark channel).  The start cell is
    drawn uniformly from the target's free component (other than the target).
    It holds the world's random numbers only; no step of the planning method."""

    def __init__(self, prob: Problem, seed: int, start: Optional[int] = None):
        self.prob = prob
        self.rng = _rng(6, seed)
        comp = prob.meta.get("component")
        if comp is None:
            comp = np.flatnonzero(prob.occ == 0)
        target = prob.meta.get("target", -1)
        cand = np.asarray(comp)[np.asarray(comp) != target]
        self.s = int(start) if start is not None else int(cand[self.rng.integers(0, cand.size)])
        self.cum = np.cumsum(prob.slip.astype(np.float64), axis=1)
        self.lm_id = None
        if prob.L > 0:
            self.lm_id = np.zeros(prob.S, dtype=np.int32)
            self.lm_id[prob.lm_cell] = np.arange(1, prob.L + 1)

    def step(self, a: int):
        """Executes action a: returns (observation z, collided), where
        collided means the drawn move aimed at a blocked or off-grid cell."""
        p = self.prob
        self.s, z, hit = _env_step(self.rng, p.occ, p.W, p.H, self.cum, p.flip, self.s, int(a),
                                   self.lm_id, p.lm_p)
        return z, hit


# ---------------------------------------------------------------------------
# logged trajectories for the differentiable filter
# ---------------------------------------------------------------------------

@dataclass
class TrajectorySet:
    problem: Problem                # map, sensor layout, b0 (no goal)
    theta_true: np.ndarray          # float32 [A, 9] slip logits
    phi_true: np.ndarray            # float32 [4] flip logits
    theta: np.ndarray               # float32 [A, 9] evaluation point
    phi: np.ndarray                 # float32 [4] evaluation point
    acts: np.ndarray                # int32 [ntraj, T]
    obs: np.ndarray                 # int32 [ntraj, T]


def _env_step(rng, occ, W, H, cum, flip, s, a, lm_id=None, lm_p=0.0):
    """One step of the generative model of Sec. V from cell s under action a:
    the slip outcome k ~ slip[a] (cum: its running totals), the move
    succeeds when its target is inside the grid and free, each wall bit is
    read correctly with probability 1 - flip[j]; on a cell with landmark id
    l > 0 the landmark channel reports l with probability lm_p, else 0.
    Returns (new cell, z = zw + 16 zl, whether the move hit an obstacle)."""
    k = int(np.searchsorted(cum[a], rng.random() * cum[a, -1], side="right"))
    k = min(k, 8)
    dy, dx = NEIGHBOURS[k]
    y, x = divmod(s, W)
    ny, nx = y + dy, x + dx
    hit = False
    if 0 <= ny < H and 0 <= nx < W and occ[ny * W + nx] == 0:
        s = ny * W + nx
    elif k != 4:
        hit = True
    y, x = divmod(s, W)
    zw = 0
    for j, (ddy, ddx) in enumerate(((-1, 0), (0, -1), (0, 1), (1, 0))):
        qy, qx = y + ddy, x + ddx
        bit = 1 if not (0 <= qy < H and 0 <= qx < W) or occ[qy * W + qx] else 0
        if rng.random() < flip[j]:
            bit ^= 1
        zw |= bit << j
    zl = 0
    if lm_id is not None and lm_id[s] > 0 and rng.random() < lm_p:
        zl = int(lm_id[s])
    return s, zw + 16 * zl, hit


def _simulate(rng, occ, W, H, slip, flip, s0, acts, lm_id=None, lm_p=0.0):
    """A state path and its observations under the generative model of
    Sec. V (see _env_step) for the action sequence acts."""
    T = acts.shape[0]
    obs = np.zeros(T, dtype=np.int32)
    s = s0
    cum = np.cumsum(slip.astype(np.float64), axis=1)
    for t in range(T):
        s, obs[t], _ = _env_step(rng, occ, W, H, cum, flip, s, int(acts[t]), lm_id, lm_p)
    return obs


def _softmax_rows(x):
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(x - x.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def make_trajectories(seed: int = 0, side: int = 128, frac: float = 0.15,
                      ntraj: int = 1024, T: int = 50,
                      cfg_index: int = 3, n_landmarks: int = 0,
                      lm_p: float = 0.9) -> TrajectorySet:
    """Logged runs for filter calibration: a side x side grid with exactly
    round(frac*S) blocked cells, 8 actions with 9-outcome slip given by true
    logits log(p + 0.01) + N(0, 0.1^2) around the 8-neighbour slip table p,
    true flip probabilities U[0.05, 0.2] per wall bit, actions uniform, start
    state drawn from the uniform belief over free cells.  The evaluation
    point is the truth plus N(0, 0.5^2) noise on every logit.  With
    n_landmarks > 0, that many distinct free cells carry landmarks with
    ids 1..n_landmarks, seen with probability lm_p."""
    rng = _rng(cfg_index, seed)
    W = H = side
    occ = occ_exact_count(rng, W, H, frac)
    free = np.flatnonzero(occ == 0)
    p2 = slip_table_8().astype(np.float64)
    theta_true = np.log(p2 + 0.01) + rng.normal(0.0, 0.1, size=p2.shape)
    f_true = rng.uniform(0.05, 0.2, size=4)
    phi_true = np.log(f_true / (1.0 - f_true))
    slip_true = _softmax_rows(theta_true)
    acts = rng.integers(0, 8, size=(ntraj, T)).astype(np.int32)
    lm_cell = np.zeros(0, dtype=np.int32)
    lm_id = None
    if n_landmarks > 0:
        lm_cell = np.sort(rng.choice(free, size=n_landmarks, replace=False)).astype(np.int32)
        lm_id = np.zeros(W * H, dtype=np.int32)
        lm_id[lm_cell] = np.arange(1, n_landmarks + 1)
    obs = np.zeros((ntraj, T), dtype=np.int32)
    for i in range(ntraj):
        s0 = int(free[rng.integers(0, free.size)])
        obs[i] = _simulate(rng, occ, W, H, slip_true, f_true, s0, acts[i], lm_id, lm_p)
    theta = theta_true + rng.normal(0.0, 0.5, size=theta_true.shape)
    phi = phi_true + rng.normal(0.0, 0.5, size=4)
    b0 = belief_uniform_cells(W * H, free)
    prob = Problem(name=f"filter{W}x{H}-8act-{ntraj}x{T}", W=W, H=H,
                   occ=occ, slip=slip_true.astype(np.float32),
                   flip=f_true.astype(np.float32),
                   lm_cell=lm_cell, lm_p=lm_p,
                   R=np.zeros((W * H, 8), dtype=np.float32), goal=-1,
                   gamma=0.95, b0=b0)
    return TrajectorySet(problem=prob,
                         theta_true=theta_true.astype(np.float32),
                         phi_true=phi_true.astype(np.float32),
                         theta=theta.astype(np.float32),
                         phi=phi.astype(np.float32), acts=acts, obs=obs)
