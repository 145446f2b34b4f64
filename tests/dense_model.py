"""Dense-matrix form of the POMDP of Sec. II/V, for brute-force checks.

Written independently of the oracle (it never calls it): the transition
matrices T[a] (|X| x |X|) and the observation matrix O (|X| x |Z|) are
assembled entry by entry from the model definitions, and every brute-force
check below (Bellman recursion, HMM path sums, linear policy evaluation)
works on these matrices with numpy.
"""
import itertools

import numpy as np


def transition_matrices(prob):
    """T[a][x, y]: the slip outcome aimed at an occupied or off-grid cell
    keeps the robot at x (Sec. V); blocked cells and the goal map to
    themselves."""
    W, H, A = prob.W, prob.H, prob.A
    S = W * H
    occ = np.asarray(prob.occ).reshape(H, W)
    slip = np.asarray(prob.slip, dtype=np.float64)
    T = np.zeros((A, S, S))
    for a in range(A):
        for y in range(H):
            for x in range(W):
                i = y * W + x
                if occ[y, x] or i == prob.goal:
                    T[a, i, i] = 1.0
                    continue
                for dy, dx in itertools.product((-1, 0, 1), (-1, 0, 1)):
                    k = (dy + 1) * 3 + (dx + 1)
                    yy, xx = y + dy, x + dx
                    inside = 0 <= yy < H and 0 <= xx < W
                    if inside and not occ[yy, xx]:
                        T[a, i, yy * W + xx] += slip[a, k]
                    else:
                        T[a, i, i] += slip[a, k]
    return T


def wall_pattern(prob):
    """4-bit true wall reading per cell: bit 0 up, 1 left, 2 right, 3 down;
    1 = occupied or outside the map."""
    W, H = prob.W, prob.H
    occ = np.asarray(prob.occ).reshape(H, W)
    w = np.zeros(W * H, dtype=np.int64)
    for y in range(H):
        for x in range(W):
            bits = 0
            for j, (dy, dx) in enumerate(((-1, 0), (0, -1), (0, 1), (1, 0))):
                yy, xx = y + dy, x + dx
                if not (0 <= yy < H and 0 <= xx < W) or occ[yy, xx]:
                    bits |= 1 << j
            w[y * W + x] = bits
    return w


def observation_matrix(prob, flip=None):
    """O[s, z] = P(z | s) for z = zw + 16 zl."""
    S = prob.W * prob.H
    L = len(prob.lm_cell)
    Z = 16 * (L + 1)
    flip = np.asarray(prob.flip if flip is None else flip, dtype=np.float64)
    rho = float(np.float32(prob.lm_p))
    w = wall_pattern(prob)
    lm = np.zeros(S, dtype=np.int64)
    for l, c in enumerate(prob.lm_cell):
        lm[c] = l + 1
    O = np.zeros((S, Z))
    for s in range(S):
        for zw in range(16):
            pw = 1.0
            for j in range(4):
                same = ((zw >> j) & 1) == ((w[s] >> j) & 1)
                pw *= (1.0 - flip[j]) if same else flip[j]
            if lm[s] == 0:
                O[s, zw] = pw
            else:
                O[s, zw] = pw * (1.0 - rho)
                O[s, zw + 16 * lm[s]] = pw * rho
    return O


def bellman_full(T, O, R, Q, gamma, b, depth):
    """Depth-limited POMDP Bellman recursion (Sec. III) with every
    observation expanded and max_a b.Q at the leaves.  Returns per-action
    values at b."""
    A = T.shape[0]
    if depth == 0:
        return b @ Q
    out = np.zeros(A)
    for a in range(A):
        bp = b @ T[a]
        pz = bp @ O
        val = b @ R[:, a]
        for z in np.flatnonzero(pz > 0):
            post = O[:, z] * bp / pz[z]
            val += gamma * pz[z] / pz.sum() * np.max(bellman_full(T, O, R, Q, gamma, post, depth - 1))
        out[a] = val
    return out
