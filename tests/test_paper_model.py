"""The experiment model of Sec. V (CPU): the nine-action slip table, the
stage reward r/R worked by hand on a 3 x 3 map, and the world simulator of
closed-loop runs checked against the slip table and the sensor by counting."""
import numpy as np
import pytest

from paper_1810_00204_amd import workloads as wl


def test_nine_action_slip_table():
    t = wl.slip_table_9().astype(np.float64)
    assert t.shape == (9, 9)
    np.testing.assert_allclose(t.sum(1), 1.0, atol=1e-7)
    assert t[4, 4] == 1.0 and t[4].sum() == 1.0          # stay is deterministic
    # "up" (a = 1, neighbour N_1): 0.8 on N_1, 0.05 on N_0 and N_2, 0.1 stay
    np.testing.assert_allclose(t[1], [0.05, 0.8, 0.05, 0, 0.1, 0, 0, 0, 0], atol=1e-7)
    # "down-right" (a = 8): ring neighbours are right (5) and down (7)
    np.testing.assert_allclose(t[8], [0, 0, 0, 0, 0.1, 0.05, 0, 0.05, 0.8], atol=1e-7)
    for a in range(9):
        if a != 4:
            assert t[a, a] == pytest.approx(0.8)


def test_paper_reward_by_hand():
    """3 x 3 map, row 0 = '. . #', row 1 = '. x .', row 2 = '. G .'; the
    target G is cell 7, x is cell 4.  r = -2 blocked or off-grid, 0 at G, -1
    elsewhere; R(x, a) = sum_y r(y) T'(x, a, y), R(x, stay) = -2 off target."""
    W = H = 3
    occ = np.zeros(9, np.uint8)
    occ[2] = 1
    slip = wl.slip_table_9()
    R = wl.reward_paper(occ, W, H, slip, target=7).astype(np.float64)
    # up from the centre: 0.8 r(1) + 0.05 r(0) + 0.05 r(2) + 0.1 r(4)
    assert R[4, 1] == pytest.approx(0.8 * -1 + 0.05 * -1 + 0.05 * -2 + 0.1 * -1)   # -1.05
    # down from the centre: 0.8 r(7) = 0, 0.05 r(6) + 0.05 r(8) + 0.1 r(4)
    assert R[4, 7] == pytest.approx(0.05 * -1 + 0.05 * -1 + 0.1 * -1)             # -0.2
    assert R[4, 4] == -2.0                  # stay away from the target
    assert R[7, 4] == 0.0                   # stay at the target
    # up-left from the corner cell 0: target and both ring neighbours off grid
    assert R[0, 0] == pytest.approx(0.8 * -2 + 0.05 * -2 + 0.05 * -2 + 0.1 * -1)   # -1.9
    # right from cell 1 aims at the blocked cell 2
    assert R[1, 5] == pytest.approx(0.8 * -2 + 0.05 * -2 + 0.05 * -1 + 0.1 * -1)   # -1.85
    assert np.all(R[2] == 0.0)              # blocked cell


def test_paper_workload_shape():
    p = wl.make_paper(seed=0)
    assert (p.W, p.H, p.A, p.L) == (100, 40, 9, 0)
    assert p.goal == -1 and p.occ[p.meta["target"]] == 0
    np.testing.assert_allclose(p.flip, 0.05)
    assert abs(float(p.b0.astype(np.float64).sum()) - 1) < 1e-6
    assert np.all(p.b0[p.occ == 1] == 0) and np.all(p.b0[p.occ == 0] > 0)
    assert p.R.max() == 0.0 and p.R.min() >= -2.0


def test_environment_follows_the_slip_table_and_sensor():
    """From a cell with all nine neighbours free and no wall in sight, the
    landing frequencies of 20000 steps match T'(a, .) within 4 sigma, and
    each wall bit reads 1 (a misread of a free neighbour) about 5% of the
    time; into a wall, the move counts as a collision and the robot stays."""
    W, H = 7, 7
    occ = np.zeros(W * H, np.uint8)
    prob = wl.make_paper(seed=1, W=W, H=H, frac=0.0, walls=None)
    prob.occ = occ
    centre = 3 * W + 3
    N = 20000
    for a in (1, 6):
        env = wl.Environment(prob, seed=10 + a, start=centre)
        counts = np.zeros(9)
        bits = np.zeros(4)
        for _ in range(N):
            env.s = centre
            z, hit = env.step(a)
            assert not hit
            dy, dx = divmod(env.s - centre + 3 * W + 3, W)
            k = (dy - 2) * 3 + (dx - 2)
            counts[k] += 1
            bits += [(z >> j) & 1 for j in range(4)]
        p = prob.slip[a].astype(np.float64)
        sig = np.sqrt(N * p * (1 - p)) + 1e-9
        assert np.all(np.abs(counts - N * p) <= 4 * sig + 1e-9), (a, counts, N * p)
        fp = 0.05
        assert np.all(np.abs(bits - N * fp) <= 4 * np.sqrt(N * fp * (1 - fp)))
    # a robot against the top wall moving up: collisions whenever the drawn
    # move aims off the grid (up, up-left, up-right: 0.9 of the time)
    env = wl.Environment(prob, seed=3, start=3)
    hits = 0
    for _ in range(4000):
        env.s = 3
        _, hit = env.step(1)
        hits += hit
        assert env.s in (3, 2, 4) or not hit
    assert abs(hits / 4000 - 0.9) < 4 * np.sqrt(0.09 / 4000)
