"""Pins of the grid-search oracle (Section 6.2.1, eqs. 4-9) to geometry.

The four grids shifted by d put cell centres on every multiple of d, so the
centre-most cell of a point is the 2d x 2d cell centred at the nearest such
lattice point: an independent description of the selection used below as a
brute force.  From it follow two containment facts that catch a wrong centre
formula or shift: every candidate lies within 2d (per axis) of some sample
point, and every feature within d/2 (per axis) of a sample point is one."""
import math

import numpy as np

from oracle.grid import grid_candidates, line_points, two_nearest


def _F_line(a, b, c):
    """An F whose line for the query (0, 0) is (a, b, c)."""
    F = np.zeros((3, 3))
    F[:, 2] = (a, b, c)
    return F


def test_samples_of_a_horizontal_line():
    px, py = line_points(_F_line(0.0, 1.0, -300.0), 0.0, 0.0, (0.0, 0.0, 1000.0, 750.0), 4.0)
    assert px.size == 251                       # K = 1000 / 4, points k = 0..K
    assert np.all(py == 300.0)
    assert np.allclose(np.sort(px), np.arange(251) * 4.0)
    # A is the crossing found first (x = x0), so p_K = A and p_0 = B.
    assert px[-1] == 0.0 and px[0] == 1000.0


def test_samples_round_k_up_and_corner_touch():
    px, _ = line_points(_F_line(0.0, 1.0, -10.0), 0.0, 0.0, (0.0, 0.0, 10.0, 20.0), 3.0)
    assert px.size == 5                         # |AB| = 10, K = ceil(10 / 3) = 4
    assert np.max(np.abs(np.diff(px))) <= 3.0
    # x + y = 0 touches the box (0, 0, 5, 5) only at its corner: one point.
    px, py = line_points(_F_line(1.0, 1.0, 0.0), 0.0, 0.0, (0.0, 0.0, 5.0, 5.0), 1.0)
    assert px.size == 1 and px[0] == 0.0 and py[0] == 0.0
    # A line that misses the box has no points.
    px, _ = line_points(_F_line(1.0, 1.0, 100.0), 0.0, 0.0, (0.0, 0.0, 5.0, 5.0), 1.0)
    assert px.size == 0


def _lattice_candidates(xy, px, py, d):
    """Brute force: centre = nearest multiple of d per axis, cell = [c-d, c+d)."""
    member = np.zeros(xy.shape[0], bool)
    for x, y in zip(px, py):
        cx, cy = math.floor(x / d + 0.5) * d, math.floor(y / d + 0.5) * d
        member |= ((xy[:, 0] >= cx - d) & (xy[:, 0] < cx + d) &
                   (xy[:, 1] >= cy - d) & (xy[:, 1] < cy + d))
    return np.nonzero(member)[0]


def test_candidates_equal_lattice_brute_force_and_containment():
    rng = np.random.default_rng(0)
    for trial in range(12):
        n = 3000
        xy = np.column_stack([rng.uniform(0, 640, n), rng.uniform(0, 480, n)]).astype(np.float32)
        d = float(rng.choice([2.0, 3.5, 6.0]))
        F = rng.normal(size=(3, 3))
        xa, ya = float(rng.uniform(0, 640)), float(rng.uniform(0, 480))
        got = grid_candidates(xy, F, xa, ya, d)
        box = (float(xy[:, 0].min()), float(xy[:, 1].min()),
               float(xy[:, 0].max()), float(xy[:, 1].max()))
        px, py = line_points(F, xa, ya, box, d)
        assert np.array_equal(got, _lattice_candidates(xy.astype(np.float64), px, py, d))
        if px.size == 0:
            continue
        # Containment: within 2d of a sample (per axis) ...
        cheb = np.min(np.maximum(np.abs(xy[got, 0:1] - px[None, :]),
                                 np.abs(xy[got, 1:2] - py[None, :])), axis=1)
        assert np.all(cheb <= 2 * d)
        # ... and everything within d/2 of a sample is a candidate.
        near = np.min(np.maximum(np.abs(xy[:, 0:1] - px[None, :]),
                                 np.abs(xy[:, 1:2] - py[None, :])), axis=1) <= d / 2
        assert set(np.nonzero(near)[0]) <= set(got.tolist())


def test_two_nearest_rules():
    rng = np.random.default_rng(1)
    b = rng.integers(0, 128, size=(6, 128), dtype=np.uint8)
    q = b[4].copy()
    b[2] = q                                    # exact duplicate at a lower index
    m, d1, d2, n, acc = two_nearest(q, b, np.array([1, 2, 4]))
    assert (m, d1, d2, n, acc) == (2, 0, 0, 3, False)   # tie: lower index, D2 = D1, rejected
    m, d1, d2, n, acc = two_nearest(q, b, np.array([0, 4, 5]))
    assert m == 4 and d1 == 0 and d2 > 0 and acc
    assert two_nearest(q, b, np.array([], np.int64))[:4] == (-1, 2**31 - 1, 2**31 - 1, 0)
    assert two_nearest(q, b, np.array([3]))[4] is False
    assert two_nearest(q, b, np.array([3]), accept_single=True)[4] is True


def test_query_groups_by_hand():
    """Horizontal lines y = y_a (F maps (x, y, 1) to (0, 1, -y)) cross the box
    x in [0, 100] at A = (0, y), B = (100, y).  Sorted by y, a new group starts
    where y jumps by more than 2 px from the previous line: the chain 10, 11.5,
    13 stays one group although its ends are 3 px apart."""
    from oracle.grid import query_groups
    F = np.zeros((3, 3))
    F[1, 2] = 1.0
    F[2, 1] = -1.0
    ys = np.array([20.0, 10.0, 13.0, 21.0, 11.5, 40.0, 500.0, 10.0], np.float32)
    xy_a = np.column_stack([np.zeros_like(ys), ys]).astype(np.float32)
    xy_b = np.array([[0.0, 0.0], [100.0, 100.0]], np.float32)
    order, starts = query_groups(xy_a, xy_b, F)
    # y = 500 misses the box [0, 100]^2: last, a group of its own.
    assert order.tolist() == [1, 7, 4, 2, 0, 3, 5, 6]
    assert starts.tolist() == [0, 4, 6, 7]
    order0, starts0 = query_groups(xy_a, xy_b, F, tol_px=0.0)
    assert starts0.tolist() == [0, 2, 3, 4, 5, 6, 7]          # only the duplicate y = 10 shares
    # Against the group's first line instead: 13 is 3 px from 10, a new group.
    _, starts1 = query_groups(xy_a, xy_b, F, to_leader=True)
    assert starts1.tolist() == [0, 3, 4, 6, 7]


def test_grouped_queries_share_the_leaders_candidates():
    from oracle.grid import grid_match, query_groups
    rng = np.random.default_rng(5)
    n = 600
    xy = np.column_stack([rng.uniform(0, 300, n), rng.uniform(0, 200, n)]).astype(np.float32)
    desc = rng.integers(0, 128, size=(n, 128), dtype=np.uint8)
    # A pencil through a point far to the left: nearby queries give nearby lines.
    F = np.array([[0.0, -1.0, 100.0], [1.0, 0.0, 1500.0], [-100.0, -1500.0, 0.0]])
    imgs = [(xy, desc), (xy, desc)]
    plain = grid_match(imgs, [(0, 1, 3.0)], [F])[0]
    grouped = grid_match(imgs, [(0, 1, 3.0)], [F], group_px=2.0)[0]
    order, starts = query_groups(xy, xy, F)
    ends = np.append(starts[1:], n)
    assert len(starts) < n                                  # some groups hold several queries
    for s0, s1 in zip(starts, ends):
        lead = order[s0]
        assert grouped["count"][lead] == plain["count"][lead]
        assert np.all(grouped["count"][order[s0:s1]] == plain["count"][lead])
