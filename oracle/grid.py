"""Grid-based approximate candidate search -- TEST INFRASTRUCTURE.

Only tests/ and the benchmark's CPU-baseline leg may use this module.  It
restates the grid search of Section 6.2.1 (eqs. 4-9, Fig. 4c) and the match
of Section 6.2.2 on its candidates, and shares no code with the GPU library.

Steps, for a query x_a of image a with line l = F (x_a, 1) = (a, b, c) in
image b (every product and sum in IEEE double, left to right, no fused
multiply-add, so another implementation can reproduce each decision):

* the "image" of b is the bounding box of b's keypoints (the library takes
  no image size); the line's end points A, B are its crossings with the box,
  found on the edges x = x0, x = x1, y = y0, y = y1 in that order (inclusive
  ranges); A is the first crossing, B the crossing farthest from A (the first
  of equal ones); no crossing, no candidates;
* K is the smallest integer >= 0 with K^2 d^2 >= |AB|^2 (eq. 5 prints
  K = |AB| / d, which need not be an integer), and the K + 1 points of
  eqs. (4)-(5) are p_k = (k A + (K - k) B) / K, k = 0..K (p_0 = A when K = 0);
* grid g = 0..3 has cells of 2d x 2d shifted by (s_x, s_y) = (0,0), (d,0),
  (0,d), (d,d): the cell of (x, y) is (floor((x - s_x) / 2d),
  floor((y - s_y) / 2d)) and its centre cx * 2d + s_x + d (eqs. 6-9 as
  printed put the centre at floor(x / 2d) d + 2d, which is not a centre of a
  2d-wide cell; this is the reading of them);
* each point takes the centre-most of its four cells (squared distance to the
  centre; equal distances: the lower grid), and C' is the set of features of
  b that lie in any selected cell;
* the two nearest features of C' by exact squared L2 (lower index first among
  equal distances) and the ratio test, as in guided matching; fewer than two
  candidates: rejected (one candidate accepted with accept_single).

`d` is the cell parameter; the paper notes that a slightly larger grid than
the band makes up for the approximation, which is the caller's choice of d.
"""
from __future__ import annotations

import math

import numpy as np

SHIFTS = ((0, 0), (1, 0), (0, 1), (1, 1))   # in units of d


def crossings(F, xa: float, ya: float, box):
    """(A, B) of the line of (xa, ya) with the box, or None without a crossing."""
    F = [float(v) for v in np.asarray(F, dtype=np.float64).reshape(9)]
    a = F[0] * xa + F[1] * ya + F[2]
    b = F[3] * xa + F[4] * ya + F[5]
    c = F[6] * xa + F[7] * ya + F[8]
    x0, y0, x1, y1 = box
    hits = []
    for xe in (x0, x1):
        if b != 0.0:
            y = -(a * xe + c) / b
            if y0 <= y <= y1:
                hits.append((xe, y))
    for ye in (y0, y1):
        if a != 0.0:
            x = -(b * ye + c) / a
            if x0 <= x <= x1:
                hits.append((x, ye))
    if not hits:
        return None
    xA, yA = hits[0]
    xB, yB, best = xA, yA, -1.0
    for x, y in hits:
        dx, dy = x - xA, y - yA
        r = dx * dx + dy * dy
        if r > best:
            xB, yB, best = x, y, r
    return (xA, yA), (xB, yB)


def line_points(F, xa: float, ya: float, box, d: float):
    """The sample points of eqs. (4)-(5) on the line of (xa, ya), as two float
    arrays (empty without a crossing)."""
    ab = crossings(F, xa, ya, box)
    if ab is None:
        return np.zeros(0), np.zeros(0)
    (xA, yA), (xB, yB) = ab
    dx, dy = xB - xA, yB - yA
    len2 = dx * dx + dy * dy
    d2 = d * d
    K = int(math.ceil(math.sqrt(len2) / d))
    while K > 0 and float((K - 1) * (K - 1)) * d2 >= len2:
        K -= 1
    while float(K * K) * d2 < len2:
        K += 1
    if K == 0:
        return np.array([xA]), np.array([yA])
    k = np.arange(K + 1, dtype=np.float64)
    return (k * xA + (K - k) * xB) / K, (k * yA + (K - k) * yB) / K


def keypoint_box(xy_b):
    xy_b = np.asarray(xy_b, dtype=np.float32).reshape(-1, 2)
    return (float(xy_b[:, 0].min()), float(xy_b[:, 1].min()),
            float(xy_b[:, 0].max()), float(xy_b[:, 1].max()))


def grid_candidates(xy_b, F, xa: float, ya: float, d: float) -> np.ndarray:
    """C' of one query: ascending feature indices of b."""
    xy_b = np.asarray(xy_b, dtype=np.float32).reshape(-1, 2)
    if xy_b.shape[0] == 0:
        return np.zeros(0, np.int64)
    box = keypoint_box(xy_b)
    px, py = line_points(F, float(xa), float(ya), box, d)
    if px.size == 0:
        return np.zeros(0, np.int64)
    two_d = 2.0 * d
    xb = xy_b[:, 0].astype(np.float64)
    yb = xy_b[:, 1].astype(np.float64)
    # The centre-most cell of each sample point.
    best = np.full(px.size, np.inf)
    sel_g = np.zeros(px.size, np.int64)
    sel_c = np.zeros((px.size, 2), np.int64)
    for g, (sx, sy) in enumerate(SHIFTS):
        sx, sy = sx * d, sy * d
        cx = np.floor((px - sx) / two_d)
        cy = np.floor((py - sy) / two_d)
        ex = px - (cx * two_d + sx + d)
        ey = py - (cy * two_d + sy + d)
        r = ex * ex + ey * ey
        take = r < best
        best[take] = r[take]
        sel_g[take] = g
        sel_c[take, 0] = cx[take]
        sel_c[take, 1] = cy[take]
    member = np.zeros(xy_b.shape[0], bool)
    big = np.int64(1) << 32
    for g, (sx, sy) in enumerate(SHIFTS):
        cells = sel_c[sel_g == g]
        if cells.shape[0] == 0:
            continue
        sx, sy = sx * d, sy * d
        fx = np.floor((xb - sx) / two_d).astype(np.int64)
        fy = np.floor((yb - sy) / two_d).astype(np.int64)
        member |= np.isin(fx * big + fy, cells[:, 0] * big + cells[:, 1])
    return np.nonzero(member)[0]


def two_nearest(q_desc, b_desc, cand, ratio_num=64, ratio_den=100, accept_single=False):
    """(match, d1, d2, count, accept) over the candidate indices `cand`."""
    INF = 2**31 - 1
    n = len(cand)
    if n == 0:
        return -1, INF, INF, 0, False
    diff = b_desc[cand].astype(np.int64) - np.asarray(q_desc, dtype=np.int64)[None, :]
    D = np.sum(diff * diff, axis=1)
    order = np.lexsort((cand, D))
    j, d1 = int(cand[order[0]]), int(D[order[0]])
    if n == 1:
        return j, d1, INF, 1, bool(accept_single)
    d2 = int(D[order[1]])
    return j, d1, d2, n, ratio_den * d1 < ratio_num * d2


def query_groups(xy_a, xy_b, F, tol_px=2.0, to_leader=False):
    """The 2-px grouping of Section 6.2.2 (App. A step 2): the queries sorted by
    their line's crossings (A.x, A.y, B.x, B.y, then query index; lines without
    a crossing last), and a new group wherever a line's A or B lies more than
    tol_px from the previous line's (App. A's stencil), or with to_leader from
    the group's first line's (a line without a crossing is a group of its
    own).  Returns the sorted query order and the start of every group in
    it."""
    n = xy_a.shape[0]
    if n == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    if np.asarray(xy_b).reshape(-1, 2).shape[0] == 0:
        ab = [None] * n
    else:
        box = keypoint_box(xy_b)
        ab = [crossings(F, float(xy_a[i, 0]), float(xy_a[i, 1]), box) for i in range(n)]
    inf = float("inf")
    keys = np.array([(inf, inf, inf, inf) if c is None else (c[0][0], c[0][1], c[1][0], c[1][1])
                     for c in ab], dtype=np.float64).reshape(n, 4)
    order = np.lexsort((np.arange(n), keys[:, 3], keys[:, 2], keys[:, 1], keys[:, 0]))
    tol2 = tol_px * tol_px
    starts = [0]
    for s in range(1, n):
        cur, prev = ab[order[s]], ab[order[starts[-1] if to_leader else s - 1]]
        if cur is None or prev is None:
            starts.append(s)
            continue
        (ax, ay), (bx, by) = cur
        (px, py), (qx, qy) = prev
        dA = (ax - px) * (ax - px) + (ay - py) * (ay - py)
        dB = (bx - qx) * (bx - qx) + (by - qy) * (by - qy)
        if dA > tol2 or dB > tol2:
            starts.append(s)
    return order, np.array(starts, np.int64)


def grid_match(images, pairs, Fs, queries=None, ratio_num=64, ratio_den=100,
               accept_single=False, group_px=None, to_leader=False):
    """images: list of (xy, desc); pairs: list of (a, b, d); Fs (n_pairs, 3, 3).
    Per pair a dict of per-query arrays (match, d1, d2, count, accept) over
    the queries listed in queries[p] (default: all of a).  With group_px, the
    queries are grouped as in query_groups and every query takes the C' of
    its group's first line."""
    out = []
    for p, (a, b, d) in enumerate(pairs):
        xa, da = images[int(a)]
        xb, db = images[int(b)]
        qs = np.arange(xa.shape[0]) if queries is None else np.asarray(queries[p])
        leader = np.arange(xa.shape[0])
        if group_px is not None:
            order, starts = query_groups(xa, xb, Fs[p], group_px, to_leader)
            ends = np.append(starts[1:], len(order))
            for s0, s1 in zip(starts, ends):
                leader[order[s0:s1]] = order[s0]
        res = {k: np.zeros(len(qs), np.int64) for k in ("match", "d1", "d2", "count")}
        res["accept"] = np.zeros(len(qs), bool)
        for t, i in enumerate(qs):
            li = leader[i]
            cand = grid_candidates(xb, Fs[p], float(xa[li, 0]), float(xa[li, 1]), float(d))
            m, d1, d2, n, acc = two_nearest(da[i], db, cand, ratio_num, ratio_den, accept_single)
            res["match"][t], res["d1"][t], res["d2"][t], res["count"][t] = m, d1, d2, n
            res["accept"][t] = acc
        out.append(res)
    return out
