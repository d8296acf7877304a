"""Track merging and triangulation -- TEST INFRASTRUCTURE.

Only tests/ and the benchmark's CPU-baseline leg may use this module.  It
restates Section 6.3 directly and shares no code with the GPU library:

* tracks are the connected components of the match graph (nodes are
  observations, edges accepted matches), found by a graph search as in the
  paper; each node is labelled with the smallest node id of its component
  (visiting start nodes in ascending order makes that the search's start);
* each track is triangulated by linear least squares: an observation (x, y)
  in camera P (rows p1, p2, p3) contributes the rows x p3 - p1 and y p3 - p2
  of A, and X solves A[:, :3] X = -A[:, 3] (numpy's SVD-based lstsq); a track
  of one observation has no point (NaN).  Tracks are not split when two of
  their features lie in one image: the paper does not say, so none are.
"""
from __future__ import annotations

import numpy as np


def tracks(n_nodes: int, edges) -> np.ndarray:
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    order = np.argsort(np.concatenate([edges[:, 0], edges[:, 1]]), kind="stable")
    src = np.concatenate([edges[:, 0], edges[:, 1]])[order]
    dst = np.concatenate([edges[:, 1], edges[:, 0]])[order]
    start = np.searchsorted(src, np.arange(n_nodes + 1))
    label = np.full(n_nodes, -1, dtype=np.int64)
    for s in range(n_nodes):
        if label[s] >= 0:
            continue
        label[s] = s
        stack = [s]
        while stack:
            x = stack.pop()
            for y in dst[start[x]:start[x + 1]]:
                if label[y] < 0:
                    label[y] = s
                    stack.append(int(y))
    return label


def triangulate(label, node_image, node_xy, P):
    """X (n, 3) and number of observations (n,) for every root; zeros and NaN
    elsewhere (non-roots: n_obs 0)."""
    label = np.asarray(label)
    n = label.shape[0]
    X = np.full((n, 3), np.nan)
    n_obs = np.zeros(n, dtype=np.int64)
    order = np.argsort(label, kind="stable")
    bounds = np.flatnonzero(np.diff(label[order])) + 1
    for grp in np.split(order, bounds):
        if grp.size == 0:
            continue
        r = int(label[grp[0]])
        n_obs[r] = grp.size
        if grp.size < 2:
            continue
        rows = []
        for i in grp:
            p = np.asarray(P[int(node_image[i])], dtype=np.float64).reshape(3, 4)
            x, y = float(node_xy[i][0]), float(node_xy[i][1])
            rows.append(x * p[2] - p[0])
            rows.append(y * p[2] - p[1])
        A = np.asarray(rows)
        X[r] = np.linalg.lstsq(A[:, :3], -A[:, 3], rcond=None)[0]
    return X, n_obs
