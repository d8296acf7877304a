"""Pins for the track oracle (Section 6.3): components against a boolean
transitive closure, triangulation against noise-free planted points."""
import numpy as np

import scenes
from oracle import tracks as tr


def test_components_hand_example():
    edges = [(5, 2), (2, 9), (7, 8), (3, 3)]
    lab = tr.tracks(10, edges)
    assert lab.tolist() == [0, 1, 2, 3, 4, 2, 6, 7, 7, 2]


def test_components_against_transitive_closure():
    rng = np.random.default_rng(31)
    for trial in range(15):
        n = int(rng.integers(1, 30))
        m = int(rng.integers(0, 40))
        edges = rng.integers(0, n, size=(m, 2))
        R = np.eye(n, dtype=bool)
        for u, v in edges:
            R[u, v] = R[v, u] = True
        for k in range(n):               # Floyd-Warshall on reachability
            R |= R[:, k:k + 1] & R[k:k + 1, :]
        expect = np.array([np.flatnonzero(R[i]).min() for i in range(n)])
        assert np.array_equal(tr.tracks(n, edges), expect)


def _cameras():
    cams = [scenes.look_at_camera(c) for c in scenes.generator._ring(5, 20.0, 5.0)]
    return [c.K @ np.hstack([c.R, c.t[:, None]]) for c in cams]


def test_triangulation_recovers_planted_points():
    P = _cameras()
    rng = np.random.default_rng(32)
    Xs = rng.uniform(-3, 3, size=(40, 3))
    label, img, xy = [], [], []
    for k, Xw in enumerate(Xs):
        views = rng.choice(5, size=int(rng.integers(2, 6)), replace=False)
        root = len(label)
        for v in views:
            h = P[v] @ np.append(Xw, 1.0)
            label.append(root)
            img.append(v)
            xy.append(h[:2] / h[2])
    X, n_obs = tr.triangulate(np.array(label), np.array(img), np.array(xy), np.stack(P))
    roots = sorted(set(label))
    assert np.allclose(X[roots], Xs, atol=1e-8)
    assert [int(n_obs[r]) for r in roots] == [label.count(r) for r in roots]


def test_single_observation_has_no_point():
    P = _cameras()
    X, n_obs = tr.triangulate(np.array([0, 1, 1]), np.array([0, 0, 1]),
                              np.array([[10.0, 20.0], [30.0, 40.0], [35.0, 41.0]]), np.stack(P))
    assert np.isnan(X[0]).all() and n_obs[0] == 1 and n_obs[1] == 2 and np.isfinite(X[1]).all()
