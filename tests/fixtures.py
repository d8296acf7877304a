"""Small seeded or hand-made inputs shared by the CPU and GPU tests."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_hand_fixture(name="hand_pure_translation.txt"):
    """Parse a text fixture: returns (xy_a, desc_a, xy_b, desc_b, F, band, expect)."""
    F = None
    band = None
    q, t, expect = [], [], []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "F":
                F = np.array([float(v) for v in tok[1:10]]).reshape(3, 3)
            elif tok[0] == "band":
                band = float(tok[1])
            elif tok[0] in ("query", "target"):
                d = np.zeros(128, np.uint8)
                for kv in tok[4:]:
                    k, v = kv.split(":")
                    d[int(k)] = int(v)
                (q if tok[0] == "query" else t).append((int(tok[1]), float(tok[2]),
                                                        float(tok[3]), d))
            elif tok[0] == "expect":
                expect.append(tuple(int(v) for v in tok[1:7]))
    q.sort(key=lambda r: r[0])
    t.sort(key=lambda r: r[0])
    xy_a = np.array([[r[1], r[2]] for r in q], np.float32)
    xy_b = np.array([[r[1], r[2]] for r in t], np.float32)
    desc_a = np.stack([r[3] for r in q])
    desc_b = np.stack([r[3] for r in t])
    return xy_a, desc_a, xy_b, desc_b, F, band, sorted(expect)


def random_pair(n_a, n_b, seed, F=None, spread=1.0):
    """Uniform keypoints in a 1024x768 image and random descriptors 0..127.

    Without F, uses the fundamental matrix of two cameras 15 deg apart on a
    circle of radius 20 (epipole about 7.6k px to the side)."""
    import scenes
    rng = np.random.default_rng(seed)
    xy_a = np.stack([rng.uniform(0, 1024, n_a), rng.uniform(0, 768, n_a)], 1).astype(np.float32)
    xy_b = np.stack([rng.uniform(0, 1024, n_b), rng.uniform(0, 768, n_b)], 1).astype(np.float32)
    desc_a = np.clip(rng.normal(64, 30 * spread, (n_a, 128)), 0, 127).astype(np.uint8)
    desc_b = np.clip(rng.normal(64, 30 * spread, (n_b, 128)), 0, 127).astype(np.uint8)
    if F is None:
        F = scenes.make_two_view_2k().F
    return xy_a, desc_a, xy_b, desc_b, np.asarray(F, np.float64)


def translation_F(e):
    """F = [e]_x: pure translation with K = I, R = I; epipole e = (ex, ey, ez)."""
    x, y, z = e
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])
