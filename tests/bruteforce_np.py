"""A second, deliberately different CPU matcher for tiny inputs.

Where the oracle keeps a running pair of nearest candidates, this one lists
every in-band candidate with its distance, sorts the list by (distance,
index) and reads the first two entries.  It pins the oracle's selection,
tie-breaking and ratio-test logic; the band predicate itself is pinned
separately by closed-form geometry.
"""
import numpy as np


def match_pair(xy_a, desc_a, xy_b, desc_b, F, band, ratio_num=64, ratio_den=100,
               accept_single=False, ignore_band=False):
    xa = np.asarray(xy_a, np.float64)
    xb = np.asarray(xy_b, np.float64)
    da = np.asarray(desc_a, np.int64)
    db = np.asarray(desc_b, np.int64)
    F = np.asarray(F, np.float64).reshape(3, 3)
    out = []
    for i in range(xa.shape[0]):
        a, b, c = F @ np.array([xa[i, 0], xa[i, 1], 1.0])
        norm = np.hypot(a, b)
        if ignore_band:
            inband = np.ones(xb.shape[0], bool)
        elif not (norm > 0 and np.isfinite(norm) and np.isfinite(c)):
            inband = np.zeros(xb.shape[0], bool)
        else:
            inband = np.abs(a * xb[:, 0] + b * xb[:, 1] + c) / norm <= band
        js = np.nonzero(inband)[0]
        D = ((db[js] - da[i][None, :]) ** 2).sum(axis=1)
        order = np.lexsort((js, D))          # primary key D, then index
        cand = [(int(D[k]), int(js[k])) for k in order]
        match = cand[0][1] if cand else -1
        d1 = cand[0][0] if cand else 2**31 - 1
        d2 = cand[1][0] if len(cand) > 1 else 2**31 - 1
        if len(cand) >= 2:
            acc = ratio_den * d1 < ratio_num * d2
        else:
            acc = len(cand) == 1 and accept_single
        out.append((match, d1, d2, len(cand), bool(acc)))
    return out
