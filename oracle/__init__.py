"""CPU oracle for geometry-aware guided matching -- TEST INFRASTRUCTURE.

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It wraps `liboracle.so`, a plain C++ reference built
from `sfm_oracle.cpp` (FP64 epipolar geometry of Section 6.2 eqs. 2-3, linear
search over every target feature, exact integer squared-L2 distances, the two
nearest candidates and the ratio test).  It shares no code with the GPU
library and never calls it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "sfm_oracle.cpp")]

INT32_MAX = 2**31 - 1


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (no contraction of FP64 expressions)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["g++", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
           "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", tmp] + SOURCES
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Image(C.Structure):
    _fields_ = [("xy", C.c_void_p), ("desc", C.c_void_p), ("n", C.c_int32)]


class _Pair(C.Structure):
    _fields_ = [("a", C.c_int32), ("b", C.c_int32), ("band_px", C.c_double)]


class _Options(C.Structure):
    _fields_ = [("ratio_num", C.c_int32), ("ratio_den", C.c_int32),
                ("accept_single", C.c_int32), ("ignore_band", C.c_int32),
                ("borderline_px", C.c_double)]


class _Result(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in
                ("match", "d1", "d2", "count", "borderline", "accept",
                 "n_comparisons", "n_borderline", "n_accepted")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.sfm_oracle_match.restype = C.c_int
        L.sfm_oracle_match.argtypes = [C.POINTER(_Image), C.c_int32, C.POINTER(_Pair), C.c_int32,
                                       C.c_void_p, C.POINTER(_Options), C.POINTER(_Result),
                                       C.c_int32]
        L.sfm_oracle_desc_dist.restype = C.c_int32
        L.sfm_oracle_desc_dist.argtypes = [C.c_void_p, C.c_void_p]
        L.sfm_oracle_epipolar_distance.restype = C.c_double
        L.sfm_oracle_epipolar_distance.argtypes = [C.c_void_p, C.c_float, C.c_float,
                                                   C.c_float, C.c_float]
        L.sfm_oracle_threads_used.restype = C.c_int32
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class OracleResult:
    """Per-query arrays (pair-major, query order) and per-pair totals."""

    def __init__(self, q_off, match, d1, d2, count, borderline, accept, n_cmp, n_bl, n_acc):
        self.q_off = q_off
        self.match, self.d1, self.d2 = match, d1, d2
        self.count, self.borderline, self.accept = count, borderline, accept
        self.n_comparisons, self.n_borderline, self.n_accepted = n_cmp, n_bl, n_acc

    def pair(self, p: int) -> dict:
        s, e = int(self.q_off[p]), int(self.q_off[p + 1])
        return {k: getattr(self, k)[s:e] for k in
                ("match", "d1", "d2", "count", "borderline", "accept")}

    def matches(self, p: int):
        """Accepted (query, match, d1, d2) rows of pair p in ascending query order."""
        r = self.pair(p)
        q = np.nonzero(r["accept"])[0].astype(np.int32)
        return q, r["match"][q], r["d1"][q], r["d2"][q]


def match(images, pairs, Fs, ratio_num=64, ratio_den=100, accept_single=False,
          ignore_band=False, borderline_px=1e-3, n_threads=0) -> OracleResult:
    """Run the oracle.

    images: list of (xy float32 (n,2), desc uint8 (n,128)); pairs: list of
    (a, b, band_px); Fs: array (n_pairs, 3, 3) float64 with x_b^T F x_a = 0.
    """
    keep = []
    imgs = (_Image * max(1, len(images)))()
    for k, (xy, desc) in enumerate(images):
        xy = np.ascontiguousarray(xy, dtype=np.float32).reshape(-1, 2)
        desc = np.ascontiguousarray(desc, dtype=np.uint8).reshape(-1, 128)
        assert xy.shape[0] == desc.shape[0]
        keep += [xy, desc]
        imgs[k] = _Image(_ptr(xy), _ptr(desc), xy.shape[0])
    P = len(pairs)
    prs = (_Pair * max(1, P))()
    for k, (a, b, band) in enumerate(pairs):
        prs[k] = _Pair(int(a), int(b), float(band))
    F = np.ascontiguousarray(np.asarray(Fs, dtype=np.float64).reshape(P, 9))
    q_off = np.zeros(P + 1, np.int64)
    for k, (a, _, _) in enumerate(pairs):
        q_off[k + 1] = q_off[k] + (images[a][0].shape[0] if 0 <= a < len(images) else 0)
    nq = int(q_off[-1])
    m = np.empty(nq, np.int32); d1 = np.empty(nq, np.int32); d2 = np.empty(nq, np.int32)
    cnt = np.empty(nq, np.int32); bl = np.empty(nq, np.int32); acc = np.empty(nq, np.uint8)
    n_cmp = np.empty(P, np.int64); n_bl = np.empty(P, np.int64); n_acc = np.empty(P, np.int64)
    res = _Result(*[_ptr(x) for x in (m, d1, d2, cnt, bl, acc, n_cmp, n_bl, n_acc)])
    opt = _Options(ratio_num, ratio_den, int(accept_single), int(ignore_band), borderline_px)
    rc = lib().sfm_oracle_match(imgs, len(images), prs, P, _ptr(F), C.byref(opt), C.byref(res),
                                int(n_threads))
    if rc != 0:
        raise ValueError(f"sfm_oracle_match rejected its arguments (status {rc})")
    return OracleResult(q_off, m, d1, d2, cnt, bl, acc.astype(bool), n_cmp, n_bl, n_acc)


def desc_dist(p: np.ndarray, q: np.ndarray) -> int:
    p = np.ascontiguousarray(p, dtype=np.uint8)
    q = np.ascontiguousarray(q, dtype=np.uint8)
    return int(lib().sfm_oracle_desc_dist(_ptr(p), _ptr(q)))


def epipolar_distance(F, xa, ya, xb, yb) -> float:
    F = np.ascontiguousarray(np.asarray(F, dtype=np.float64).reshape(9))
    return float(lib().sfm_oracle_epipolar_distance(_ptr(F), xa, ya, xb, yb))


def threads_used() -> int:
    return int(lib().sfm_oracle_threads_used())
