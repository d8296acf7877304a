"""MI355X-native geometry-aware guided feature matching.

Thin ctypes binding of libsfmgm.so (C ABI declared in include/sfm_gm.h).  The
functions below carry the C names and only marshal arguments; every step of
the matching runs in the library's HIP kernels.  PyTorch supplies device
memory and streams.  Importing this package does not need a GPU; calling
into the library does, and fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from .build import LIB_PATH, build  # noqa: F401

SFM_OK = 0
SFM_EINVAL = -1
SFM_ENOMEM = -2
SFM_EHIP = -3
SFM_ECAPACITY = -4
SFM_EKERNEL = -5
SFM_EBUSY = -6
SFM_ETIMEOUT = -7
SFM_ENOTFOUND = -8
INT32_MAX = 2**31 - 1


class SfmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class sfm_image(C.Structure):
    _fields_ = [("xy", C.c_void_p), ("desc", C.c_void_p), ("n", C.c_int32)]


class sfm_pair(C.Structure):
    _fields_ = [("a", C.c_int32), ("b", C.c_int32), ("band_px", C.c_double)]


class sfm_options(C.Structure):
    _fields_ = [("ratio_num", C.c_int32), ("ratio_den", C.c_int32),
                ("accept_single", C.c_int32), ("emit_all", C.c_int32),
                ("recheck_margin_px", C.c_double)]


class sfm_matches(C.Structure):
    _fields_ = [("query", C.c_void_p), ("match", C.c_void_p), ("d1", C.c_void_p),
                ("d2", C.c_void_p), ("capacity", C.c_int64), ("offset", C.c_void_p),
                ("n_comparisons", C.c_void_p), ("all_match", C.c_void_p),
                ("all_d1", C.c_void_p), ("all_d2", C.c_void_p), ("all_count", C.c_void_p),
                ("n_borderline", C.c_void_p)]


class sfm_candidates(C.Structure):
    _fields_ = [("cand", C.c_void_p), ("n_shared", C.c_void_p), ("n_cand", C.c_void_p),
                ("pairs", C.c_void_p), ("n_pairs", C.c_void_p)]


class sfm_server_cfg(C.Structure):
    _fields_ = [("max_batch_pairs", C.c_int32), ("max_inflight", C.c_int32),
                ("max_batch_queries", C.c_int64), ("opt", sfm_options)]


class sfm_preemptive_cfg(C.Structure):
    _fields_ = [("query_pct", C.c_int32), ("target_pct", C.c_int32),
                ("min_matches", C.c_int32), ("enough", C.c_int32),
                ("small_image", C.c_int32), ("pad", C.c_int32)]


class sfm_result_view(C.Structure):
    _fields_ = [("query", C.c_void_p), ("match", C.c_void_p), ("d1", C.c_void_p),
                ("d2", C.c_void_p), ("capacity", C.c_int64), ("n_matches", C.c_int64),
                ("n_comparisons", C.c_int64), ("arrival_ns", C.c_int64), ("done_ns", C.c_int64),
                ("status", C.c_int32), ("pad", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    """The loaded libsfmgm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run paper_1512_06235_amd.build() first "
                           "(there is no fallback path)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    sig = {
        "sfm_create": [C.POINTER(vp), i32, sz],
        "sfm_destroy": [vp],
        "sfm_register_images": [vp, C.POINTER(sfm_image), i32],
        "sfm_workspace_size": [vp, C.POINTER(sfm_pair), i32, C.POINTER(sz)],
        "sfm_guided_match": [vp, C.POINTER(sfm_pair), i32, vp, C.POINTER(sfm_options),
                             C.POINTER(sfm_matches), vp],
        "sfm_guided_match_plain": [vp, C.POINTER(sfm_pair), i32, vp, C.POINTER(sfm_options),
                                   C.POINTER(sfm_matches), vp],
        "sfm_guided_match_noalloc": [vp, C.POINTER(sfm_pair), i32, vp, C.POINTER(sfm_options),
                                     C.POINTER(sfm_matches), vp],
        "sfm_bruteforce_match": [vp, C.POINTER(sfm_pair), i32, vp, C.POINTER(sfm_options),
                                 C.POINTER(sfm_matches), vp],
        "sfm_band_error": [vp, C.POINTER(sfm_pair), i32, vp, C.POINTER(C.c_double),
                           C.POINTER(i64), vp],
        "sfm_grid_match": [vp, C.POINTER(sfm_pair), i32, vp, C.POINTER(sfm_options),
                           C.POINTER(sfm_matches), vp],
        "sfm_set_grid_grouping": [vp, C.c_double, i32],
        "sfm_grid_groups": [vp, C.POINTER(i64)],
        "sfm_preemptive_match": [vp, C.POINTER(sfm_pair), i32, C.POINTER(sfm_preemptive_cfg),
                                 C.POINTER(sfm_options), C.POINTER(sfm_matches), vp, vp],
        "sfm_sync": [vp, vp],
        "sfm_set_profiling": [vp, i32],
        "sfm_phase_times": [vp, C.POINTER(C.c_double), C.POINTER(i64)],
        "sfm_last_stats": [vp, C.POINTER(i64)],
        "sfm_last_error": [vp, C.c_char_p, sz],
        "sfm_server_start": [vp, C.POINTER(sfm_server_cfg)],
        "sfm_server_submit": [vp, C.POINTER(sfm_pair), vp, i64, C.POINTER(C.c_uint64)],
        "sfm_server_submit_batch": [vp, C.POINTER(sfm_pair), i32, vp, i64, vp],
        "sfm_server_poll": [vp, C.c_uint64, C.POINTER(sfm_result_view), i32],
        "sfm_server_stats": [vp, C.POINTER(i64)],
        "sfm_server_stop": [vp],
        "sfm_set_tuning": [vp, i32, i32],
        "sfm_set_graph_replay": [vp, i32],
        "sfm_set_covis_method": [vp, i32],
        "sfm_tracks": [vp, i64, vp, i64, vp, vp],
        "sfm_triangulate": [vp, i64, vp, vp, vp, vp, i32, vp, vp, vp],
        "sfm_candidate_images": [vp, vp, vp, i64, i32, i32, i32, i32, C.POINTER(sfm_candidates),
                                 vp],
        "sfm_get_tuning": [vp, C.POINTER(i32), C.POINTER(i32)],
        "sfm_autotune": [vp, C.POINTER(sfm_pair), i32, vp, C.POINTER(sfm_options), vp, i32,
                         C.POINTER(C.c_double)],
        "sfm_autotune_cached": [vp, C.POINTER(sfm_pair), i32, vp, C.POINTER(sfm_options), vp,
                                i32, C.c_char_p, C.POINTER(C.c_double), C.POINTER(i32)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.sfm_strerror.argtypes = [C.c_int]
    L.sfm_strerror.restype = C.c_char_p
    L.sfm_server_now_ns.argtypes = []
    L.sfm_server_now_ns.restype = C.c_int64
    _lib = L
    return L


def exported_symbols():
    """Names of the entry points include/sfm_gm.h declares."""
    return ["sfm_create", "sfm_destroy", "sfm_register_images", "sfm_workspace_size",
            "sfm_guided_match", "sfm_guided_match_plain", "sfm_guided_match_noalloc",
            "sfm_bruteforce_match",
            "sfm_band_error", "sfm_sync",
            "sfm_set_profiling", "sfm_phase_times", "sfm_last_stats", "sfm_strerror",
            "sfm_last_error", "sfm_server_now_ns", "sfm_server_start", "sfm_server_submit",
            "sfm_server_submit_batch", "sfm_server_poll", "sfm_server_stats", "sfm_server_stop", "sfm_set_tuning",
            "sfm_get_tuning", "sfm_autotune", "sfm_autotune_cached", "sfm_set_graph_replay",
            "sfm_candidate_images",
            "sfm_set_covis_method", "sfm_tracks", "sfm_triangulate", "sfm_preemptive_match",
            "sfm_grid_match", "sfm_set_grid_grouping", "sfm_grid_groups"]


# --- C names, marshalling only ------------------------------------------------------------

def sfm_strerror(status: int) -> str:
    return lib().sfm_strerror(int(status)).decode()


def sfm_last_error(ctx) -> str:
    buf = C.create_string_buffer(512)
    lib().sfm_last_error(ctx, buf, len(buf))
    return buf.value.decode()


def _check(ctx, status: int):
    if status != SFM_OK:
        msg = sfm_last_error(ctx) if ctx else ""
        raise SfmError(status, f"{sfm_strerror(status)}: {msg}")


def sfm_create(device: int = 0, workspace_budget_bytes: int = 0):
    ctx = C.c_void_p()
    st = lib().sfm_create(C.byref(ctx), int(device), int(workspace_budget_bytes))
    if st != SFM_OK:
        raise SfmError(st, f"sfm_create failed: {sfm_strerror(st)}")
    return ctx


def sfm_destroy(ctx) -> None:
    _check(None, lib().sfm_destroy(ctx))


def sfm_register_images(ctx, images) -> None:
    """images: list of (xy, desc) torch tensors on the context's device."""
    arr = (sfm_image * max(1, len(images)))()
    for k, (xy, desc) in enumerate(images):
        arr[k] = sfm_image(xy.data_ptr() if xy.numel() else None,
                           desc.data_ptr() if desc.numel() else None, int(xy.shape[0]))
    _check(ctx, lib().sfm_register_images(ctx, arr, len(images)))


_PAIR_DTYPE = np.dtype([("a", "<i4"), ("b", "<i4"), ("band_px", "<f8")])
assert _PAIR_DTYPE.itemsize == C.sizeof(sfm_pair)


class PairBatch:
    """Pairs and their fundamental matrices marshalled once for repeated calls:
    a host sfm_pair[n] and double[9n] that every matching call can take as is."""

    def __init__(self, pairs, F=None):
        n = len(pairs)
        self.n = n
        self.host = np.zeros(max(1, n), dtype=_PAIR_DTYPE)
        if n:
            arr = np.asarray(pairs, dtype=np.float64).reshape(n, 3)
            self.host["a"][:n] = arr[:, 0].astype(np.int32)
            self.host["b"][:n] = arr[:, 1].astype(np.int32)
            self.host["band_px"][:n] = arr[:, 2]
        self.F = None if F is None else np.ascontiguousarray(
            np.asarray(F, dtype=np.float64).reshape(n, 9))
        self.c_pairs = self.host.ctypes.data_as(C.POINTER(sfm_pair))

    def __len__(self):
        return self.n


def _pairs(pairs):
    return pairs.c_pairs if isinstance(pairs, PairBatch) else PairBatch(pairs).c_pairs


def sfm_workspace_size(ctx, pairs) -> int:
    n = C.c_size_t()
    _check(ctx, lib().sfm_workspace_size(ctx, _pairs(pairs), len(pairs), C.byref(n)))
    return n.value


def _call(fn_name, ctx, pairs, F, out: "MatchBuffers", opt: sfm_options, stream):
    """pairs: list of (a, b, band_px) or a PairBatch (then F may be None to use
    the batch's matrices)."""
    if isinstance(pairs, PairBatch) and (F is None or F is pairs.F):
        batch = pairs
    else:
        batch = PairBatch(pairs, F)
    st = getattr(lib(), fn_name)(ctx, batch.c_pairs, batch.n,
                                 batch.F.ctypes.data if batch.F is not None else None,
                                 C.byref(opt), C.byref(out.c_struct_cached()),
                                 stream.cuda_stream if stream is not None else None)
    _check(ctx, st)


def sfm_guided_match(ctx, pairs, F, out, opt, stream=None):
    _call("sfm_guided_match", ctx, pairs, F, out, opt, stream)


def sfm_guided_match_plain(ctx, pairs, F, out, opt, stream=None):
    _call("sfm_guided_match_plain", ctx, pairs, F, out, opt, stream)


NOALLOC_SCRATCH_BYTES = 64 << 20   # SFM_NOALLOC_SCRATCH_BYTES
NOALLOC_MAX_PAIRS = 8192           # SFM_NOALLOC_MAX_PAIRS


def sfm_guided_match_noalloc(ctx, pairs, F, out, opt, stream=None):
    """sfm_guided_match on the device's fixed scratch array: allocates nothing."""
    _call("sfm_guided_match_noalloc", ctx, pairs, F, out, opt, stream)


def sfm_bruteforce_match(ctx, pairs, F, out, opt, stream=None):
    _call("sfm_bruteforce_match", ctx, pairs, F, out, opt, stream)


def sfm_band_error(ctx, pairs, F=None, stream=None):
    """(largest |FP32 - FP64| epipolar distance in px over the evaluated slots
    within 2d, number of those slots); host-synchronous."""
    batch = pairs if isinstance(pairs, PairBatch) and F is None else PairBatch(pairs, F)
    err = C.c_double()
    n = C.c_int64()
    _check(ctx, lib().sfm_band_error(ctx, batch.c_pairs, batch.n,
                                     batch.F.ctypes.data if batch.F is not None else None,
                                     C.byref(err), C.byref(n),
                                     stream.cuda_stream if stream is not None else None))
    return err.value, n.value


def preemptive_cfg(query_pct=10, target_pct=20, min_matches=4, enough=0,
                   small_image=1000) -> sfm_preemptive_cfg:
    return sfm_preemptive_cfg(int(query_pct), int(target_pct), int(min_matches), int(enough),
                              int(small_image), 0)


def sfm_preemptive_match(ctx, pairs, out, opt=None, cfg=None, stream=None) -> np.ndarray:
    """Staged coarse matching; returns the stages each pair ran (0 whole, 1, 2).
    pairs: list of (a, b) or (a, b, band) (the band is ignored) or a PairBatch."""
    if not isinstance(pairs, PairBatch):
        pairs = PairBatch([(p[0], p[1], 0.0) for p in pairs], None)
    stages = np.zeros(max(1, pairs.n), np.int32)
    st = lib().sfm_preemptive_match(
        ctx, pairs.c_pairs, pairs.n, C.byref(cfg if cfg is not None else preemptive_cfg()),
        C.byref(opt if opt is not None else options()), C.byref(out.c_struct_cached()),
        stages.ctypes.data, stream.cuda_stream if stream is not None else None)
    _check(ctx, st)
    return stages[:pairs.n]


def sfm_grid_match(ctx, pairs, F, out, opt, stream=None):
    """The grid search of Section 6.2.1; band_px of each pair is the cell parameter d."""
    _call("sfm_grid_match", ctx, pairs, F, out, opt, stream)


def sfm_set_grid_grouping(ctx, px: float, to_leader: bool = False) -> None:
    """Group queries whose lines cross b's box within px (0 = off) of the
    previous line's crossings, or of the group's first line's, in sfm_grid_match."""
    _check(ctx, lib().sfm_set_grid_grouping(ctx, float(px), int(bool(to_leader))))


def sfm_grid_groups(ctx) -> int:
    n = C.c_int64()
    _check(ctx, lib().sfm_grid_groups(ctx, C.byref(n)))
    return n.value


def sfm_sync(ctx, stream=None) -> None:
    _check(ctx, lib().sfm_sync(ctx, stream.cuda_stream if stream is not None else None))


def sfm_set_profiling(ctx, enable: bool) -> None:
    _check(ctx, lib().sfm_set_profiling(ctx, int(bool(enable))))


def sfm_phase_times(ctx):
    """(prepare_ms, match_ms, emit_ms, n_records) summed since the last call."""
    ms = (C.c_double * 3)()
    n = C.c_int64()
    _check(ctx, lib().sfm_phase_times(ctx, ms, C.byref(n)))
    return ms[0], ms[1], ms[2], n.value


def sfm_last_stats(ctx) -> dict:
    """Totals of the last matching call (waits for it)."""
    v = (C.c_int64 * 5)()
    _check(ctx, lib().sfm_last_stats(ctx, v))
    return {"comparisons": v[0], "slots": v[1], "tie_passes": v[2], "accepted": v[3],
            "borderline": v[4]}


def sfm_server_now_ns() -> int:
    return int(lib().sfm_server_now_ns())


def sfm_server_start(ctx, max_batch_pairs=256, max_inflight=2, max_batch_queries=1 << 22,
                     opt: sfm_options = None) -> None:
    cfg = sfm_server_cfg(int(max_batch_pairs), int(max_inflight), int(max_batch_queries),
                         opt if opt is not None else options())
    _check(ctx, lib().sfm_server_start(ctx, C.byref(cfg)))


def sfm_server_submit(ctx, pair, F, arrival_ns: int = 0) -> int:
    a, b, band = pair
    p = sfm_pair(int(a), int(b), float(band))
    Fh = np.ascontiguousarray(np.asarray(F, dtype=np.float64).reshape(9))
    t = C.c_uint64()
    _check(ctx, lib().sfm_server_submit(ctx, C.byref(p), Fh.ctypes.data, int(arrival_ns),
                                        C.byref(t)))
    return t.value


def sfm_server_submit_batch(ctx, pairs, F=None, arrival_ns: int = 0) -> np.ndarray:
    """Submit a burst of requests at once; returns their tickets (uint64[n]).
    `pairs` may be a PairBatch holding its F."""
    b = pairs if isinstance(pairs, PairBatch) else PairBatch(pairs, F)
    Fh = b.F if F is None else np.ascontiguousarray(np.asarray(F, dtype=np.float64).reshape(-1, 9))
    if Fh is None or Fh.shape[0] != b.n:
        raise ValueError("one F per pair is required")
    tickets = np.zeros(max(1, b.n), dtype=np.uint64)
    _check(ctx, lib().sfm_server_submit_batch(ctx, b.c_pairs, b.n, Fh.ctypes.data,
                                              int(arrival_ns), tickets.ctypes.data))
    return tickets[:b.n]


def sfm_server_poll(ctx, ticket: int, capacity: int, timeout_ms: int = -1):
    """The request's result as a dict with host arrays, or None on SFM_ETIMEOUT."""
    bufs = [np.empty(max(1, int(capacity)), dtype=np.int32) for _ in range(4)]
    v = sfm_result_view(*(b.ctypes.data for b in bufs), int(capacity), 0, 0, 0, 0, 0, 0)
    st = lib().sfm_server_poll(ctx, int(ticket), C.byref(v), int(timeout_ms))
    if st == SFM_ETIMEOUT:
        return None
    _check(ctx, st)
    n = int(v.n_matches)
    # Copies of the filled rows, so a held result does not pin `capacity` rows.
    return {"status": int(v.status), "query": bufs[0][:n].copy(), "match": bufs[1][:n].copy(),
            "d1": bufs[2][:n].copy(), "d2": bufs[3][:n].copy(),
            "n_comparisons": int(v.n_comparisons),
            "arrival_ns": int(v.arrival_ns), "done_ns": int(v.done_ns)}


def sfm_server_stats(ctx) -> dict:
    v = (C.c_int64 * 3)()
    _check(ctx, lib().sfm_server_stats(ctx, v))
    return {"launches": v[0], "launched": v[1], "waiting": v[2]}


def sfm_server_stop(ctx) -> None:
    _check(ctx, lib().sfm_server_stop(ctx))


class CandidateBuffers:
    """Device outputs of sfm_candidate_images for n_images images, top_k each."""

    def __init__(self, n_images: int, top_k: int, device="cuda:0", with_pairs: bool = True):
        import torch
        self.n_images, self.top_k = int(n_images), int(top_k)
        n = max(1, self.n_images * self.top_k)
        self.cand = torch.full((n,), -1, dtype=torch.int32, device=device)
        self.n_shared = torch.zeros(n, dtype=torch.int32, device=device)
        self.n_cand = torch.zeros(max(1, self.n_images), dtype=torch.int32, device=device)
        self.pairs = torch.zeros(2 * n, dtype=torch.int32, device=device) if with_pairs else None
        self.n_pairs = torch.zeros(1, dtype=torch.int64, device=device)

    def c_struct(self):
        return sfm_candidates(self.cand.data_ptr(), self.n_shared.data_ptr(),
                              self.n_cand.data_ptr(),
                              self.pairs.data_ptr() if self.pairs is not None else None,
                              self.n_pairs.data_ptr())

    def lists(self):
        """Host lists per image q of (candidate, shared count) in rank order."""
        cand = self.cand.cpu().numpy().reshape(-1)
        shared = self.n_shared.cpu().numpy().reshape(-1)
        nc = self.n_cand.cpu().numpy()
        k = self.top_k
        return [[(int(cand[q * k + r]), int(shared[q * k + r])) for r in range(int(nc[q]))]
                for q in range(self.n_images)]

    def unique_pairs(self):
        n = int(self.n_pairs.cpu()[0])
        return self.pairs[:2 * n].cpu().numpy().reshape(n, 2)


def sfm_candidate_images(ctx, vis_off, vis_pts, n_points: int, threshold: int, top_k: int,
                         out: "CandidateBuffers", stream=None) -> None:
    """vis_off (int32[n_images + 1]) and vis_pts (int32[nnz]) are device tensors."""
    n_images = int(vis_off.shape[0]) - 1
    nnz = int(vis_pts.shape[0])
    s = out.c_struct()
    _check(ctx, lib().sfm_candidate_images(ctx, vis_off.data_ptr(), vis_pts.data_ptr(), nnz,
                                           n_images, int(n_points), int(threshold), int(top_k),
                                           C.byref(s),
                                           stream.cuda_stream if stream is not None else None))


def sfm_tracks(ctx, n_nodes: int, edges, label, stream=None) -> None:
    """edges: device int32 tensor (n_edges, 2) of node ids; label: device int32[n_nodes]."""
    n_edges = int(edges.shape[0]) if edges is not None else 0
    _check(ctx, lib().sfm_tracks(ctx, int(n_nodes), edges.data_ptr() if n_edges else None,
                                 n_edges, label.data_ptr() if n_nodes else None,
                                 stream.cuda_stream if stream is not None else None))


def sfm_triangulate(ctx, label, node_image, node_xy, P, X, n_obs, stream=None) -> None:
    """Device tensors: label, node_image int32[n]; node_xy float32[n, 2];
    P float64[n_images, 3, 4]; X float64[n, 3]; n_obs int32[n]."""
    n = int(label.shape[0])
    _check(ctx, lib().sfm_triangulate(ctx, n, label.data_ptr(), node_image.data_ptr(),
                                      node_xy.data_ptr(), P.data_ptr(), int(P.shape[0]),
                                      X.data_ptr(), n_obs.data_ptr(),
                                      stream.cuda_stream if stream is not None else None))


def sfm_set_covis_method(ctx, method: int) -> None:
    _check(ctx, lib().sfm_set_covis_method(ctx, int(method)))


def sfm_set_graph_replay(ctx, enable: bool) -> None:
    _check(ctx, lib().sfm_set_graph_replay(ctx, 1 if enable else 0))


def sfm_set_tuning(ctx, group_tiles: int, features_per_bin: int) -> None:
    _check(ctx, lib().sfm_set_tuning(ctx, int(group_tiles), int(features_per_bin)))


def sfm_get_tuning(ctx):
    """(group_tiles, features_per_bin) of the context."""
    t, f = C.c_int32(), C.c_int32()
    _check(ctx, lib().sfm_get_tuning(ctx, C.byref(t), C.byref(f)))
    return t.value, f.value


AUTOTUNE_GROUP_TILES = (4, 8)
AUTOTUNE_FEATURES_PER_BIN = (4, 8, 16)


def sfm_autotune(ctx, pairs, F, opt=None, stream=None, repeats: int = 3):
    """Time every tuning on this batch, keep the fastest; returns
    {(group_tiles, features_per_bin): ms per call}."""
    batch = pairs if isinstance(pairs, PairBatch) and F is None else PairBatch(pairs, F)
    ms = (C.c_double * (len(AUTOTUNE_GROUP_TILES) * len(AUTOTUNE_FEATURES_PER_BIN)))()
    st = lib().sfm_autotune(ctx, batch.c_pairs, batch.n, batch.F.ctypes.data,
                            C.byref(opt if opt is not None else options()),
                            stream.cuda_stream if stream is not None else None, int(repeats), ms)
    _check(ctx, st)
    return {(t, f): ms[3 * i + j] for i, t in enumerate(AUTOTUNE_GROUP_TILES)
            for j, f in enumerate(AUTOTUNE_FEATURES_PER_BIN)}


TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def sfm_autotune_cached(ctx, pairs, F, cache_path=TUNE_CACHE, opt=None, stream=None,
                        repeats: int = 3):
    """sfm_autotune through the tuning cache at cache_path; returns
    (from_cache, {(group_tiles, features_per_bin): ms per call} or None)."""
    batch = pairs if isinstance(pairs, PairBatch) and F is None else PairBatch(pairs, F)
    ms = (C.c_double * (len(AUTOTUNE_GROUP_TILES) * len(AUTOTUNE_FEATURES_PER_BIN)))()
    hit = C.c_int32()
    st = lib().sfm_autotune_cached(ctx, batch.c_pairs, batch.n, batch.F.ctypes.data,
                                   C.byref(opt if opt is not None else options()),
                                   stream.cuda_stream if stream is not None else None,
                                   int(repeats), os.fsencode(cache_path), ms, C.byref(hit))
    _check(ctx, st)
    if hit.value:
        return True, None
    return False, {(t, f): ms[3 * i + j] for i, t in enumerate(AUTOTUNE_GROUP_TILES)
                   for j, f in enumerate(AUTOTUNE_FEATURES_PER_BIN)}


def options(ratio_num=64, ratio_den=100, accept_single=False, emit_all=False,
            recheck_margin_px=1e-3) -> sfm_options:
    return sfm_options(int(ratio_num), int(ratio_den), int(bool(accept_single)),
                       int(bool(emit_all)), float(recheck_margin_px))


class MatchBuffers:
    """Device output tensors for up to `capacity` queries over `n_pairs` pairs."""

    def __init__(self, capacity: int, n_pairs: int, device, emit_all: bool = False):
        import torch
        i32 = dict(dtype=torch.int32, device=device)
        cap = max(1, int(capacity))
        self.capacity = int(capacity)
        self.n_pairs = int(n_pairs)
        self.query = torch.empty(cap, **i32)
        self.match = torch.empty(cap, **i32)
        self.d1 = torch.empty(cap, **i32)
        self.d2 = torch.empty(cap, **i32)
        self.offset = torch.zeros(n_pairs + 1, dtype=torch.int64, device=device)
        self.n_comparisons = torch.zeros(max(1, n_pairs), dtype=torch.int64, device=device)
        self.n_borderline = torch.zeros(max(1, n_pairs), dtype=torch.int64, device=device)
        self.emit_all = emit_all
        if emit_all:
            self.all_match = torch.empty(cap, **i32)
            self.all_d1 = torch.empty(cap, **i32)
            self.all_d2 = torch.empty(cap, **i32)
            self.all_count = torch.empty(cap, **i32)

    def c_struct_cached(self) -> sfm_matches:
        if getattr(self, "_c", None) is None:
            self._c = self.c_struct()
        return self._c

    def c_struct(self) -> sfm_matches:
        ea = self.emit_all
        return sfm_matches(self.query.data_ptr(), self.match.data_ptr(), self.d1.data_ptr(),
                           self.d2.data_ptr(), self.capacity, self.offset.data_ptr(),
                           self.n_comparisons.data_ptr(),
                           self.all_match.data_ptr() if ea else None,
                           self.all_d1.data_ptr() if ea else None,
                           self.all_d2.data_ptr() if ea else None,
                           self.all_count.data_ptr() if ea else None,
                           self.n_borderline.data_ptr())

    def pair(self, p: int):
        """Host copies of pair p's accepted (query, match, d1, d2)."""
        off = self.offset.cpu().numpy()
        s, e = int(off[p]), int(off[p + 1])
        return tuple(t[s:e].cpu().numpy() for t in (self.query, self.match, self.d1, self.d2))


class Matcher:
    """Context + registered images; results land in MatchBuffers."""

    def __init__(self, device: int = 0, workspace_budget_bytes: int = 0):
        self.device = device
        self.ctx = sfm_create(device, workspace_budget_bytes)
        self.images = []

    def close(self):
        if self.ctx is not None:
            sfm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def register(self, images):
        """images: list of (xy, desc) numpy arrays or device tensors."""
        import torch
        dev = torch.device("cuda", self.device)
        held = []
        for xy, desc in images:
            xy_t = torch.as_tensor(np.ascontiguousarray(xy, dtype=np.float32)).reshape(-1, 2) \
                if not torch.is_tensor(xy) else xy
            d_t = torch.as_tensor(np.ascontiguousarray(desc, dtype=np.uint8)).reshape(-1, 128) \
                if not torch.is_tensor(desc) else desc
            held.append((xy_t.to(dev).contiguous(), d_t.to(dev).contiguous()))
        sfm_register_images(self.ctx, held)
        self.images = held
        return self

    def n_features(self, k: int) -> int:
        return int(self.images[k][0].shape[0])

    def buffers(self, pairs, emit_all: bool = False) -> MatchBuffers:
        cap = sum(self.n_features(a) for a, _, _ in pairs)
        return MatchBuffers(cap, len(pairs), f"cuda:{self.device}", emit_all)

    def match(self, pairs, F, form: str = "batched", emit_all: bool = False, out=None,
              stream=None, sync: bool = True, **opt_kw) -> MatchBuffers:
        out = out if out is not None else self.buffers(pairs, emit_all)
        opt = options(emit_all=emit_all, **opt_kw)
        if form == "batched":
            sfm_guided_match(self.ctx, pairs, F, out, opt, stream)
        elif form == "plain":
            sfm_guided_match_plain(self.ctx, pairs, F, out, opt, stream)
        elif form == "noalloc":
            sfm_guided_match_noalloc(self.ctx, pairs, F, out, opt, stream)
        elif form == "bruteforce":
            sfm_bruteforce_match(self.ctx, pairs, F, out, opt, stream)
        elif form == "grid":
            sfm_grid_match(self.ctx, pairs, F, out, opt, stream)
        else:
            raise ValueError(form)
        if sync:
            sfm_sync(self.ctx, stream)
        return out


def infinite_band() -> float:
    return math.inf
