/*
 * sfm_gm.h -- geometry-aware guided feature matching on one MI355X (gfx950).
 *
 * C ABI of libsfmgm.so.  No exceptions, C++ types or torch types cross it;
 * every call returns an int status (SFM_OK or a negative SFM_E* code) and
 * sfm_strerror() names it.
 *
 * What it computes (Section 6.2 of the paper, "Fast Geometry-aware Feature
 * Matching", and Appendix A).  For an image pair (a, b) with fundamental
 * matrix F, every feature of a is a query.  Its epipolar line in b is
 * l = F (x, y, 1)^T (convention x_b^T F x_a = 0).  Its candidate set is
 *     C = { features p' of b : |l . (x', y', 1)| / sqrt(l_0^2 + l_1^2) <= d }
 * (eqs. 2-3, inclusive, d = band_px, the maximum perpendicular distance).  Its
 * match is the candidate with the smallest squared L2 descriptor distance D1
 * (exact integer over uint8 values 0..127, ties to the lowest index of b),
 * accepted when at least two candidates exist and
 *     ratio_den * D1 < ratio_num * D2            (default 100*D1 < 64*D2),
 * D2 being the second-smallest distance over the other candidates (the 2-NN
 * ratio test of Section 6.2.2 / Appendix A step 4 with ratio 0.8 on
 * distances).  A query whose line is degenerate (l_0 = l_1 = 0) has no
 * candidates.
 *
 * Exactness.  Epipolar distances are evaluated in FP32 on centred
 * coordinates from lines normalised in FP64.  A candidate whose FP32 distance
 * lies within recheck_margin_px of d (sfm_options, default 1e-3 px) is
 * decided again in FP64 on the caller's F and the original keypoints, with
 * the operations of the definition above in order: l = F (x, y, 1)^T row by
 * row, s = sqrt(l_0^2 + l_1^2), |l . (x', y', 1)| / s <= d.  The FP32 error
 * is below 1e-4 px on centred coordinates (sfm_band_error measures it), so
 * with the default margin membership, the match index, D1, D2 and the
 * candidate count all equal that FP64 evaluation bit for bit.  The number of
 * candidates decided in FP64 is reported per pair (sfm_matches.n_borderline).
 *
 * Memory.  All image, descriptor and output buffers are device memory owned
 * by the caller.  Pair lists and fundamental matrices are host memory, read
 * before the call returns.  The library owns only its context: the table of
 * registered images, per-feature squared norms and a workspace it grows on
 * demand up to the budget given to sfm_create().
 *
 * Around the matcher, the library also selects the image pairs to match
 * from the coarse model's point-camera visibility (Section 6.1,
 * sfm_candidate_images) and merges the accepted matches of all pairs into
 * tracks and triangulates them (Section 6.3, sfm_tracks, sfm_triangulate).
 *
 * Streams.  Matching calls enqueue their work on the given HIP stream
 * (hipStream_t passed as void*, NULL = the default stream) and return without
 * waiting.  Errors found on the host return immediately; an error raised on
 * the device is reported by sfm_sync() as SFM_EKERNEL.  Calls on one context
 * must not overlap: they share its workspace.
 */
#ifndef SFM_GM_H
#define SFM_GM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SFM_OK = 0,
  SFM_EINVAL = -1,     /* an argument is invalid (message in sfm_last_error) */
  SFM_ENOMEM = -2,     /* a device or pinned host allocation failed */
  SFM_EHIP = -3,       /* the HIP runtime returned an error */
  SFM_ECAPACITY = -4,  /* workspace budget or output capacity too small */
  SFM_EKERNEL = -5,    /* a kernel raised its device error flag */
  SFM_EBUSY = -6,      /* the server queue is full, or the server is not running */
  SFM_ETIMEOUT = -7,   /* sfm_server_poll: result not ready within the timeout */
  SFM_ENOTFOUND = -8   /* sfm_server_poll: unknown or already collected ticket */
};

typedef struct sfm_ctx sfm_ctx;

/* One image: n features, keypoints xy = float[2*n] (x, y in pixels, x to the
 * right, y down) and descriptors desc = uint8[128*n] row-major, every byte in
 * 0..127.  Both are device pointers; n may be 0 (pointers then unused). */
typedef struct {
  const float* xy;
  const uint8_t* desc;
  int32_t n;
} sfm_image;

/* Match the features of registered image a (queries) into image b (targets)
 * with band half-width band_px >= 0 (pixels; +inf = every feature of b). */
typedef struct {
  int32_t a;
  int32_t b;
  double band_px;
} sfm_pair;

typedef struct {
  int32_t ratio_num;      /* 64: accept iff ratio_den * D1 < ratio_num * D2 */
  int32_t ratio_den;      /* 100 */
  int32_t accept_single;  /* 0: a query with exactly one candidate is rejected */
  int32_t emit_all;       /* 0: fill the all_* arrays of sfm_matches when nonzero */
  double recheck_margin_px; /* 1e-3: FP32 distances within this of d are decided
                             * again in FP64 (0: FP32 only); finite, >= 0 */
} sfm_options;

/* Outputs, all device memory owned by the caller.
 * Accepted matches are written pair after pair in input order and, within a
 * pair, in ascending query index: rows offset[p] .. offset[p+1]-1 belong to
 * pair p and hold (query index in a, match index in b, D1, D2).
 * capacity must be >= the sum of n_a over the pairs (one row per query at
 * most), so a call never runs out of room.
 * n_comparisons (optional, int64[n_pairs]) receives the number of candidate
 * comparisons of each pair, i.e. the sum over its queries of |C|.
 * n_borderline (optional, int64[n_pairs]) receives the number of (query,
 * candidate) slots of each pair whose FP32 distance lay within
 * recheck_margin_px of d and was decided again in FP64.
 * With emit_all, all_match/all_d1/all_d2/all_count (int32[sum n_a], pair-major,
 * query order) receive every query's match (-1 if no candidate), D1, D2
 * (INT32_MAX if absent) and |C|. */
typedef struct {
  int32_t* query;
  int32_t* match;
  int32_t* d1;
  int32_t* d2;
  int64_t capacity;
  int64_t* offset;          /* int64[n_pairs + 1] */
  int64_t* n_comparisons;   /* optional */
  int32_t* all_match;       /* optional, emit_all */
  int32_t* all_d1;
  int32_t* all_d2;
  int32_t* all_count;
  int64_t* n_borderline;    /* optional */
} sfm_matches;

/* Create a context on HIP device `device`.  workspace_budget_bytes caps the
 * device workspace (0 = 8 GiB).  Returns SFM_EINVAL for a bad device. */
int sfm_create(sfm_ctx** ctx, int32_t device, size_t workspace_budget_bytes);

/* Stop the server if running, free the context and everything it owns. */
int sfm_destroy(sfm_ctx* ctx);

/* Register the images that pairs refer to by index (replaces any previous
 * set).  Checks that every descriptor byte is <= 127 (SFM_EINVAL otherwise),
 * precomputes squared norms and keypoint bounding boxes.  Blocks until done.
 * The caller's buffers must stay valid while the registration is in use. */
int sfm_register_images(sfm_ctx* ctx, const sfm_image* images, int32_t n_images);

/* Device workspace bytes that guided matching of these pairs needs (the
 * batched, plain and no-alloc forms).  Exhaustive matching needs, on top,
 * 8 bytes per query per 1,024 targets of b and 8 bytes per work item of
 * 256 queries x 1,024 targets. */
int sfm_workspace_size(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, size_t* bytes);

/* Batched guided matching (Section 6.2, Appendix A steps 1-4), every pair in
 * one sequence of launches: per-pair geometry, binning of b along the
 * epipolar pencil, query lines and tiles, the fused band test + int8-MFMA
 * distance + two-nearest kernel, ordered emission.
 * pairs: host sfm_pair[n_pairs]; F: host double[9*n_pairs], row-major,
 * x_b^T F x_a = 0, finite and not all zero; opt may be NULL (defaults).
 * SFM_EINVAL: bad index, band, F or options; SFM_ECAPACITY: out->capacity or
 * the workspace budget is too small. */
int sfm_guided_match(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
                     const sfm_options* opt, const sfm_matches* out, void* stream);

/* Same result as sfm_guided_match, computed one pair per launch sequence
 * (the plain per-pair form the batched form is measured against). */
int sfm_guided_match_plain(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs,
                           const double* F, const sfm_options* opt, const sfm_matches* out,
                           void* stream);

/* Limits of sfm_guided_match_noalloc. */
#define SFM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
#define SFM_NOALLOC_MAX_PAIRS 8192

/* For callers that cannot allocate memory while they run (tight serving
 * loops, harnesses that forbid allocation): sfm_guided_match with the same
 * arguments and bit-identical outputs, computed without any device, pinned
 * or heap allocation in the call.  Its workspace is a fixed device array of
 * SFM_NOALLOC_SCRATCH_BYTES per GPU, loaded with the library's device code
 * and held until the process ends; sfm_create looks up its address once per
 * device.  Pair table, F and binning order go through a fixed host buffer.
 * Limits: at most SFM_NOALLOC_MAX_PAIRS pairs, and a workspace
 * (sfm_workspace_size) of at most SFM_NOALLOC_SCRATCH_BYTES; beyond either
 * the call returns SFM_ECAPACITY and enqueues nothing.
 * Sharing: every context on a GPU uses that GPU's one array, which keeps the
 * last call's contents (nothing of it is read before it is rewritten).  The
 * library orders the calls of this entry point on one GPU: each call's
 * kernels wait for the previous call's, so calls from different streams or
 * contexts run one after another; work that escapes that order (a replay of
 * a captured call) would race with any other call on the GPU and is not
 * supported.  The call waits on the host for the previous call's staging
 * copy to finish.  sfm_last_stats reports nothing after this call.
 * Errors: as sfm_guided_match, and SFM_EINVAL on a device index >= 64. */
int sfm_guided_match_noalloc(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs,
                             const double* F, const sfm_options* opt, const sfm_matches* out,
                             void* stream);

/* Exhaustive matching: every feature of b is a candidate of every query
 * (band and F ignored; F may be NULL).  Same outputs; equals guided matching
 * with band_px = +inf on queries whose line is not degenerate.  n_borderline
 * is 0.  Errors: as sfm_guided_match, and SFM_ECAPACITY for an image of more
 * than 8,388,352 queries or 67,107,840 targets in a pair. */
int sfm_bruteforce_match(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
                         const sfm_options* opt, const sfm_matches* out, void* stream);

/* Accuracy of the FP32 band test (eqs. 2-3).  Runs the batched form's
 * preparation for these pairs and then, over every (query, candidate) slot
 * that the match kernel evaluates (every candidate range of every query
 * tile), compares the FP32 distance the kernel computes with the FP64
 * distance of the definition (the caller's F, the original keypoints, no
 * contraction).  Writes to host memory the largest |FP32 - FP64| in pixels
 * over the slots whose FP64 distance is at most 2 band_px (*max_err_px, 0
 * if there are none) and their number (*n_slots).  Host-synchronous; uses
 * the context's workspace like a matching call.  SFM_EINVAL: as
 * sfm_guided_match, or a NULL output pointer. */
int sfm_band_error(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
                   double* max_err_px, int64_t* n_slots, void* stream);

/* Grid-based approximate candidate search (Section 6.2.1, eqs. 4-9; the
 * paper's own search, kept as an alternative to the exact band).  band_px of
 * each pair is the cell parameter d > 0 (finite): b's features are binned
 * into four grids of 2d x 2d cells shifted by (0,0), (d,0), (0,d), (d,d); the
 * query's line (x_b^T F x_a = 0) is cut by the bounding box of b's keypoints
 * at A (first crossing on the edges x = min, x = max, y = min, y = max) and B
 * (the crossing farthest from A); K + 1 points p_k = (k A + (K - k) B) / K,
 * K the smallest integer with K d >= |AB|, each select the centre-most of the
 * four cells holding them (lower grid on ties); C' is the set of features in
 * the selected cells.  The two nearest of C' and the ratio test of `opt`
 * decide the match; outputs as sfm_guided_match (n_comparisons = sum of
 * |C'|).  C' approximates the band: it may include features up to 2d from
 * the line's sample points and miss band members near cell corners.
 * Limits: n_b <= 65536 per pair; at most 2^22 cells per grid (SFM_ECAPACITY);
 * a query (with grouping, a group) whose C' exceeds 1024 features raises
 * the device error flag (SFM_EKERNEL at sfm_sync) and keeps the first 1024
 * found.
 * SFM_EINVAL: bad index, d, F or options. */
int sfm_grid_match(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
                   const sfm_options* opt, const sfm_matches* out, void* stream);

/* Query grouping for sfm_grid_match (Section 6.2.2, App. A step 2); px = 0
 * (the default) turns it off, px = 2 is the paper's setting.  With grouping,
 * the queries of each pair are sorted by their line's crossings with b's box
 * (A.x, A.y, B.x, B.y, then query index; lines without a crossing last), a
 * new group starts where A or B lies more than px from the previous line's
 * (to_leader = 0, App. A's stencil) or from the group's first line's
 * (to_leader = 1), or where either line has no crossing; every query of a
 * group takes the C' of the group's first line.  A grouped call is
 * host-synchronous: the host reads the group count before the last launch.
 * sfm_grid_groups reports the groups of the last grouped call.  Pairs, F and
 * the outputs are as for sfm_grid_match.  SFM_EINVAL: px negative or not
 * finite. */
int sfm_set_grid_grouping(sfm_ctx* ctx, double px, int32_t to_leader);
int sfm_grid_groups(sfm_ctx* ctx, int64_t* n_groups);

/* Staged matching of coarse features (Section 4, the hybrid scheme modelled
 * on preemptive matching).  Each registered image must list its features in
 * decreasing scale, so that a prefix is its highest-scale part.  For a pair
 * (a, b) with n_a, n_b features:
 *   - if n_a or n_b is below cfg.small_image, all features of a are matched
 *     against all of b in one stage;
 *   - otherwise stage 1 matches the first q = ceil(n_a * query_pct / 100)
 *     features of a against the first r = ceil(n_b * target_pct / 100) of b;
 *     stage 2 matches the next min(q, n_a - q) features of a against the same
 *     r, and runs only when stage 1 accepted more than cfg.min_matches and,
 *     with cfg.enough > 0, fewer than cfg.enough (enough matches for the
 *     geometry: the pair stops early).
 * Every stage is exhaustive 2-NN matching with the ratio test of `opt`
 * (band_px of the pairs is ignored; emit_all must be 0).  Rows of a pair are
 * its stage-1 rows then its stage-2 rows, in ascending query index of a (the
 * registered indexing); n_comparisons sums both stages.  out->capacity must
 * be >= the sum over pairs of the queries their stages take (sum of n_a
 * always suffices).  stages (optional, host int32[n_pairs]) receives 0 for a
 * pair matched whole, 1 when only stage 1 ran, 2 when both ran.
 * Host-synchronous: the host reads stage 1's counts to choose the stage-2
 * pairs, and the call returns once `out` is written.  Default cfg (NULL):
 * query_pct 10, target_pct 20, min_matches 4, enough 0, small_image 1000.
 * SFM_EINVAL: bad index, cfg or options; SFM_ECAPACITY: out->capacity or the
 * workspace budget is too small; SFM_EKERNEL: a device error flag. */
typedef struct {
  int32_t query_pct;     /* 10 */
  int32_t target_pct;    /* 20 */
  int32_t min_matches;   /* 4 */
  int32_t enough;        /* 0: no early stop */
  int32_t small_image;   /* 1000 */
  int32_t pad;
} sfm_preemptive_cfg;
int sfm_preemptive_match(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs,
                         const sfm_preemptive_cfg* cfg, const sfm_options* opt,
                         const sfm_matches* out, int32_t* stages, void* stream);

/* Wait for the context's work on `stream`, then report a device error flag
 * raised since the last sfm_sync (SFM_EKERNEL) or a HIP error (SFM_EHIP). */
int sfm_sync(sfm_ctx* ctx, void* stream);

/* Phase timing.  While enabled, every matching call records HIP events on its
 * stream around its three phases: preparation (geometry, binning, query
 * tiles), the match kernel, and emission (one record per pair in the plain
 * form).  sfm_phase_times() waits for the recorded calls, writes the summed
 * milliseconds of each phase to ms[0..2] and the number of records to
 * *n_records, and clears the records. */
int sfm_set_profiling(sfm_ctx* ctx, int32_t enable);
int sfm_phase_times(sfm_ctx* ctx, double ms[3], int64_t* n_records);

/* Totals of the last matching call, summed over its pairs (waits for it):
 * out[0] candidate comparisons (sum of |C|), out[1] (query, candidate) slots
 * the match kernel evaluated (superset ranges padded to whole MFMA blocks, so
 * out[0] / out[1] is the fraction of useful work), out[2] chunks that took the
 * exact tie-break pass, out[3] accepted matches, out[4] slots decided in FP64
 * (the sum of n_borderline). */
int sfm_last_stats(sfm_ctx* ctx, int64_t out[5]);

/* ---------------------------------------------------------------------------
 * Serving loop.  Single-pair requests (the image pairs that Section 6.1
 * selects, arriving one at a time) are batched on the fly: a worker thread
 * concatenates the waiting requests into one sfm_guided_match launch on the
 * server's own stream whenever one of max_inflight result slots is free, and
 * a completion thread copies each request's accepted matches into pinned host
 * memory.  Latency = done_ns - arrival_ns, on the sfm_server_now_ns() clock.
 * One server per context; while it runs, other calls on the context still
 * work (calls on a context are ordered through its workspace). */
typedef struct {
  int32_t max_batch_pairs;     /* requests per launch (default 256) */
  int32_t max_inflight;        /* launches whose results are outstanding, 1..8 (default 2) */
  int64_t max_batch_queries;   /* cap on the summed n_a of one launch (default 2^22);
                                  a single larger request fails with SFM_ECAPACITY */
  sfm_options opt;             /* emit_all must be 0 */
} sfm_server_cfg;
/* Admission: a launch takes waiting requests in arrival order while it stays
 * within max_batch_pairs and max_batch_queries and its workspace (an upper
 * bound from the pairs' feature counts) within the context's workspace budget
 * (sfm_create); the next request waits for the next launch.  A request whose
 * workspace alone exceeds the budget fails with SFM_ECAPACITY. */

typedef struct {
  int32_t* query;              /* host, caller-owned, capacity rows: accepted matches */
  int32_t* match;              /* in ascending query order, as in sfm_matches */
  int32_t* d1;
  int32_t* d2;
  int64_t capacity;
  int64_t n_matches;           /* out */
  int64_t n_comparisons;       /* out: candidate comparisons of the request */
  int64_t arrival_ns;          /* out: the request's arrival time */
  int64_t done_ns;             /* out: when its rows were in host memory */
  int32_t status;              /* out: SFM_OK or the error of its launch */
  int32_t pad;
} sfm_result_view;

/* Monotonic clock of the server, nanoseconds (CLOCK_MONOTONIC). */
int64_t sfm_server_now_ns(void);

/* Start the serving threads (cfg may be NULL for defaults).  Allocates the
 * result slots: per slot four int32 device and pinned host arrays of
 * max_batch_queries rows.  SFM_EBUSY if a server already runs on ctx. */
int sfm_server_start(sfm_ctx* ctx, const sfm_server_cfg* cfg);

/* Queue one pair (host sfm_pair and double F[9], read before returning).
 * arrival_ns is the request's arrival time (<= 0: now).  Checks the image
 * indices, band and F (SFM_EINVAL); SFM_EBUSY if no server runs.  *ticket
 * identifies the request for sfm_server_poll. */
int sfm_server_submit(sfm_ctx* ctx, const sfm_pair* pair, const double* F, int64_t arrival_ns,
                      uint64_t* ticket);

/* Submit n requests at once (a burst that the visibility filter emits
 * together): pairs[0..n) with F (host, n * 9 doubles, as in
 * sfm_guided_match), all arriving at arrival_ns (<= 0: now).  Every request
 * is checked first; if any is invalid nothing is queued and SFM_EINVAL is
 * returned.  Otherwise all n enter the queue together, in order, and
 * tickets[k] (host, n entries, caller-owned) identifies pairs[k].  n = 0 is a
 * no-op. */
int sfm_server_submit_batch(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n, const double* F,
                            int64_t arrival_ns, uint64_t* tickets);

/* Collect a request's result into *out, waiting up to timeout_ms
 * (0: do not wait, < 0: wait for ever).  SFM_ETIMEOUT: not ready yet;
 * SFM_ENOTFOUND: unknown or already collected ticket; SFM_ECAPACITY: out
 * cannot hold its n_matches rows (out->n_matches says how many; the result
 * stays collectable); SFM_EBUSY: no server runs, or it was stopped while this
 * call waited.  A collected result is released.  Polls, submissions and a
 * stop may run on different threads at once. */
int sfm_server_poll(sfm_ctx* ctx, uint64_t ticket, sfm_result_view* out, int32_t timeout_ms);

/* out[0] launches so far, out[1] requests launched, out[2] requests waiting. */
int sfm_server_stats(sfm_ctx* ctx, int64_t out[3]);

/* Launch every waiting request, wait for all results, stop the threads and
 * free the slots.  Uncollected results are dropped. */
int sfm_server_stop(sfm_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Tuning.  Two parameters of the batched form trade evaluated slots against
 * scheduling and preparation costs (Appendix A steps 1-2 leave them open):
 *   group_tiles       query tiles of 16 queries (in pencil order) that one
 *                     match workgroup of four waves streams one candidate
 *                     range for: 4 or 8 (default 8);
 *   features_per_bin  average target features per bin of b's pencil
 *                     binning, 1..1024 (default 8).
 * Results do not depend on them.  They apply to later calls on the context. */
int sfm_set_tuning(sfm_ctx* ctx, int32_t group_tiles, int32_t features_per_bin);
int sfm_get_tuning(sfm_ctx* ctx, int32_t* group_tiles, int32_t* features_per_bin);

/* Graph replay of the batched form (enable != 0; off by default).  With it
 * on, a call whose launch layout (pairs, feature counts, workspace, outputs,
 * options and tuning) equals the previous batched call's has the kernels
 * captured into a HIP graph, which later calls with the same layout replay; a
 * layout seen for the first time is launched directly, so callers whose
 * batches change every call pay no capture.  The copy of the pairs and F into
 * the workspace stays a stream copy.  Results are identical to stream
 * launches.  Measured on MI355X, replay is no faster than launching the
 * kernels on the stream (the 500-pair batch: 0.667 vs 0.660 ms; one 16k pair:
 * 0.132 vs 0.127 ms) and a capture costs a few milliseconds, hence off by
 * default.  Disabling frees the graph.  Profiling (sfm_set_profiling) uses
 * stream launches. */
int sfm_set_graph_replay(sfm_ctx* ctx, int32_t enable);

/* ---------------------------------------------------------------------------
 * Candidate images (Section 6.1): which image pairs to match.  The covisible
 * points of images i and j are the coarse-model points both observe; image
 * q's candidates are the images sharing more than `threshold` points with it
 * (the paper's T = 8), ranked by that count (ties: lower index), at most
 * top_k of them (the paper keeps about 10% of the images).  The unique
 * unordered pairs over all queries are the pairs to match.
 *
 * Input (device, caller-owned): the points each image observes, as CSR:
 * image i observes vis_pts[vis_off[i] .. vis_off[i + 1]), point ids in
 * 0..n_points-1, each at most once per image; nnz = vis_off[n_images].
 * n_images <= 4096 (one row of counts lives in LDS).  A point id out of
 * range, or ranges inconsistent with nnz, raise the device error flag
 * (SFM_EKERNEL at sfm_sync); the outputs are then unspecified.
 * Outputs (device, caller-owned), per image q in rank order:
 * cand[q * top_k + r] and n_shared[q * top_k + r] for r < n_cand[q], -1 and 0
 * after.  If pairs is not NULL, the unique pairs (i, j), i < j, ascending, go
 * to pairs[2 p], pairs[2 p + 1] (room for n_images * top_k pairs) and their
 * number to *n_pairs.  Asynchronous on `stream`; uses the context's workspace
 * (about 4 (3 n_points + nnz) bytes and a bit per image pair; see
 * sfm_set_covis_method for the other method). */
typedef struct {
  int32_t* cand;        /* n_images * top_k */
  int32_t* n_shared;    /* n_images * top_k */
  int32_t* n_cand;      /* n_images */
  int32_t* pairs;       /* optional: 2 * n_images * top_k */
  int64_t* n_pairs;     /* 1; needed with pairs */
} sfm_candidates;
int sfm_candidate_images(sfm_ctx* ctx, const int32_t* vis_off, const int32_t* vis_pts,
                         int64_t nnz, int32_t n_images, int32_t n_points, int32_t threshold,
                         int32_t top_k, const sfm_candidates* out, void* stream);

/* How sfm_candidate_images counts covisible points (the results are the
 * same): 1 = a histogram of every image's co-observers (work grows with the
 * sum over points of their observers squared: short tracks), 2 = a bit matrix
 * of images x points and popcounts of row ANDs (work grows with images^2 x
 * points / 32: dense visibility), 0 = choose from nnz, n_images and n_points
 * (default).  Method 2 also needs n_images * (n_points / 8 + 4 n_images)
 * bytes of workspace. */
int sfm_set_covis_method(sfm_ctx* ctx, int32_t method);

/* ---------------------------------------------------------------------------
 * Track merging and triangulation (Section 6.3).
 *
 * sfm_tracks: the tracks are the connected components of the match graph,
 * whose nodes are observations (a feature of an image; the caller numbers
 * them 0..n_nodes-1, e.g. an image's first node plus the feature index) and
 * whose edges are accepted matches: edges[2 k], edges[2 k + 1] (device,
 * n_edges pairs of node ids).  label[i] (device, n_nodes, caller-owned)
 * receives the smallest node id of i's component, whatever the order of the
 * edges.  A node id out of range raises the device error flag (SFM_EKERNEL at
 * sfm_sync).  No workspace.  Asynchronous on `stream`.
 *
 * sfm_triangulate: for every track root r (label[r] == r), the least-squares
 * point of its observations: node i was seen at node_xy[2 i], node_xy[2 i + 1]
 * (pixels) in image node_image[i], whose camera is the row-major 3 x 4 matrix
 * P[12 image ..] (x ~ P (X, 1)); each observation gives the two linear
 * equations (x p3 - p1).(X, 1) = 0, (y p3 - p2).(X, 1) = 0, solved by the
 * FP64 normal equations.  X[3 r ..] (device, 3 n_nodes doubles) receives the
 * point, NaN for tracks of one observation or a singular system;
 * n_obs[r] its number of observations, 0 for non-roots.  Uses 16 n_nodes
 * bytes of workspace (per-track member lists) plus a scan's storage.  A
 * label or image index out of range raises the device error flag.
 * Asynchronous on `stream`. */
int sfm_tracks(sfm_ctx* ctx, int64_t n_nodes, const int32_t* edges, int64_t n_edges,
               int32_t* label, void* stream);
int sfm_triangulate(sfm_ctx* ctx, int64_t n_nodes, const int32_t* label, const int32_t* node_image,
                    const float* node_xy, const double* P, int32_t n_images, double* X,
                    int32_t* n_obs, void* stream);

/* Time the batched form on the given batch for every group_tiles in
 * {4, 8} and features_per_bin in {4, 8, 16} (one warm-up and `repeats`
 * timed calls each, HIP events on `stream`), keep the fastest setting on the
 * context, and write the mean milliseconds per call to ms_out[3 * i + j]
 * (i over group_tiles, j over features_per_bin; ms_out may be NULL).  Uses
 * scratch outputs it allocates and frees; blocks until done. */
int sfm_autotune(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
                 const sfm_options* opt, void* stream, int32_t repeats, double* ms_out);

/* sfm_autotune with a persisted result.  cache_path names a JSON file of
 * tunings keyed by the device (architecture and CU count) and the batch's
 * shape (log2 buckets of its total queries and of its mean target count, its
 * mean band in half-octaves).  When the key is present the stored tuning is
 * set on the context and *from_cache is 1 (ms_out untouched); otherwise the
 * batch is tuned as sfm_autotune does, the winner is added to the file
 * (created if missing) and *from_cache is 0.  SFM_EINVAL: as sfm_autotune,
 * no pairs, NULL cache_path or from_cache, or a file that cannot be
 * written. */
int sfm_autotune_cached(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
                        const sfm_options* opt, void* stream, int32_t repeats,
                        const char* cache_path, double* ms_out, int32_t* from_cache);

/* Human-readable name of a status code (static string). */
const char* sfm_strerror(int status);

/* Copy the last error message of this context into buf (NUL-terminated). */
int sfm_last_error(sfm_ctx* ctx, char* buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* SFM_GM_H */
