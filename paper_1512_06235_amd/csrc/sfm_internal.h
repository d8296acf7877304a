// Internal layouts shared by the host driver and the HIP kernels of libsfmgm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfm_gm.h"

namespace sfm {

constexpr int kDescBytes = 128;
constexpr int kQueryTile = 16;          // queries per tile (MFMA N); also candidates per MFMA step
constexpr int kMatchWaves = 4;          // waves per match workgroup
constexpr int kXcds = 8;                // XCDs of the GPU (each with its own L2): schedule shares
constexpr int kMaxGroupTiles = 8;       // query tiles sharing one candidate stream, at most
constexpr int kDefaultGroupTiles = 8;   // the default (4 or 8: one or two tiles per wave)
constexpr int kDefaultFeaturesPerBin = 8;
constexpr int kCandPad = 16;            // padding positions after each pair's candidates
constexpr int kChunk = 1024;            // candidate positions one key encodes
constexpr int kPosBits = 10;            // log2(kChunk)
constexpr uint32_t kKeyInf = 0xFFFFFFFFu;
constexpr int32_t kDistInf = 0x7FFFFFFF;
constexpr uint32_t kDistBias = 1u << 21;  // makes norm2(c) - 2 q.c >= 0
constexpr int kMaxBins = 8192;          // LDS histogram size per pair
constexpr double kBandSlackPx = 1e-2;   // bin windows widen the band by this
constexpr int32_t kGroupStartCost = 48;  // schedule cost of starting a tile group
constexpr int32_t kSegCost = 4;          // schedule cost of streaming one 64-position segment
constexpr int32_t kStepCost = 2;         // schedule cost of one 16 x 16 step of one tile

// Per image, built at registration.
struct ImageDev {
  const float* xy;          // float2[n]
  const uint8_t* desc;      // uint8[n][128]
  const int32_t* norm2;     // int32[n], owned by the context
  int32_t n;
  int32_t pad;
  float bbox[4];            // min x, min y, max x, max y of the keypoints
};

// Per pair, filled on the host: sizes and workspace offsets.
struct PairDesc {
  int32_t a, b;
  int32_t na, nb;
  int32_t nbins;            // bins of b (full-scan mode uses bin 0 only)
  int32_t nblocks;          // ceil(na / kQueryTile)
  int64_t q_off;            // into per-query arrays (prefix of na)
  int64_t c_off;            // into per-candidate arrays (prefix of nb + kCandPad)
  int64_t bin_off;          // into bin arrays (prefix of nbins + 1)
  int64_t blk_off;          // into per-block arrays and the work-item space
  int64_t grp_off;          // into the tile-group table
  int32_t ngroups;          // ceil(nblocks / group tiles)
  int32_t pad2;
  double band;              // d, pixels (may be +inf)
  int32_t ignore_band;      // exhaustive matching
  int32_t pad;
  int64_t ex_off;           // exhaustive matching: first partial result (prefix of n_a * slices)
};

enum GeomMode : int32_t {
  kModeFullScan = 0,        // every query scans all of b
  kModePencil = 1,          // finite epipole: key = S * tan(angle about e)
  kModeParallel = 2,        // epipole at infinity: key = offset across lines
};

// Per pair, written by the geometry kernel (a1).
struct PairGeom {
  double F[9];              // F / ||F||_F
  double ex, ey;            // finite epipole in b (pencil mode)
  double ux, uy;            // frame: u along the pencil centre line, n = (-uy, ux)
  double ox, oy;            // origin of the FP32 centred coordinates
  double S;                 // key scale (min distance along u, pencil mode)
  double kmin, kmax;        // key range of b's bounding box
  double inv_delta;         // nbins / (kmax - kmin)
  double rbox;              // max distance of a bbox corner from the origin
  double half_width;        // d + slack, pixels
  float band_lo, band_hi;   // d - margin and d + margin in FP32 (+inf allowed)
  int32_t mode;
  int32_t nbins;
};

// Targets in binned order are kept as four arrays (x, y, key word, index),
// each with kCandPad positions after every pair's n_b: the padding has a NaN
// x (no band test passes) and index 0.
//   x, y   centred FP32 coordinates
//   nc     ((norm2 + kDistBias) << kPosBits) | (position & (kChunk - 1))
//   j      original index in b

// One query in tile order (16 bytes): normalised line on centred coordinates.
struct QueryRec {
  float a, b, c;
  int32_t i;                // original index in a
};

// Per-query result in original query order (16 bytes).  The match kernel
// writes the binned position of the match in `match`; emission turns it into
// the index in b (BatchView::cand_j set), other producers write the index.
struct QueryResult {
  int32_t match;            // -1 if no candidate
  int32_t d1, d2;           // kDistInf if absent
  int32_t flags;            // bit 0 accept; count << 1 when counts are kept
};

struct PairCounters {
  unsigned long long comparisons;
  unsigned long long elements;   // (query, candidate) slots evaluated, padding included
  unsigned long long borderline; // slots whose FP32 distance lay within the margin of d
  uint32_t accepted;
  uint32_t ties;            // chunks that needed the tie-break pass
};

// Up to kMaxGroupTiles consecutive query tiles of one pair and the union of
// their candidate ranges; one workgroup streams the union through LDS.  The
// record holds everything the match kernel needs about the pair (176 bytes,
// read with scalar loads).
struct TileGroup {
  int32_t pair, tile0, ntiles, na;  // na: queries of the pair
  int32_t s_begin, s_end;   // union candidate range (s_begin >= s_end: empty)
  float band_lo, band_hi;   // FP32 |e| <= band_lo: in; > band_hi: out; else FP64 decides
  int64_t q_off, c_off;     // the pair's query and candidate offsets
  const uint8_t* a_desc;
  const uint8_t* b_desc;
  const int32_t* a_norm;
  const float* a_xy;        // keypoints of a and b (FP64 decisions)
  const float* b_xy;
  double band;              // d
  int32_t nb, pad[3];       // targets of the pair
  int32_t t_begin[kMaxGroupTiles], t_end[kMaxGroupTiles];   // per tile candidate range
};
static_assert(sizeof(TileGroup) == 176, "TileGroup is read as eleven 16-byte words");

// Everything a batch launch needs, passed by value.
struct BatchView {
  const ImageDev* images;
  const PairDesc* pairs;
  PairGeom* geom;
  float* cand_x;            // binned targets (see above), sum of (n_b + kCandPad)
  float* cand_y;
  uint32_t* cand_nc;
  int32_t* cand_j;
  int32_t* bin_start;       // nbins + 1 per pair
  QueryRec* qrec;
  int2* twin;               // per query tile: first, last bin of its queries (first > last: none)
  TileGroup* groups;
  int32_t* gcost;           // per tile group: estimated cost of matching it
  long long* pcost;         // per pair: the sum of its groups' costs
  int32_t* wg_start;        // share x (one per XCD) holds groups [wg_start[x], wg_start[x + 1])
  QueryResult* res;
  PairCounters* counters;
  const double* F;          // 9 per pair
  int32_t* err;             // device error flag
  int32_t n_pairs;
  int32_t total_blocks;
  int32_t ratio_num, ratio_den;
  int32_t accept_single;
  int32_t keep_counts;
  int32_t group_tiles;      // tiles per group (4 or 8: one or two per match wave)
  int32_t max_na;           // most queries of one pair (sizes the emission grid)
  int32_t max_nb;           // most targets of one pair (sizes the gather grid)
  int32_t pad_nb;
  double margin;            // FP64 re-decision margin around d, pixels (0 = FP32 only)
};

}  // namespace sfm

struct sfm_ctx;

namespace sfm {

// Context accessors for the serving loop, and its teardown (called by
// sfm_destroy before the context goes away).
int32_t ctx_device(const sfm_ctx* ctx);
int32_t ctx_n_images(const sfm_ctx* ctx);
int32_t ctx_image_size(const sfm_ctx* ctx, int32_t image);
// Candidate images from covisibility (kernels_covis.hip).  One query image's
// row of covisible counts and its sort keys live in LDS: at most this many
// images per call.
constexpr int kMaxCovisImages = 4096;
struct CovisArgs {
  const int32_t* vis_off;   // points of image i: vis_pts[vis_off[i] .. vis_off[i + 1])
  const int32_t* vis_pts;
  int64_t nnz;
  int32_t n_images, n_points, threshold, top_k;
  // Workspace: observers per point (counts, offsets, cursors, image ids),
  // scan block sums, pair bits and per-row pair counts and offsets.
  int32_t *pt_count, *pt_off, *cursor, *pt_imgs, *sums, *row_count, *row_off;
  uint32_t* bits;
  // Bit-matrix path (when gram is not NULL): image bitsets, n x n counts.
  uint32_t* bitset;
  int32_t* gram;
  // Outputs.
  int32_t *cand, *n_shared, *n_cand, *pairs;
  int64_t* n_pairs;
  int32_t* err;
};
hipError_t launch_candidates(const CovisArgs& a, hipStream_t st);

// Device-wide prefix sums of int32 (kernels_scan.hip): out[i] = sum of in[0..i)
// (exclusive) or in[0..i] (inclusive), in place allowed; `copy` (may be NULL)
// receives the same values.  sums: scan_temp_bytes(n) bytes of scratch.
// hipErrorInvalidValue for n > scan_limit().
int64_t scan_limit();
size_t scan_temp_bytes(int64_t n);
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, bool inclusive,
                       int32_t* sums, int32_t* copy, hipStream_t st);

// Tracks and triangulation (kernels_tracks.hip).
hipError_t launch_tracks(int64_t n_nodes, const int32_t* edges, int64_t n_edges, int32_t* label,
                         int32_t* err, hipStream_t st);
// ws: 4 n_nodes int32 (counts, starts, fill cursors, member lists); temp:
// the scan's storage (triangulate_temp_bytes).
hipError_t triangulate_temp_bytes(int64_t n_nodes, size_t* bytes);
hipError_t launch_triangulate(int64_t n_nodes, const int32_t* label, const int32_t* node_image,
                              const float* node_xy, const double* P, int32_t n_images,
                              int32_t* ws, void* temp, size_t temp_bytes, double* X,
                              int32_t* n_obs, int32_t* err, hipStream_t st);

// Grid-based approximate candidate search (kernels_grid.hip).
constexpr int32_t kGridMaxTargets = 65536;            // features of b (one LDS bit each)
constexpr int32_t kGridMaxCand = 1024;                // |C'| per query (LDS slots)
constexpr int32_t kGridQueriesPerBlock = 16;          // queries one workgroup takes in turn
constexpr int64_t kGridMaxCells = int64_t(1) << 22;   // cells of one grid of one pair

// Per pair, filled on the host: the four grids over b's keypoint box.
struct GridPair {
  int32_t a, b, na, nb;
  int64_t q_off;            // into per-query results
  int64_t item_off;         // into the binned feature lists (4 nb per pair)
  int64_t cell_off[4];      // into the cell tables (cells + 1 per grid)
  int32_t cx0[4], cy0[4];   // first cell of each grid
  int32_t ncx[4], ncy[4];   // cells of each grid
  double d;                 // cell parameter: cells are 2d x 2d, grids shifted by d
  double box[4];            // min x, min y, max x, max y of b's keypoints
};

struct GridView {
  const ImageDev* images;
  const GridPair* pairs;
  const double* F;          // 9 per pair, as given
  int32_t* cell_start;      // per grid: cells + 1 starts
  int32_t* cursor;          // per grid: counts, then fill positions
  int32_t* items;           // feature indices of b ordered by cell, per grid
  const int2* blocks;       // per query workgroup: (pair, first query)
  QueryResult* res;
  PairCounters* counters;
  int32_t* err;
  int32_t n_pairs;
  int32_t ratio_num, ratio_den;
  int32_t accept_single;
  int32_t keep_counts;
  int32_t bitmap_words;     // ceil(largest n_b of the call / 32)
  int32_t lds_cells;        // cell counts the binning keeps in LDS (larger grids use HBM)
};
constexpr int32_t kGridLdsCells = 15360;              // 60 KB of LDS counts (64 KB with the scan)
// Bins b's features into the four grids of every pair, then finds C', the
// two nearest candidates and the ratio test for every query (n_blocks
// entries of the block table; 0 = binning only).
hipError_t launch_grid(const GridView& v, int64_t n_blocks, hipStream_t st);

// Query grouping (Section 6.2.2): buffers over the n query positions of a
// call (position = the pair's first query + query index).
struct GroupView {
  double* cross;                 // 4 per position: A.x, A.y, B.x, B.y
  int32_t* hit;                  // 1 if the line crosses b's box
  int32_t* val[2];               // positions in sorted order, ping-pong (result in val[0])
  const int32_t* seg_begin;      // per pair: first position
  const int32_t* seg_end;        // per pair: one past the last
  int32_t* stencil;              // 1 where a group starts
  int32_t* gid;                  // inclusive scan of the stencil
  int32_t* gstart;               // per group: its first sorted position
  void* temp;                    // radix-sort counts and scan sums (grid_group_temp_bytes)
  size_t temp_bytes;
  int32_t n;
  int32_t to_leader;             // compare with the group's first line, not the previous one
  double tol2;                   // squared grouping distance (px^2)
};
hipError_t grid_group_temp_bytes(int32_t n, int32_t n_pairs, size_t* bytes);
// Crossings, the lexicographic sort of (A.x, A.y, B.x, B.y) within each pair,
// the stencil, its scan and the group starts; gid[n - 1] is the group count.
hipError_t launch_grid_group_prepare(const GridView& v, const GroupView& g, hipStream_t st);
// One wave per group: C' of the group's first line, then every member's
// two nearest and ratio test.
hipError_t launch_grid_groups(const GridView& v, const GroupView& g, int32_t n_groups,
                              hipStream_t st);

// Staged (preemptive) matching (kernels_stage.hip).
// A view is a run of consecutive features of one registered image: spec holds
// (image, first feature, count) per view, checked on the host.
hipError_t launch_make_views(const ImageDev* images, const int32_t* spec, int32_t n_views,
                             ImageDev* views, hipStream_t st);
// Rows of one pair's two stages, placed one after the other at dst.
struct StageMerge {
  int64_t src1, src2, dst;
  int32_t n1, n2;
  int32_t shift;   // added to a second-stage query index (the first stage's query count)
  int32_t s2;      // the pair's index in the second stage, -1 if it had none
};
struct StageRows {
  const int32_t *q, *m, *d1, *d2;
  const int64_t* n_cmp;
};
hipError_t launch_merge_stages(const StageMerge* merge, int32_t n_pairs, StageRows one,
                               StageRows two, int32_t* out_q, int32_t* out_m, int32_t* out_d1,
                               int32_t* out_d2, int64_t* out_cmp, hipStream_t st);

// Workspace admission for the serving loop: an upper bound on the bytes one
// pair adds to a batched call's workspace, the bytes every call needs
// besides its pairs, and the context's workspace budget.
size_t ctx_request_bytes(const sfm_ctx* ctx, int32_t a, int32_t b);
size_t ctx_call_bytes(const sfm_ctx* ctx);
size_t ctx_budget(const sfm_ctx* ctx);
void server_release(sfm_ctx* ctx);
// A workspace of its own for one server slot (device workspace within
// `budget`, pinned staging, events): batched launches on different slots'
// spaces and streams overlap on the device.  serve_match is the batched form
// (sfm_guided_match) on that space; NULL from serve_space_create when HIP
// fails.
struct ServeSpace;
ServeSpace* serve_space_create(sfm_ctx* ctx, size_t budget);
void serve_space_destroy(ServeSpace* sp);
int serve_match(sfm_ctx* ctx, ServeSpace* sp, const sfm_pair* pairs, int32_t n_pairs,
                const double* F, const sfm_options* opt, const sfm_matches* out, hipStream_t st);

// Host launchers (one translation unit each).
hipError_t launch_register(const ImageDev* imgs_host, ImageDev* imgs_dev, int32_t n_images,
                           int32_t* norm2_all, const int64_t* norm_off, float* bbox_dev,
                           int32_t* bad_flag, hipStream_t st);
// Preparation of pairs [pair_begin, pair_begin + pair_count), whose tile groups
// are [grp_begin, grp_begin + grp_count), for `wgs` match workgroups (the
// groups are split into min(kXcds, wgs) shares of about equal cost, one per
// XCD).  `order` (device, may be NULL) lists the pairs in the order binning
// takes them; `max_queries` is the largest n_a among the pairs.
hipError_t launch_prepare(const BatchView& v, int32_t pair_begin, int32_t pair_count,
                          int32_t grp_begin, int32_t grp_count, int32_t wgs,
                          const int32_t* order, int32_t max_queries, hipStream_t st);
// Workgroups the match kernel uses for `groups` tile groups (one resident wave
// of workgroups at most).
int32_t match_workgroups(int32_t device, int32_t group_tiles, int64_t groups);
// Matches the groups of the last preparation with `wgs` workgroups.
hipError_t launch_match(const BatchView& v, int32_t wgs, hipStream_t st);
hipError_t launch_emit(const BatchView& v, int32_t pair_begin, int32_t pair_count,
                       int64_t* offset, int32_t* out_q, int32_t* out_m, int32_t* out_d1,
                       int32_t* out_d2, int64_t* n_cmp, int64_t* n_bl, int32_t* all_m,
                       int32_t* all_d1, int32_t* all_d2, int32_t* all_c, hipStream_t st);
// Exhaustive matching (kernels_exhaustive.hip), without preparation: work
// items of (pair, 256 queries, 1024 targets).  exhaustive_plan sets each
// pair's ex_off and, when `items` is not NULL, writes the item table (one
// int2 {pair, query block << 16 | slice} per item); n_part receives the
// partial results (uint2) the call needs.  launch_exhaustive resets the
// pairs' counters, matches every item and merges each query's slices into
// v.res (the index in b: emission runs with v.cand_j NULL).
constexpr int32_t kExhaustiveMaxQueries = 32767 * 256;   // query blocks fit 15 bits
constexpr int32_t kExhaustiveMaxTargets = 65535 * 1024;  // slices fit 16 bits
void exhaustive_plan(PairDesc* pd, int32_t n_pairs, int2* items, int64_t* n_items,
                     int64_t* n_part);
hipError_t launch_exhaustive(const BatchView& v, const int2* items, int64_t n_items, uint2* part,
                             hipStream_t st);
// Diagnostic after a preparation: out[0] receives (atomic max) the bits of
// the largest |FP32 - FP64| epipolar distance over the evaluated slots whose
// FP64 distance is at most 2d, out[1] (atomic add) their number.
hipError_t launch_band_error(const BatchView& v, int64_t n_groups, unsigned long long* out,
                             hipStream_t st);

}  // namespace sfm
