/*
 * CPU oracle for geometry-aware guided matching -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct reference of what the GPU library
 * computes.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never does.  It shares no
 * source, header or helper with the GPU library.
 *
 * Definition followed (Section 6.2 of the paper):
 *   eq. (1) context: F maps a query point of image a to its epipolar line in
 *           image b, l = F (x, y, 1)^T, with x_b^T F x_a = 0;
 *   eq. (2): the candidate set C = { p' in b : dist(p', l) <= d } (inclusive);
 *   eq. (3): dist(p', l) = |a x' + b y' + c| / sqrt(a^2 + b^2) (absolute value);
 *   Section 6.2.1 "linear search": every feature of b is tested against l;
 *   Section 6.2.2 / Appendix A step 4: the two nearest candidates by descriptor
 *           distance followed by the ratio test.
 * Readings of points the paper leaves open (all fixed here, identically in the
 * GPU library):
 *   - distance is the exact integer squared L2 over uint8 descriptors;
 *   - ratio test on distances r = 0.8 is ratio_den * D1 < ratio_num * D2 on
 *     squared distances (100 * D1 < 64 * D2), strict;
 *   - fewer than two candidates: rejected unless accept_single is set;
 *   - equal distances: the lowest index in b wins; a tie at the minimum makes
 *     D2 == D1, which the ratio test rejects;
 *   - a degenerate line (a = b = 0, or non-finite) has no candidates.
 */
#ifndef SFM_ORACLE_H
#define SFM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One image: host pointers. xy is float[2*n] (x, y), desc is uint8[128*n]. */
typedef struct {
  const float* xy;
  const uint8_t* desc;
  int32_t n;
} sfm_oracle_image;

/* Query image a is matched into target image b with band half-width band_px. */
typedef struct {
  int32_t a;
  int32_t b;
  double band_px;
} sfm_oracle_pair;

typedef struct {
  int32_t ratio_num;      /* 64 */
  int32_t ratio_den;      /* 100 */
  int32_t accept_single;  /* 0 */
  int32_t ignore_band;    /* 0; 1 = exhaustive matching (every feature of b) */
  double borderline_px;   /* 1e-3: |e - d| <= this counts as borderline */
} sfm_oracle_options;

/*
 * Per-query results, pair-major, each pair's queries in index order; the row
 * of query i of pair p is q_off[p] + i with q_off the exclusive prefix sum of
 * n_a over pairs.  All arrays are caller-owned host memory with that many
 * entries (or NULL to skip).
 *   match      J1, the lowest-index nearest candidate, or -1 when count == 0
 *   d1, d2     nearest / second-nearest squared distance (INT32_MAX if absent)
 *   count      number of candidates (features of b inside the band)
 *   borderline number of features of b with | e - d | <= borderline_px
 *   accept     1 if the query passes the ratio test
 * Per pair (n_pairs entries, or NULL): n_comparisons = sum of count,
 * n_borderline = sum of borderline, n_accepted = sum of accept.
 */
typedef struct {
  int32_t* match;
  int32_t* d1;
  int32_t* d2;
  int32_t* count;
  int32_t* borderline;
  uint8_t* accept;
  int64_t* n_comparisons;
  int64_t* n_borderline;
  int64_t* n_accepted;
} sfm_oracle_result;

/*
 * Match every pair.  F holds n_pairs row-major 3x3 matrices (double[9*n_pairs]).
 * n_threads <= 0 uses the hardware concurrency.  Returns 0 on success,
 * -1 on invalid arguments (bad image index, negative band, NULL pointers).
 */
int sfm_oracle_match(const sfm_oracle_image* images, int32_t n_images,
                     const sfm_oracle_pair* pairs, int32_t n_pairs,
                     const double* F, const sfm_oracle_options* opt,
                     sfm_oracle_result* out, int32_t n_threads);

/* Squared L2 distance of two 128-byte descriptors, as an exact integer. */
int32_t sfm_oracle_desc_dist(const uint8_t* p, const uint8_t* q);

/* Point-line distance of eq. (3) with the line F (x, y, 1)^T, in FP64. */
double sfm_oracle_epipolar_distance(const double* F, float xa, float ya, float xb, float yb);

/* Threads the last sfm_oracle_match call used. */
int32_t sfm_oracle_threads_used(void);

#ifdef __cplusplus
}
#endif
#endif
