// CPU oracle for geometry-aware guided matching -- TEST INFRASTRUCTURE ONLY.
// See sfm_oracle.h for the definition followed and the readings fixed.
//
// Built with -ffp-contract=off so every FP64 expression is evaluated exactly
// as written, left to right, with no fused multiply-add.
#include "sfm_oracle.h"

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstddef>
#include <thread>
#include <vector>

namespace {

std::atomic<int32_t> g_threads_used{0};

// Epipolar line l = F (x, y, 1)^T of a query point (Section 6.2), row by row.
void epipolar_line(const double* F, double x, double y, double* a, double* b, double* c) {
  *a = F[0] * x + F[1] * y + F[2];
  *b = F[3] * x + F[4] * y + F[5];
  *c = F[6] * x + F[7] * y + F[8];
}

// Exact integer squared L2 over 128 uint8 values (at most 128 * 127^2).
int32_t desc_dist(const uint8_t* p, const uint8_t* q) {
  int32_t s = 0;
  for (int k = 0; k < 128; ++k) {
    int32_t t = int32_t(p[k]) - int32_t(q[k]);
    s += t * t;
  }
  return s;
}

struct QueryResult {
  int32_t match = -1;
  int32_t d1 = INT32_MAX;
  int32_t d2 = INT32_MAX;
  int32_t count = 0;
  int32_t borderline = 0;
  uint8_t accept = 0;
};

// One query of one pair: linear search over every feature of b (Section 6.2.1),
// band test of eqs. (2)-(3), running two nearest (Section 6.2.2), ratio test.
QueryResult match_query(const sfm_oracle_image& A, const sfm_oracle_image& B, int32_t i,
                        const double* F, double d, const sfm_oracle_options& opt) {
  QueryResult r;
  const double xa = A.xy[2 * i];
  const double ya = A.xy[2 * i + 1];
  double a, b, c;
  epipolar_line(F, xa, ya, &a, &b, &c);
  const double s = std::sqrt(a * a + b * b);
  const bool line_ok = s > 0.0 && std::isfinite(s) && std::isfinite(c);
  if (!line_ok && !opt.ignore_band) return r;
  const uint8_t* q = A.desc + size_t(i) * 128;
  for (int32_t j = 0; j < B.n; ++j) {
    bool member;
    if (opt.ignore_band) {
      member = true;
    } else {
      const double xb = B.xy[2 * j];
      const double yb = B.xy[2 * j + 1];
      const double e = std::fabs(a * xb + b * yb + c) / s;
      member = e <= d;
      if (std::fabs(e - d) <= opt.borderline_px) r.borderline += 1;
    }
    if (!member) continue;
    r.count += 1;
    const int32_t D = desc_dist(q, B.desc + size_t(j) * 128);
    // j ascends, so a strict comparison keeps the lowest index among equal
    // distances; an equal distance still becomes the second-nearest value.
    if (D < r.d1) {
      r.d2 = r.d1;
      r.d1 = D;
      r.match = j;
    } else if (D < r.d2) {
      r.d2 = D;
    }
  }
  if (r.count >= 2) {
    r.accept = int64_t(opt.ratio_den) * r.d1 < int64_t(opt.ratio_num) * r.d2;
  } else if (r.count == 1) {
    r.accept = opt.accept_single != 0;
  }
  return r;
}

}  // namespace

extern "C" int32_t sfm_oracle_desc_dist(const uint8_t* p, const uint8_t* q) {
  return desc_dist(p, q);
}

extern "C" double sfm_oracle_epipolar_distance(const double* F, float xa, float ya, float xb,
                                               float yb) {
  double a, b, c;
  epipolar_line(F, xa, ya, &a, &b, &c);
  return std::fabs(a * double(xb) + b * double(yb) + c) / std::sqrt(a * a + b * b);
}

extern "C" int32_t sfm_oracle_threads_used(void) { return g_threads_used.load(); }

extern "C" int sfm_oracle_match(const sfm_oracle_image* images, int32_t n_images,
                                const sfm_oracle_pair* pairs, int32_t n_pairs,
                                const double* F, const sfm_oracle_options* opt,
                                sfm_oracle_result* out, int32_t n_threads) {
  if (n_pairs < 0 || n_images < 0 || (n_pairs > 0 && (!pairs || !F || !images)) || !opt || !out)
    return -1;
  if (opt->ratio_den <= 0 || opt->ratio_num < 0) return -1;
  std::vector<int64_t> q_off(size_t(n_pairs) + 1, 0);
  for (int32_t p = 0; p < n_pairs; ++p) {
    const sfm_oracle_pair& pr = pairs[p];
    if (pr.a < 0 || pr.a >= n_images || pr.b < 0 || pr.b >= n_images) return -1;
    if (!(pr.band_px >= 0.0)) return -1;  // also rejects NaN
    q_off[p + 1] = q_off[p] + images[pr.a].n;
  }

  // Work items: (pair, block of 256 queries), handed out by an atomic counter.
  struct Item { int32_t pair, begin, end; };
  std::vector<Item> items;
  for (int32_t p = 0; p < n_pairs; ++p) {
    const int32_t na = images[pairs[p].a].n;
    for (int32_t s = 0; s < na; s += 256) items.push_back({p, s, std::min(na, s + 256)});
  }
  std::vector<QueryResult> res(size_t(q_off[n_pairs]));
  std::atomic<size_t> next{0};
  auto worker = [&]() {
    for (;;) {
      const size_t k = next.fetch_add(1);
      if (k >= items.size()) break;
      const Item& it = items[k];
      const sfm_oracle_pair& pr = pairs[it.pair];
      for (int32_t i = it.begin; i < it.end; ++i)
        res[size_t(q_off[it.pair] + i)] =
            match_query(images[pr.a], images[pr.b], i, F + 9 * size_t(it.pair), pr.band_px, *opt);
    }
  };
  int32_t nt = n_threads > 0 ? n_threads : int32_t(std::thread::hardware_concurrency());
  if (nt < 1) nt = 1;
  if (size_t(nt) > items.size()) nt = int32_t(std::max<size_t>(1, items.size()));
  g_threads_used.store(nt);
  std::vector<std::thread> pool;
  for (int32_t t = 1; t < nt; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();

  for (int32_t p = 0; p < n_pairs; ++p) {
    int64_t cmp = 0, bl = 0, acc = 0;
    for (int64_t r = q_off[p]; r < q_off[p + 1]; ++r) {
      const QueryResult& q = res[size_t(r)];
      if (out->match) out->match[r] = q.match;
      if (out->d1) out->d1[r] = q.d1;
      if (out->d2) out->d2[r] = q.d2;
      if (out->count) out->count[r] = q.count;
      if (out->borderline) out->borderline[r] = q.borderline;
      if (out->accept) out->accept[r] = q.accept;
      cmp += q.count;
      bl += q.borderline;
      acc += q.accept;
    }
    if (out->n_comparisons) out->n_comparisons[p] = cmp;
    if (out->n_borderline) out->n_borderline[p] = bl;
    if (out->n_accepted) out->n_accepted[p] = acc;
  }
  return 0;
}
