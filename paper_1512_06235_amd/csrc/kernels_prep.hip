// Registration, per-pair geometry and binning kernels.
//
// Geometry (a1) follows the epipolar relations of Section 6.2: every line
// l = F x_a passes through the epipole e of image b (e^T F = 0), so the band
// of eq. (2) around l only holds features of b whose own line through e is
// close to l.  Binning (a3, Appendix A step 1) sorts b's features by a
// coordinate of that pencil of lines; query tiling (a2, Appendix A step 2)
// sorts a's queries by the same coordinate of their lines, so that a tile of
// consecutive queries needs one contiguous range of b.  Unlike the paper's
// four overlapping 2d x 2d grids and centre-most cells (eqs. 6-9), the range
// is a provable superset of every member of the band; the exact test happens
// in the match kernel.
#include <algorithm>
#include <cmath>

#include "sfm_internal.h"

namespace sfm {
namespace {

// ---------------------------------------------------------------------------
// Registration: squared norms, byte range check, keypoint bounding box.
// One workgroup per image.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void register_kernel(ImageDev* imgs, int32_t* norm2_all,
                                                       const int64_t* norm_off, int32_t* bad) {
  const int k = blockIdx.x;
  const ImageDev im = imgs[k];
  int32_t* nrm = norm2_all + norm_off[k];
  float mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  uint32_t orbits = 0;
  for (int32_t f = threadIdx.x; f < im.n; f += blockDim.x) {
    const uint4* row = reinterpret_cast<const uint4*>(im.desc + int64_t(f) * kDescBytes);
    int32_t s = 0;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      const uint4 v = row[w];
      const uint32_t d[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        orbits |= d[t];
        s = __builtin_amdgcn_udot4(d[t], d[t], uint32_t(s), false);
      }
    }
    nrm[f] = s;
    const float x = im.xy[2 * f], y = im.xy[2 * f + 1];
    if (!(isfinite(x) && isfinite(y))) orbits |= 0x80u;  // reported as invalid input
    mnx = fminf(mnx, x); mny = fminf(mny, y);
    mxx = fmaxf(mxx, x); mxy = fmaxf(mxy, y);
  }
  if (orbits & 0x80808080u) atomicOr(bad, 1);
  __shared__ float red[4][256];
  red[0][threadIdx.x] = mnx; red[1][threadIdx.x] = mny;
  red[2][threadIdx.x] = mxx; red[3][threadIdx.x] = mxy;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) {
      red[0][threadIdx.x] = fminf(red[0][threadIdx.x], red[0][threadIdx.x + s]);
      red[1][threadIdx.x] = fminf(red[1][threadIdx.x], red[1][threadIdx.x + s]);
      red[2][threadIdx.x] = fmaxf(red[2][threadIdx.x], red[2][threadIdx.x + s]);
      red[3][threadIdx.x] = fmaxf(red[3][threadIdx.x], red[3][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (im.n == 0) {
      imgs[k].bbox[0] = imgs[k].bbox[1] = imgs[k].bbox[2] = imgs[k].bbox[3] = 0.0f;
    } else {
      imgs[k].bbox[0] = red[0][0]; imgs[k].bbox[1] = red[1][0];
      imgs[k].bbox[2] = red[2][0]; imgs[k].bbox[3] = red[3][0];
    }
  }
}

// ---------------------------------------------------------------------------
// a1: per-pair geometry in FP64.
// ---------------------------------------------------------------------------
__device__ inline void cross3(const double* p, const double* q, double* r) {
  r[0] = p[1] * q[2] - p[2] * q[1];
  r[1] = p[2] * q[0] - p[0] * q[2];
  r[2] = p[0] * q[1] - p[1] * q[0];
}

__device__ void setup_pair(const PairDesc& P, const ImageDev& B, const double* Fin, double margin,
                           PairGeom& g) {
  double fro = 0.0;
  for (int k = 0; k < 9; ++k) fro += Fin[k] * Fin[k];
  fro = sqrt(fro);
  for (int k = 0; k < 9; ++k) g.F[k] = Fin[k] / fro;
  const double* F = g.F;

  // Epipole of b: e^T F = 0, orthogonal to every column of F.  Take the
  // cross product of the best-conditioned pair of columns.
  const double c0[3] = {F[0], F[3], F[6]}, c1[3] = {F[1], F[4], F[7]}, c2[3] = {F[2], F[5], F[8]};
  double e[3], t[3];
  cross3(c0, c1, e);
  double best = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
  cross3(c0, c2, t);
  double n2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  if (n2 > best) { best = n2; e[0] = t[0]; e[1] = t[1]; e[2] = t[2]; }
  cross3(c1, c2, t);
  n2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  if (n2 > best) { best = n2; e[0] = t[0]; e[1] = t[1]; e[2] = t[2]; }
  const double en = sqrt(best);

  const double bx0 = B.bbox[0], by0 = B.bbox[1], bx1 = B.bbox[2], by1 = B.bbox[3];
  g.ox = floor(0.5 * (bx0 + bx1));
  g.oy = floor(0.5 * (by0 + by1));
  const double cx[4] = {bx0, bx1, bx0, bx1}, cy[4] = {by0, by0, by1, by1};
  double rbox = 0.0;
  for (int k = 0; k < 4; ++k) rbox = fmax(rbox, hypot(cx[k] - g.ox, cy[k] - g.oy));
  g.rbox = rbox;
  g.half_width = P.band + kBandSlackPx;
  // The match kernel decides |e| <= band_lo as in and |e| > band_hi as out in
  // FP32; distances in between are decided again in FP64.
  g.band_lo = float(P.band - margin);
  g.band_hi = float(P.band + margin);
  g.nbins = P.nbins;
  g.mode = kModeFullScan;
  g.ex = g.ey = 0.0; g.ux = 1.0; g.uy = 0.0; g.S = 1.0;
  g.kmin = 0.0; g.kmax = 0.0; g.inv_delta = 0.0;
  if (P.ignore_band || !(P.band < 1e30) || P.nb == 0 || !(en > 0.0)) return;

  for (int k = 0; k < 3; ++k) e[k] /= en;
  const double exy = hypot(e[0], e[1]);
  double kmin = INFINITY, kmax = -INFINITY;
  if (fabs(e[2]) <= 1e-12 * exy) {
    // Epipole at infinity: all lines run along u; key = offset along n.
    g.ux = e[0] / exy; g.uy = e[1] / exy;
    const double nx = -g.uy, ny = g.ux;
    for (int k = 0; k < 4; ++k) {
      const double key = nx * (cx[k] - g.ox) + ny * (cy[k] - g.oy);
      kmin = fmin(kmin, key); kmax = fmax(kmax, key);
    }
    g.mode = kModeParallel;
  } else {
    const double Ex = e[0] / e[2], Ey = e[1] / e[2];
    double ux = g.ox - Ex, uy = g.oy - Ey;
    const double un = hypot(ux, uy);
    if (!(un > 0.0)) return;
    ux /= un; uy /= un;
    double vmin = INFINITY;
    for (int k = 0; k < 4; ++k) vmin = fmin(vmin, (cx[k] - Ex) * ux + (cy[k] - Ey) * uy);
    // The pencil coordinate needs b's box strictly on one side of the epipole,
    // well clear of the band; otherwise fall back to scanning all of b.
    if (!(vmin > 4.0 * g.half_width) || !(vmin > 1.0)) return;
    g.ex = Ex; g.ey = Ey; g.ux = ux; g.uy = uy; g.S = vmin;
    for (int k = 0; k < 4; ++k) {
      const double vx = cx[k] - Ex, vy = cy[k] - Ey;
      const double key = vmin * (-uy * vx + ux * vy) / (ux * vx + uy * vy);
      kmin = fmin(kmin, key); kmax = fmax(kmax, key);
    }
    g.mode = kModePencil;
  }
  g.kmin = kmin; g.kmax = kmax;
  g.inv_delta = (kmax > kmin) ? double(P.nbins) / (kmax - kmin) : 0.0;
}

__global__ void geometry_kernel(BatchView v, int32_t pb, int32_t pc) {
  const int32_t p = pb + blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= pb + pc) return;
  const PairDesc P = v.pairs[p];
  PairGeom g;
  setup_pair(P, v.images[P.b], v.F + 9 * int64_t(p), v.margin, g);
  v.geom[p] = g;
  PairCounters z;
  z.comparisons = 0;
  z.elements = 0;
  z.borderline = 0;
  z.accepted = 0;
  z.ties = 0;
  v.counters[p] = z;
  v.pcost[p] = 0;
}

// ---------------------------------------------------------------------------
// Keys of the pencil coordinate (shared by a2 and a3).
// ---------------------------------------------------------------------------
__device__ inline double point_key(const PairGeom& g, double x, double y) {
  if (g.mode == kModePencil) {
    const double vx = x - g.ex, vy = y - g.ey;
    return g.S * (-g.uy * vx + g.ux * vy) / (g.ux * vx + g.uy * vy);
  }
  if (g.mode == kModeParallel) return -g.uy * (x - g.ox) + g.ux * (y - g.oy);
  return 0.0;
}

__device__ inline int32_t key_bin(const PairGeom& g, double key) {
  double t = (key - g.kmin) * g.inv_delta;
  t = fmin(fmax(t, 0.0), double(g.nbins - 1));
  return int32_t(floor(t));
}

// Query line on centred coordinates, its sort bin and its window of bins.
struct QueryLine {
  float a, b, c;
  int32_t wlo, whi;     // wlo > whi: no feature of b can be in the band
};

__device__ QueryLine query_line(const PairGeom& g, float xq, float yq) {
  QueryLine q;
  const double* F = g.F;
  const double x = xq, y = yq;
  double a = F[0] * x + F[1] * y + F[2];
  double b = F[3] * x + F[4] * y + F[5];
  double c = F[6] * x + F[7] * y + F[8];
  const double s = sqrt(a * a + b * b);
  if (!(s > 0.0) || !isfinite(s) || !isfinite(c)) {
    q.a = q.b = q.c = NAN;   // the FP32 band test is false for every target
    q.wlo = 1; q.whi = 0;
    return q;
  }
  const double inv_s = 1.0 / s;
  a *= inv_s; b *= inv_s; c *= inv_s;
  const double cc = c + a * g.ox + b * g.oy;   // offset on centred coordinates
  q.a = float(a); q.b = float(b); q.c = float(cc);
  if (g.mode == kModeFullScan) {
    q.wlo = 0; q.whi = 0;
    return q;
  }
  double lam, h;
  const double nx = -g.uy, ny = g.ux;
  if (g.mode == kModePencil) {
    // Line direction w = (-b, a); key S * tan of its angle to u.
    const double wpar = -b * g.ux + a * g.uy;
    const double wper = -b * nx + a * ny;
    const double eps = fabs(a * g.ex + b * g.ey + c);  // distance of e from the line
    if (!(eps < 0.5 * g.S)) {                            // inconsistent F: scan everything
      q.wlo = 0; q.whi = g.nbins - 1;
      return q;
    }
    if (fabs(wpar) < 1e-300) { q.wlo = 1; q.whi = 0; return q; }
    const double r = wper / wpar;
    lam = g.S * r;
    h = (g.half_width + eps) * sqrt(1.0 + r * r);
  } else {
    const double dot = a * nx + b * ny;
    const double sg = dot >= 0.0 ? 1.0 : -1.0;
    lam = -sg * cc;
    const double dx = a - sg * nx, dy = b - sg * ny;
    h = g.half_width + sqrt(dx * dx + dy * dy) * g.rbox;
  }
  if (!(lam + h >= g.kmin) || !(lam - h <= g.kmax)) {
    q.wlo = 1; q.whi = 0;
    return q;
  }
  q.wlo = key_bin(g, lam - h);
  q.whi = key_bin(g, lam + h);
  return q;
}

// The bin a query is sorted by: the pencil key of its line (S * tan of the
// line's angle to u about the epipole, or the offset across parallel lines),
// clamped to b's bins; degenerate lines go to the extra bin nbins.  Only the
// order of queries depends on it (windows come from query_line), so it skips
// the normalisation and window arithmetic; both passes of the counting sort
// call this same function, so they agree on every bin.
__device__ inline int32_t query_sort_bin(const PairGeom& g, float xq, float yq) {
  const double* F = g.F;
  const double x = xq, y = yq;
  const double a = F[0] * x + F[1] * y + F[2];
  const double b = F[3] * x + F[4] * y + F[5];
  const double s2 = a * a + b * b;
  if (!(s2 > 0.0) || !isfinite(s2)) return g.nbins;
  if (g.mode == kModeFullScan) return 0;
  double lam;
  if (g.mode == kModePencil) {
    const double wpar = -b * g.ux + a * g.uy;
    const double wper = b * g.uy + a * g.ux;
    lam = g.S * wper / wpar;
  } else {
    const double c = F[6] * x + F[7] * y + F[8];
    const double dot = -a * g.uy + b * g.ux;
    lam = (dot >= 0.0 ? -1.0 : 1.0) * (c + a * g.ox + b * g.oy) / sqrt(s2);
  }
  if (!isfinite(lam)) return g.nbins;
  return key_bin(g, lam);
}

// ---------------------------------------------------------------------------
// Workgroup-wide exclusive scan of cnt[0..n) in LDS (n <= 8 * blockDim).
// ---------------------------------------------------------------------------
template <int NT>
__device__ void block_exclusive_scan(int32_t* cnt, int32_t n, int32_t* wsum) {
  constexpr int PER = (kMaxBins + 2 + NT - 1) / NT;
  const int t = threadIdx.x;
  int32_t local[PER];
  int32_t sum = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int idx = t * PER + k;
    local[k] = idx < n ? cnt[idx] : 0;
    sum += local[k];
  }
  // Inclusive scan of per-thread sums: within waves, then across waves.
  const int lane = t & 63, wv = t >> 6;
  int32_t x = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  if (t == 0) {
    int32_t run = 0;
    for (int w = 0; w < NT / 64; ++w) { const int32_t s = wsum[w]; wsum[w] = run; run += s; }
  }
  __syncthreads();
  int32_t run = x - sum + wsum[wv];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int idx = t * PER + k;
    if (idx < n) cnt[idx] = run;
    run += local[k];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// a2 + a3: one workgroup per (pair, image): one bins the targets of b, the
// other lines up and tiles the queries of a.  Counting sort:
// pass 1 counts bins in LDS, a scan gives bin starts, pass 2 scatters.  The
// bins of the first kCacheRounds rounds of items stay in registers between
// the passes, so their FP64 keys are computed once.  `order` (may be NULL)
// maps blockIdx.x to the pair, largest pairs first.
// ---------------------------------------------------------------------------
// 512 threads at 128 VGPRs fit two binning workgroups per CU, which
// overlaps one pair's barrier phases with another's work; a batch of few
// pairs (at most one workgroup per CU) takes 1,024 threads per side
// instead, which halves each side's passes.
constexpr int kBinThreads = 512;
constexpr int kBinThreadsFew = 1024;
constexpr int kBatch = 8;   // items per thread per round; their loads are issued together
constexpr int kCacheRounds = 3;

// Counting sort of one side of a pair: the targets of b into binned order
// (and the bin starts), or the queries of a into tile order.
// Global loads and stores through address-space-1 pointers (the pointers
// live in records, so the compiler would otherwise emit flat accesses, which
// also count against the LDS counter).  The passes below load every slot of a
// round unconditionally at a clamped index, so a round's loads are all in
// flight together instead of each waiting in its own branch.
template <class T>
__device__ __forceinline__ T ldg(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ void stg(T* p, const T& x) {
  *(__attribute__((address_space(1))) T*)p = x;
}

// Writes one item at its sorted position; a query also returns its bin
// window (first, last bin; first > last: none).
template <bool kTargets>
__device__ __forceinline__ int2 write_sorted(const BatchView& v, const PairDesc& P,
                                             const PairGeom& g, int32_t pos, int32_t j, float x,
                                             float y, int32_t nrm) {
  if (kTargets) {
    stg(v.cand_x + P.c_off + pos, float(double(x) - g.ox));
    stg(v.cand_y + P.c_off + pos, float(double(y) - g.oy));
    stg(v.cand_nc + P.c_off + pos,
        ((uint32_t(nrm) + kDistBias) << kPosBits) | uint32_t(pos & (kChunk - 1)));
    stg(v.cand_j + P.c_off + pos, j);
    return make_int2(1, 0);
  } else {
    const QueryLine q = query_line(g, x, y);
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    static_assert(sizeof(QueryRec) == sizeof(u4), "a query record is one 16-byte store");
    const u4 rq = {__float_as_uint(q.a), __float_as_uint(q.b), __float_as_uint(q.c), uint32_t(j)};
    stg(reinterpret_cast<u4*>(v.qrec + P.q_off + pos), rq);
    return make_int2(q.wlo, q.whi);
  }
}

// The bin window of a query tile (positions 16 t .. 16 t + 15, held by 16
// consecutive lanes): the union of its queries' windows, by min / max
// shuffles within the 16 lanes (every lane takes part; lanes without a query
// pass an empty window), stored by the tile's first lane.
__device__ __forceinline__ void store_tile_window(const BatchView& v, const PairDesc& P,
                                                  int32_t pos, int32_t n, int2 w) {
  int32_t lo = w.x <= w.y ? w.x : 0x7FFFFFFF;
  int32_t hi = w.x <= w.y ? w.y : -1;
  for (int o = kQueryTile / 2; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o, 64));
    hi = max(hi, __shfl_xor(hi, o, 64));
  }
  if ((pos & (kQueryTile - 1)) == 0 && pos < n)
    v.twin[P.blk_off + pos / kQueryTile] = make_int2(lo, hi);
}

// When `perm` is given (the side fits in LDS), pass 2 only records which
// item lands at each position; a gather pass then writes the outputs in
// position order, so the stores are coalesced instead of scattered 8- and
// 16-byte writes that the L2 cannot merge once a batch outgrows it.
template <int NT, bool kTargets>
__device__ __forceinline__ void sort_side(const BatchView& v, const PairDesc& P,
                                          const PairGeom& g, const ImageDev& I, int32_t* hist,
                                          int32_t* wsum, int32_t nh, uint16_t* perm) {
  constexpr int32_t kStride = kBatch * NT;
  const int32_t n = kTargets ? P.nb : P.na;
  // The bin of one item (FP64 key of a target, sort key of a query).
  auto item_bin = [&](float x, float y) -> int32_t {
    return kTargets ? key_bin(g, point_key(g, x, y)) : query_sort_bin(g, x, y);
  };
  // Pass 1 over round r: count bins; keep them in `keep` when given.
  auto count_round = [&](int32_t r, int32_t* keep) {
    const int32_t base = r * kStride + threadIdx.x;
    float px[kBatch], py[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int32_t j = min(base + k * NT, n - 1);
      px[k] = ldg(I.xy + 2 * j);
      py[k] = ldg(I.xy + 2 * j + 1);
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      if (base + k * NT < n) {
        const int32_t bin = item_bin(px[k], py[k]);
        atomicAdd(&hist[bin], 1);
        if (keep) keep[k] = bin;
      }
    }
  };
  // Pass 2 over round r: place every item of the round at its sorted position.
  auto place_round = [&](int32_t r, const int32_t* keep) {
    const int32_t base = r * kStride + threadIdx.x;
    float px[kBatch], py[kBatch];
    int32_t nrm[kBatch];
    if (!perm || !keep) {
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int32_t j = min(base + k * NT, n - 1);
        px[k] = ldg(I.xy + 2 * j);
        py[k] = ldg(I.xy + 2 * j + 1);
        if (kTargets) nrm[k] = ldg(I.norm2 + j);   // used by the direct path only
      }
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int32_t j = base + k * NT;
      if (j >= n) continue;
      const int32_t bin = keep ? keep[k] : item_bin(px[k], py[k]);
      const int32_t pos = atomicAdd(&hist[bin], 1);
      if (perm) {
        perm[pos] = uint16_t(j);
      } else {
        const int2 w =
            write_sorted<kTargets>(v, P, g, pos, j, px[k], py[k], kTargets ? nrm[k] : 0);
        // Scattered positions: the tile windows (cleared before the count
        // pass) are merged with atomics.
        if (!kTargets && w.x <= w.y) {
          int2* tw = v.twin + P.blk_off + pos / kQueryTile;
          atomicMin(&tw->x, w.x);
          atomicMax(&tw->y, w.y);
        }
      }
    }
  };

  const int32_t rounds = (n + kStride - 1) / kStride;
  if (!kTargets && !perm) {
    // Empty windows for the atomics of the direct path (the barriers of the
    // scan order these stores before them).
    for (int32_t t = threadIdx.x; t < P.nblocks; t += blockDim.x)
      v.twin[P.blk_off + t] = make_int2(0x7FFFFFFF, -1);
  }
  int32_t keep[kCacheRounds][kBatch];
#pragma unroll
  for (int32_t r = 0; r < kCacheRounds; ++r)
    if (r < rounds) count_round(r, keep[r]);
  for (int32_t r = kCacheRounds; r < rounds; ++r) count_round(r, nullptr);
  __syncthreads();
  block_exclusive_scan<NT>(hist, nh, wsum);
  if (kTargets) {
    for (int k = threadIdx.x; k < nh; k += blockDim.x) v.bin_start[P.bin_off + k] = hist[k];
    if (threadIdx.x == 0) v.bin_start[P.bin_off + nh] = P.nb;
    __syncthreads();
  }
#pragma unroll
  for (int32_t r = 0; r < kCacheRounds; ++r)
    if (r < rounds) place_round(r, keep[r]);
  for (int32_t r = kCacheRounds; r < rounds; ++r) place_round(r, nullptr);
  if (!perm) return;
  __syncthreads();
  if (NT == kBinThreadsFew) {
    // A batch of few pairs: the item of every position, in position order
    // (coalesced), into cand_j for targets (one of their outputs) or into
    // the records' index field for queries; gather_kernel then writes the
    // records over the whole GPU instead of this one workgroup.
    for (int32_t pos = threadIdx.x; pos < n; pos += NT) {
      const int32_t j = perm[pos];
      if (kTargets)
        stg(v.cand_j + P.c_off + pos, j);
      else
        stg(&v.qrec[P.q_off + pos].i, j);
    }
    return;
  }
  // Gather pass: positions in order, kBatch per thread per round (every
  // thread runs every round: the tile windows shuffle across lanes).
  for (int32_t r = 0; r < rounds; ++r) {
    const int32_t base = r * kStride + threadIdx.x;
    int32_t jj[kBatch], nrm[kBatch];
    float px[kBatch], py[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) jj[k] = perm[min(base + k * NT, n - 1)];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      px[k] = ldg(I.xy + 2 * jj[k]);
      py[k] = ldg(I.xy + 2 * jj[k] + 1);
      if (kTargets) nrm[k] = ldg(I.norm2 + jj[k]);
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int32_t pos = base + k * NT;
      int2 w = make_int2(1, 0);
      if (pos < n)
        w = write_sorted<kTargets>(v, P, g, pos, jj[k], px[k], py[k], kTargets ? nrm[k] : 0);
      if (!kTargets) store_tile_window(v, P, pos, n, w);
    }
  }
}

// LDS of the binning workgroup: the histogram, the scan's wave sums and,
// when the side fits, the 16-bit permutation of its items.
constexpr int kBinLdsInts = 16384;
constexpr int kBinWsumMax = kBinThreadsFew / 64;
static_assert(kMaxBins + 2 + kBinWsumMax <= kBinLdsInts, "histogram fits");

// Whether a side of n items and nh bins sorts through an LDS permutation
// (its records then come from gather_kernel) or scatters them directly.
__host__ __device__ constexpr bool perm_fits(int32_t nh, int32_t n, int32_t wsum_ints) {
  return ((nh + 2) & ~1) + (n + 1) / 2 <= kBinLdsInts - wsum_ints;
}

template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
void bin_kernel(BatchView v, int32_t pb, const int32_t* order) {
  constexpr int kBinWsum = NT / 64;
  __shared__ int32_t lds[kBinLdsInts];
  int32_t* const wsum = lds + kBinLdsInts - kBinWsum;
  int32_t* const hist = lds;
  // Workgroup 2k + 1 sorts the targets and 2k the queries of the k-th pair
  // in `order`: both sides of the largest pairs are dispatched first, the
  // costlier query side ahead of its targets.
  const int32_t rank = blockIdx.x >> 1;
  const int32_t p = order ? order[pb + rank] : pb + rank;
  const PairDesc P = v.pairs[p];
  const PairGeom g = v.geom[p];
  const bool targets = (blockIdx.x & 1) != 0;
  const int32_t nh = targets ? g.nbins : g.nbins + 1;
  const ImageDev I = v.images[targets ? P.b : P.a];

  if (P.ignore_band) {
    // Exhaustive matching keeps b in its own order: one bin, position = index.
    if (targets) {
      for (int32_t j = threadIdx.x; j < P.nb + kCandPad; j += blockDim.x) {
        const bool pad = j >= P.nb;
        v.cand_x[P.c_off + j] = pad ? NAN : 0.0f;
        v.cand_y[P.c_off + j] = 0.0f;
        v.cand_nc[P.c_off + j] =
            pad ? kKeyInf
                : ((uint32_t(I.norm2[j]) + kDistBias) << kPosBits) | uint32_t(j & (kChunk - 1));
        v.cand_j[P.c_off + j] = pad ? 0 : j;
      }
      if (threadIdx.x == 0) {
        v.bin_start[P.bin_off] = 0;
        for (int k = 1; k <= g.nbins; ++k) v.bin_start[P.bin_off + k] = P.nb;
      }
    } else {
      for (int32_t i = threadIdx.x; i < P.na; i += blockDim.x) {
        QueryRec r;
        r.a = 0.0f; r.b = 0.0f; r.c = 0.0f; r.i = i;
        v.qrec[P.q_off + i] = r;
      }
      for (int32_t t = threadIdx.x; t < P.nblocks; t += blockDim.x)
        v.twin[P.blk_off + t] = make_int2(0, 0);
    }
    return;
  }

  for (int k = threadIdx.x; k < nh; k += blockDim.x) hist[k] = 0;
  __syncthreads();
  const int32_t n = targets ? P.nb : P.na;
  const int32_t hist_ints = (nh + 2) & ~1;
  uint16_t* perm = nullptr;
  if (perm_fits(nh, n, kBinWsum)) perm = reinterpret_cast<uint16_t*>(lds + hist_ints);
  if (targets) {
    // Padding after the pair's targets: a NaN x fails every band test.
    if (int(threadIdx.x) < kCandPad) {
      const int64_t o = P.c_off + P.nb + threadIdx.x;
      v.cand_x[o] = NAN;
      v.cand_y[o] = 0.0f;
      v.cand_nc[o] = kKeyInf;
      v.cand_j[o] = 0;
    }
    sort_side<NT, true>(v, P, g, I, hist, wsum, nh, perm);
  } else {
    sort_side<NT, false>(v, P, g, I, hist, wsum, nh, perm);
  }
}

// Batches of few pairs (1,024-thread binning): the records of every side
// that binning sorted through its LDS permutation, one thread per sorted
// position of block (pair, y, side): the
// position's item (left in cand_j or the record's index by bin_kernel), its
// keypoint and norm or its FP64 line and window, the outputs in position
// order, and per 16-query tile the union of its windows (16 consecutive
// positions on 16 lanes).  Spreading these random reads and the FP64 line
// arithmetic over the GPU takes them off the one workgroup per side.
constexpr int kGatherThreads = 256;
__global__ __launch_bounds__(kGatherThreads) void gather_kernel(BatchView v, int32_t pb,
                                                                int32_t wsum_ints) {
  const int32_t p = pb + int32_t(blockIdx.x);
  const PairDesc P = v.pairs[p];
  const bool targets = blockIdx.z != 0;
  const int32_t n = targets ? P.nb : P.na;
  const int32_t base = int32_t(blockIdx.y) * kGatherThreads;
  if (P.ignore_band || base >= n) return;   // uniform
  const PairGeom& g = v.geom[p];
  const int32_t nh = targets ? g.nbins : g.nbins + 1;
  if (!perm_fits(nh, n, wsum_ints)) return;   // scattered by bin_kernel itself
  const ImageDev& I = v.images[targets ? P.b : P.a];
  const int32_t pos = base + int32_t(threadIdx.x);
  const int32_t pc = min(pos, n - 1);
  if (targets) {
    const int32_t j = ldg(v.cand_j + P.c_off + pc);
    const float x = ldg(I.xy + 2 * j), y = ldg(I.xy + 2 * j + 1);
    const int32_t nrm = ldg(I.norm2 + j);
    if (pos < n) write_sorted<true>(v, P, g, pos, j, x, y, nrm);
  } else {
    const int32_t j = ldg(&v.qrec[P.q_off + pc].i);
    const float x = ldg(I.xy + 2 * j), y = ldg(I.xy + 2 * j + 1);
    int2 w = make_int2(1, 0);
    if (pos < n) w = write_sorted<false>(v, P, g, pos, j, x, y, 0);
    store_tile_window(v, P, pos, n, w);
  }
}

// Candidate range of every query tile (its bin window mapped through b's
// bin starts) and of every group of K consecutive tiles, with the group
// record and its schedule cost.  Block (p, c) takes tiles [256c, 256c + 256)
// of pair p: one thread per tile, one thread per group.
constexpr int kRangeThreads = 256;
constexpr int kRangeTiles = kRangeThreads;
static_assert(kRangeTiles % kMaxGroupTiles == 0, "a block holds whole groups");
static_assert(kRangeTiles / 4 <= 64, "a block's groups fit in its first wave");

template <int K>
__global__ __launch_bounds__(kRangeThreads) void tile_ranges_kernel(BatchView v, int32_t pb) {
  __shared__ int2 trange[kRangeTiles];
  const int32_t p = pb + blockIdx.x;
  const PairDesc P = v.pairs[p];
  const int32_t tile0 = int32_t(blockIdx.y) * kRangeTiles;
  if (tile0 >= P.nblocks) return;
  const int t = threadIdx.x, lane = t & 63;
  // What the group records take from the pair's images and geometry, read
  // before the tile windows so the loads overlap.
  const ImageDev A = v.images[P.a];
  const ImageDev B = v.images[P.b];
  const float band_lo = v.geom[p].band_lo, band_hi = v.geom[p].band_hi;
  int2 r = make_int2(0, 0);
  if (tile0 + t < P.nblocks) {
    const int2 w = v.twin[P.blk_off + tile0 + t];
    if (w.x <= w.y)
      r = make_int2(v.bin_start[P.bin_off + w.x], v.bin_start[P.bin_off + w.y + 1]);
  }
  trange[t] = r;
  __syncthreads();
  const int32_t tiles_here = min(kRangeTiles, P.nblocks - tile0);
  const int32_t groups_here = (tiles_here + K - 1) / K;
  long long cost = 0;
  if (t < groups_here) {
    const int32_t g = int32_t(blockIdx.y) * (kRangeTiles / K) + t;
    const int32_t k0 = g * K;
    const int32_t nt = min(K, P.nblocks - k0);
    TileGroup tg;
    memset(&tg, 0, sizeof tg);
    int32_t gb = 0x7FFFFFFF, ge = 0, steps = 0;
#pragma unroll
    for (int32_t k = 0; k < K; ++k) {
      int2 r = make_int2(0, 0);
      if (k < nt) r = trange[t * K + k];
      if (r.y > r.x) {
        gb = min(gb, r.x);
        ge = max(ge, r.y);
        steps += (r.y - (r.x & ~3) + kQueryTile - 1) / kQueryTile;
      }
      tg.t_begin[k] = r.x;
      tg.t_end[k] = r.y;
    }
    tg.pair = p;
    tg.tile0 = k0;
    tg.ntiles = nt;
    tg.na = P.na;
    tg.s_begin = gb <= ge ? gb : 0;
    tg.s_end = gb <= ge ? ge : 0;
    tg.band_lo = band_lo;
    tg.band_hi = band_hi;
    tg.q_off = P.q_off;
    tg.c_off = P.c_off;
    tg.a_desc = A.desc;
    tg.b_desc = B.desc;
    tg.a_norm = A.norm2;
    tg.nb = P.nb;
    tg.a_xy = A.xy;
    tg.b_xy = B.xy;
    tg.band = P.band;
    v.groups[P.grp_off + g] = tg;
    // A group costs a fixed start-up, one stream stage per 64 positions of
    // its union (plus the stage its last steps reach into) and its tiles'
    // steps, which its four waves share.
    const int32_t segs =
        tg.s_end > tg.s_begin ? (tg.s_end + kQueryTile - 1 - (tg.s_begin & ~3) + 63) / 64 : 0;
    const int32_t c = kGroupStartCost + kSegCost * segs + (kStepCost * steps) / kMatchWaves;
    v.gcost[P.grp_off + g] = c;
    cost = c;
  }
  // The block's groups all sit in the first wave: add their costs to the pair's.
  if (t < 64) {
    for (int o = 32; o > 0; o >>= 1) cost += __shfl_xor(cost, o, 64);
    if (lane == 0 && cost) atomicAdd(reinterpret_cast<unsigned long long*>(&v.pcost[p]),
                                     (unsigned long long)cost);
  }
}

// Splits the tile groups of pairs [pb, pb + pc) into `wgs` contiguous runs
// (shares) of about equal cost: group g goes to run floor(pre(g) * wgs /
// total), pre(g) being the cost of the groups before it, so run k starts at
// the first group with pre(g) * wgs >= k * total.  One wave per pair finds the starts that
// fall inside its pair; the pair with the last group also closes the table.
__global__ __launch_bounds__(256) void schedule_kernel(BatchView v, int32_t pb, int32_t pc,
                                                       int32_t g0, int32_t n, int32_t wgs) {
  const int lane = threadIdx.x & 63;
  const int32_t p = pb + int32_t(blockIdx.x) * 4 + int32_t(threadIdx.x >> 6);
  if (p >= pb + pc) return;
  // Cost before this pair and in total.
  long long before = 0, total = 0;
#pragma unroll 4
  for (int32_t q = pb + lane; q < pb + pc; q += 64) {
    const long long c = v.pcost[q];
    total += c;
    before += q < p ? c : 0;
  }
  for (int o = 32; o > 0; o >>= 1) {
    total += __shfl_xor(total, o, 64);
    before += __shfl_xor(before, o, 64);
  }
  const PairDesc P = v.pairs[p];
  const int32_t ng = P.ngroups;
  if (ng == 0 || total <= 0) return;
  const int32_t gl = int32_t(P.grp_off) - g0;   // first group of the pair, local
  const int32_t* cost = v.gcost + g0 + gl;
  const long long W = wgs;
  // Starts that fall in this pair: k in [k_lo, k_hi].
  const long long last_pre = before + v.pcost[p] - cost[ng - 1];
  const int32_t k_hi = int32_t(last_pre * W / total);
  int32_t k = gl == 0 ? 0 : int32_t((before - v.gcost[g0 + gl - 1]) * W / total) + 1;
  long long carry = before;
  for (int32_t c0 = 0; c0 < ng && k <= k_hi; c0 += 64) {
    const int32_t j = c0 + lane;
    const long long c = j < ng ? cost[j] : 0;
    long long inc = c;   // inclusive scan over the chunk
    for (int o = 1; o < 64; o <<= 1) {
      const long long y = __shfl_up(inc, o, 64);
      inc += lane >= o ? y : 0;
    }
    const long long pre = carry + inc - c;
    while (k <= k_hi) {
      const unsigned long long hit = __ballot(j < ng && pre * W >= (long long)k * total);
      if (!hit) break;
      if (lane == 0) v.wg_start[k] = g0 + gl + c0 + __builtin_ctzll(hit);
      ++k;
    }
    carry += __shfl(inc, 63, 64);
  }
  if (gl + ng == n && lane == 0) {
    for (int32_t kk = k_hi + 1; kk <= wgs; ++kk) v.wg_start[kk] = g0 + n;
  }
}

}  // namespace

hipError_t launch_register(const ImageDev* imgs_host, ImageDev* imgs_dev, int32_t n_images,
                           int32_t* norm2_all, const int64_t* norm_off, float* bbox_dev,
                           int32_t* bad_flag, hipStream_t st) {
  (void)imgs_host;
  (void)bbox_dev;
  if (n_images == 0) return hipSuccess;
  hipLaunchKernelGGL(register_kernel, dim3(n_images), dim3(256), 0, st, imgs_dev, norm2_all,
                     norm_off, bad_flag);
  return hipGetLastError();
}

// Binning workgroups that one wave of 1,024-thread workgroups runs at once
// (one per CU).
constexpr int32_t kFewPairsWorkgroups = 256;

hipError_t launch_prepare(const BatchView& v, int32_t pb, int32_t pc, int32_t grp_begin,
                          int32_t grp_count, int32_t wgs, const int32_t* order,
                          int32_t max_queries, hipStream_t st) {
  if (pc <= 0) return hipSuccess;
  hipLaunchKernelGGL(geometry_kernel, dim3((pc + 63) / 64), dim3(64), 0, st, v, pb, pc);
  const bool few = 2 * pc <= kFewPairsWorkgroups;
  if (few)
    hipLaunchKernelGGL(bin_kernel<kBinThreadsFew>, dim3(2 * pc), dim3(kBinThreadsFew), 0, st, v,
                       pb, order);
  else
    hipLaunchKernelGGL(bin_kernel<kBinThreads>, dim3(2 * pc), dim3(kBinThreads), 0, st, v, pb,
                       order);
  if (few) {
    const int32_t nmax = std::max(std::max(max_queries, v.max_nb), 1);
    hipLaunchKernelGGL(gather_kernel, dim3(pc, (nmax + kGatherThreads - 1) / kGatherThreads, 2),
                       dim3(kGatherThreads), 0, st, v, pb, kBinThreadsFew / 64);
  }
  const int32_t tiles = (max_queries + kQueryTile - 1) / kQueryTile;
  const int32_t qblocks = (tiles + kRangeTiles - 1) / kRangeTiles;
  if (qblocks > 0) {
    const dim3 grid(pc, qblocks), block(kRangeThreads);
    if (v.group_tiles == 4)
      hipLaunchKernelGGL(tile_ranges_kernel<4>, grid, block, 0, st, v, pb);
    else
      hipLaunchKernelGGL(tile_ranges_kernel<8>, grid, block, 0, st, v, pb);
  }
  if (grp_count > 0)
    hipLaunchKernelGGL(schedule_kernel, dim3((pc + 3) / 4), dim3(256), 0, st, v, pb, pc,
                       grp_begin, grp_count, std::min(kXcds, wgs));
  return hipGetLastError();
}

}  // namespace sfm
