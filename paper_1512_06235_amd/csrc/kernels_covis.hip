// Candidate images from point-camera covisibility (Section 6.1).
//
// For images i and j of the coarse model, the covisible points are the
// points both observe, P_cv(i, j) = Points(i) ∩ Points(j).  Image q's
// candidates are the images sharing more than T points with it, ranked by
// |P_cv(q, i)| (ties: lower index), at most k of them; the unique unordered
// pairs over all queries are what the matcher then runs.
//
// GPU form:
//   1. transpose the visibility (points of each image) into the observers of
//      each point: a counting sort by point id (count, scan, scatter);
//   2. one workgroup per query image q histograms, in LDS, the other
//      observers of every point q sees: row[j] = |P_cv(q, j)| for all j at once;
//      a bitonic sort of the packed keys (count, ~j) in LDS ranks the row and
//      the first k with count > T are the candidates;
//   3. the unique pairs: a bit per (i, j), i < j, set by every candidate,
//      then counted per row, scanned, and written in ascending order with a
//      popcount prefix per row.
#include <algorithm>

#include "sfm_internal.h"

namespace sfm {
namespace {

constexpr int kCovisThreads = 1024;

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* p, int64_t n, int32_t value) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = value;
}

// The [begin, end) range of image i's points, clamped to [0, nnz).
__device__ __forceinline__ void image_range(const int32_t* vis_off, int32_t i, int64_t nnz,
                                            int64_t& b, int64_t& e) {
  b = min(max(int64_t(vis_off[i]), int64_t(0)), nnz);
  e = min(max(int64_t(vis_off[i + 1]), b), nnz);
}

// Pass 1 of the transpose: observers per point.  One block per image.
__global__ __launch_bounds__(256) void covis_count_kernel(const int32_t* vis_off,
                                                          const int32_t* vis_pts, int64_t nnz,
                                                          int32_t n_points, int32_t* pt_count,
                                                          int32_t* err) {
  int64_t b, e;
  image_range(vis_off, blockIdx.x, nnz, b, e);
  for (int64_t s = b + threadIdx.x; s < e; s += blockDim.x) {
    const int32_t p = vis_pts[s];
    if (p < 0 || p >= n_points) {
      *err = 1;
      continue;
    }
    atomicAdd(&pt_count[p], 1);
  }
}

// Pass 2 of the transpose: image i into the observer list of each of its
// points.  Positions past nnz (inconsistent input) raise the error flag.
__global__ __launch_bounds__(256) void covis_scatter_kernel(const int32_t* vis_off,
                                                            const int32_t* vis_pts, int64_t nnz,
                                                            int32_t n_points, int32_t* cursor,
                                                            int32_t* pt_imgs, int32_t* err) {
  int64_t b, e;
  image_range(vis_off, blockIdx.x, nnz, b, e);
  for (int64_t s = b + threadIdx.x; s < e; s += blockDim.x) {
    const int32_t p = vis_pts[s];
    if (p < 0 || p >= n_points) continue;
    const int32_t pos = atomicAdd(&cursor[p], 1);
    if (pos < 0 || int64_t(pos) >= nnz) {
      *err = 1;
      continue;
    }
    pt_imgs[pos] = int32_t(blockIdx.x);
  }
}

// One block per query image q: |P_cv(q, j)| for every j in LDS, then the
// ranked candidates.  Keys pack (count, 2^32 - 1 - j) so a descending sort
// ranks by count, then by lower index; keys of non-candidates are 0.
// With `gram` given (the bit-matrix path), row q is read from it instead.
__global__ __launch_bounds__(kCovisThreads) void covis_rows_kernel(
    const int32_t* vis_off, const int32_t* vis_pts, int64_t nnz, int32_t n_images,
    int32_t n_points, const int32_t* pt_off, const int32_t* pt_imgs, const int32_t* gram,
    int32_t threshold, int32_t top_k, int32_t nsort, int32_t* cand, int32_t* n_shared,
    int32_t* n_cand) {
  __shared__ uint32_t row[kMaxCovisImages];
  __shared__ unsigned long long keys[kMaxCovisImages];
  __shared__ int32_t taken;
  const int32_t q = blockIdx.x;
  const int t = threadIdx.x;
  for (int32_t j = t; j < n_images; j += kCovisThreads)
    row[j] = gram ? uint32_t(gram[int64_t(q) * n_images + j]) : 0u;
  if (t == 0) taken = top_k;
  __syncthreads();
  if (!gram) {
  // A wave takes one point at a time and its lanes the point's observers:
  // the observers of a point are distinct images, so the LDS atomics of one
  // instruction never collide (lanes each walking their own point's list hit
  // the same nearby images together and serialise).
  // Four points per wave and iteration, their loads issued before any of
  // their atomics, so the chain point -> offsets -> observers overlaps.
  int64_t b, e;
  image_range(vis_off, q, nnz, b, e);
  const int lane = t & 63, wave = t >> 6;
  constexpr int kPts = 4;
  constexpr int64_t kWaveStride = int64_t(kCovisThreads / 64) * kPts;
  for (int64_t s0 = b + int64_t(wave) * kPts; s0 < e; s0 += kWaveStride) {
    int64_t o0[kPts], o1[kPts];
#pragma unroll
    for (int u = 0; u < kPts; ++u) {
      const int32_t p = s0 + u < e ? vis_pts[s0 + u] : -1;
      o0[u] = o1[u] = 0;
      if (p >= 0 && p < n_points) {
        // Offsets past nnz only arise from inconsistent input (the scatter
        // raised the error flag); reads stay inside pt_imgs.
        o0[u] = max(int64_t(pt_off[p]), int64_t(0));
        o1[u] = min(int64_t(pt_off[p + 1]), nnz);
      }
    }
    int32_t jj[kPts];
#pragma unroll
    for (int u = 0; u < kPts; ++u) jj[u] = o0[u] + lane < o1[u] ? pt_imgs[o0[u] + lane] : -1;
#pragma unroll
    for (int u = 0; u < kPts; ++u) {
      if (jj[u] != q && jj[u] >= 0 && jj[u] < n_images) atomicAdd(&row[jj[u]], 1u);
      for (int64_t o = o0[u] + 64 + lane; o < o1[u]; o += 64) {
        const int32_t j = pt_imgs[o];
        if (j != q && j >= 0 && j < n_images) atomicAdd(&row[j], 1u);
      }
    }
  }
  }
  __syncthreads();
  for (int32_t j = t; j < nsort; j += kCovisThreads) {
    const uint32_t c = j < n_images ? row[j] : 0u;
    keys[j] = (j < n_images && j != q && c > uint32_t(threshold))
                  ? ((unsigned long long)c << 32) | (0xFFFFFFFFull - uint32_t(j))
                  : 0ull;
  }
  __syncthreads();
  // Bitonic sort, descending, of nsort (a power of two) keys.
  for (int32_t size = 2; size <= nsort; size <<= 1) {
    for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (int32_t i = t; i < nsort / 2; i += kCovisThreads) {
        const int32_t lo = 2 * i - (i & (stride - 1));
        const int32_t hi = lo + stride;
        const bool desc = (lo & size) == 0;
        const unsigned long long a = keys[lo], c = keys[hi];
        if ((a < c) == desc) {
          keys[lo] = c;
          keys[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  for (int32_t r = t; r < top_k; r += kCovisThreads) {
    const unsigned long long key = r < nsort ? keys[r] : 0ull;
    const int64_t at = int64_t(q) * top_k + r;
    if (key != 0ull) {
      cand[at] = int32_t(0xFFFFFFFFull - (key & 0xFFFFFFFFull));
      n_shared[at] = int32_t(key >> 32);
    } else {
      cand[at] = -1;
      n_shared[at] = 0;
      if (r == 0 || (r - 1 < nsort && keys[r - 1] != 0ull)) taken = r;
    }
  }
  __syncthreads();
  if (t == 0) n_cand[q] = taken;
}

// ---------------------------------------------------------------------------
// Bit-matrix path: V[i] = the bitset of image i's points (words of 32
// points), and |P_cv(i, j)| = sum over words of popcount(V[i] & V[j]).
// ---------------------------------------------------------------------------
constexpr int kBitsLdsWords = 8192;   // points per LDS pass of the bitset build: 262,144

// Bitset rows: one block per image, its row built in LDS a chunk of words at
// a time (LDS atomics) and written out coalesced.
__global__ __launch_bounds__(1024) void bitset_rows_kernel(const int32_t* vis_off,
                                                           const int32_t* vis_pts, int64_t nnz,
                                                           int32_t n_points, int64_t words,
                                                           uint32_t* V, int32_t* err) {
  __shared__ uint32_t lds[kBitsLdsWords];
  const int32_t i = blockIdx.x;
  int64_t b, e;
  image_range(vis_off, i, nnz, b, e);
  for (int64_t w0 = 0; w0 < words; w0 += kBitsLdsWords) {
    const int64_t nw = min(int64_t(kBitsLdsWords), words - w0);
    for (int64_t w = threadIdx.x; w < nw; w += blockDim.x) lds[w] = 0u;
    __syncthreads();
    const int64_t p_lo = w0 * 32, p_hi = (w0 + nw) * 32;
    for (int64_t s = b + threadIdx.x; s < e; s += blockDim.x) {
      const int32_t p = vis_pts[s];
      if (p < 0 || p >= n_points) {
        *err = 1;
        continue;
      }
      if (p < p_lo || p >= p_hi) continue;
      atomicOr(&lds[(p >> 5) - w0], 1u << (p & 31));
    }
    __syncthreads();
    for (int64_t w = threadIdx.x; w < nw; w += blockDim.x) V[int64_t(i) * words + w0 + w] = lds[w];
    __syncthreads();
  }
}

// Gram counts of one 64 x 64 block of image pairs (block I <= block J) over
// one slice of the words: 256 threads, each a 4 x 4 sub-block held in
// registers; the two 64-row slabs of each 32-word step are staged in LDS.
// Partial counts are added into the dense n x n matrix (both (i, j) and
// (j, i)), which starts at zero.
constexpr int kGramRows = 64;
constexpr int kGramStep = 32;   // words per LDS stage
__global__ __launch_bounds__(256) void gram_kernel(const uint32_t* V, int32_t n_images,
                                                   int64_t words, int32_t nblk, int32_t slices,
                                                   int32_t* gram) {
  __shared__ uint32_t A[kGramRows][kGramStep + 1];
  __shared__ uint32_t B[kGramRows][kGramStep + 1];
  // Block (I, J) with I <= J from the linear index, then the word slice.
  const int32_t pair = int32_t(blockIdx.x) / slices, slice = int32_t(blockIdx.x) % slices;
  int32_t I = 0, rem = pair;
  while (rem >= nblk - I) {
    rem -= nblk - I;
    ++I;
  }
  const int32_t J = I + rem;
  const int64_t per = (words + slices - 1) / slices;
  const int64_t k0 = int64_t(slice) * per, k1 = min(words, k0 + per);
  const int t = threadIdx.x;
  const int tr = t >> 4, tc = t & 15;   // rows 4 tr .. 4 tr + 3 of I, 4 tc .. of J
  uint32_t acc[4][4] = {};
  for (int64_t kb = k0; kb < k1; kb += kGramStep) {
    // Stage 64 rows x 32 words of each slab (zero past the ends).
    for (int x = t; x < kGramRows * kGramStep; x += 256) {
      const int r = x / kGramStep, w = x % kGramStep;
      const int64_t k = kb + w;
      const int32_t ri = I * kGramRows + r, rj = J * kGramRows + r;
      A[r][w] = (k < k1 && ri < n_images) ? V[int64_t(ri) * words + k] : 0u;
      B[r][w] = (k < k1 && rj < n_images) ? V[int64_t(rj) * words + k] : 0u;
    }
    __syncthreads();
#pragma unroll 4
    for (int w = 0; w < kGramStep; ++w) {
      uint32_t a[4], bb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = A[4 * tr + u][w];
        bb[u] = B[4 * tc + u][w];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += __builtin_popcount(a[u] & bb[v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int32_t i = I * kGramRows + 4 * tr + u, j = J * kGramRows + 4 * tc + v;
      if (i >= n_images || j >= n_images || acc[u][v] == 0u) continue;
      if (I == J && j < i) continue;   // the diagonal block: each pair once
      atomicAdd(&gram[int64_t(i) * n_images + j], int32_t(acc[u][v]));
      if (i != j) atomicAdd(&gram[int64_t(j) * n_images + i], int32_t(acc[u][v]));
    }
  }
}

// Sets bit (min(q, c), max(q, c)) for every candidate c of every q.
__global__ __launch_bounds__(256) void pair_mark_kernel(int32_t n_images, int32_t top_k,
                                                        const int32_t* cand,
                                                        const int32_t* n_cand, uint32_t* bits,
                                                        int32_t words) {
  const int64_t total = int64_t(n_images) * top_k;
  for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total;
       x += int64_t(gridDim.x) * blockDim.x) {
    const int32_t q = int32_t(x / top_k), r = int32_t(x % top_k);
    if (r >= n_cand[q]) continue;
    const int32_t c = cand[x];
    if (c < 0 || c >= n_images || c == q) continue;
    const int32_t i = min(q, c), j = max(q, c);
    atomicOr(&bits[int64_t(i) * words + (j >> 5)], 1u << (j & 31));
  }
}

// Pairs per row i (set bits), one block per row.
__global__ __launch_bounds__(256) void pair_count_kernel(const uint32_t* bits, int32_t words,
                                                         int32_t* row_count) {
  __shared__ int32_t tot;
  if (threadIdx.x == 0) tot = 0;
  __syncthreads();
  int32_t c = 0;
  for (int32_t w = threadIdx.x; w < words; w += blockDim.x)
    c += __builtin_popcount(bits[int64_t(blockIdx.x) * words + w]);
  atomicAdd(&tot, c);
  __syncthreads();
  if (threadIdx.x == 0) row_count[blockIdx.x] = tot;
}

// Writes row i's pairs (i, j) in ascending j from its offset; one block per
// row, one thread per word (words <= kMaxCovisImages / 32 = 128).
__global__ __launch_bounds__(128) void pair_write_kernel(const uint32_t* bits, int32_t words,
                                                         const int32_t* row_off, int32_t n_images,
                                                         int32_t* pairs, int64_t* n_pairs) {
  __shared__ int32_t pre[128];
  const int32_t i = blockIdx.x;
  const int w = threadIdx.x;
  const uint32_t word = w < words ? bits[int64_t(i) * words + w] : 0u;
  pre[w] = __builtin_popcount(word);
  __syncthreads();
  if (w == 0) {
    int32_t acc = 0;
    for (int k = 0; k < 128; ++k) {
      const int32_t c = pre[k];
      pre[k] = acc;
      acc += c;
    }
  }
  __syncthreads();
  int64_t at = int64_t(row_off[i]) + pre[w];
  uint32_t m = word;
  while (m) {
    const int bit = __builtin_ctz(m);
    m &= m - 1;
    pairs[2 * at] = i;
    pairs[2 * at + 1] = 32 * w + bit;
    ++at;
  }
  if (i == n_images - 1 && w == 0) *n_pairs = int64_t(row_off[n_images]);
}

int32_t grid_for(int64_t n, int32_t per_block) {
  return int32_t(std::max<int64_t>(1, std::min<int64_t>((n + per_block - 1) / per_block, 65535)));
}

}  // namespace



hipError_t launch_candidates(const CovisArgs& a, hipStream_t st) {
  const int64_t np1 = int64_t(a.n_points) + 1;
  // Observers of every point: counts, exclusive offsets (pt_off[n_points] =
  // nnz of valid entries), scatter cursors.
  int32_t nsort = 1;
  while (nsort < a.n_images) nsort <<= 1;
  if (a.gram) {
    // Bit-matrix path: bitset rows, the Gram matrix, then each row's ranking.
    const int64_t words = (int64_t(a.n_points) + 31) / 32;
    const int64_t nn = int64_t(a.n_images) * a.n_images;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(nn, 256)), dim3(256), 0, st, a.gram, nn, 0);
    if (a.n_images > 0) {
      hipLaunchKernelGGL(bitset_rows_kernel, dim3(a.n_images), dim3(1024), 0, st, a.vis_off,
                         a.vis_pts, a.nnz, a.n_points, words, a.bitset, a.err);
      const int32_t nblk = (a.n_images + kGramRows - 1) / kGramRows;
      const int32_t pairs = nblk * (nblk + 1) / 2;
      const int32_t slices = int32_t(std::max<int64_t>(
          1, std::min<int64_t>((1024 + pairs - 1) / pairs, (words + kGramStep - 1) / kGramStep)));
      hipLaunchKernelGGL(gram_kernel, dim3(pairs * slices), dim3(256), 0, st, a.bitset,
                         a.n_images, words, nblk, slices, a.gram);
      hipLaunchKernelGGL(covis_rows_kernel, dim3(a.n_images), dim3(kCovisThreads), 0, st,
                         a.vis_off, a.vis_pts, a.nnz, a.n_images, a.n_points, a.pt_off,
                         a.pt_imgs, a.gram, a.threshold, a.top_k, nsort, a.cand, a.n_shared,
                         a.n_cand);
    }
  } else {
    // Point-histogram path: observers of every point (counts, exclusive
    // offsets, scatter), then each image's co-observers in LDS.
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(np1, 256)), dim3(256), 0, st, a.pt_count,
                       np1, 0);
    if (a.n_images > 0)
      hipLaunchKernelGGL(covis_count_kernel, dim3(a.n_images), dim3(256), 0, st, a.vis_off,
                         a.vis_pts, a.nnz, a.n_points, a.pt_count, a.err);
    if (const hipError_t e = launch_scan(a.pt_count, a.pt_off, np1, false, a.sums, a.cursor, st); e != hipSuccess)
      return e;
    if (a.n_images > 0) {
      hipLaunchKernelGGL(covis_scatter_kernel, dim3(a.n_images), dim3(256), 0, st, a.vis_off,
                         a.vis_pts, a.nnz, a.n_points, a.cursor, a.pt_imgs, a.err);
      hipLaunchKernelGGL(covis_rows_kernel, dim3(a.n_images), dim3(kCovisThreads), 0, st,
                         a.vis_off, a.vis_pts, a.nnz, a.n_images, a.n_points, a.pt_off,
                         a.pt_imgs, nullptr, a.threshold, a.top_k, nsort, a.cand, a.n_shared,
                         a.n_cand);
    }
  }
  if (a.pairs && a.n_images > 0 && a.top_k > 0) {
    const int32_t words = (a.n_images + 31) / 32;
    const int64_t nbits = int64_t(a.n_images) * words;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(nbits, 256)), dim3(256), 0, st,
                       reinterpret_cast<int32_t*>(a.bits), nbits, 0);
    hipLaunchKernelGGL(pair_mark_kernel, dim3(grid_for(int64_t(a.n_images) * a.top_k, 256)),
                       dim3(256), 0, st, a.n_images, a.top_k, a.cand, a.n_cand, a.bits, words);
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(int64_t(a.n_images) + 1, 256)), dim3(256),
                       0, st, a.row_count, int64_t(a.n_images) + 1, 0);
    hipLaunchKernelGGL(pair_count_kernel, dim3(a.n_images), dim3(256), 0, st, a.bits, words,
                       a.row_count);
    if (const hipError_t e = launch_scan(a.row_count, a.row_off, int64_t(a.n_images) + 1, false, a.sums, nullptr, st); e != hipSuccess)
      return e;
    hipLaunchKernelGGL(pair_write_kernel, dim3(a.n_images), dim3(128), 0, st, a.bits, words,
                       a.row_off, a.n_images, a.pairs, a.n_pairs);
  } else if (a.pairs && a.n_pairs) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, st,
                       reinterpret_cast<int32_t*>(a.n_pairs), 2, 0);
  }
  return hipGetLastError();
}

}  // namespace sfm
