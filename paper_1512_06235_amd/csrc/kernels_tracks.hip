// Track merging and triangulation (Section 6.3).
//
// Tracks are the connected components of the match graph: its nodes are
// observations (one feature of one image), its edges the accepted matches of
// all matched pairs.  The paper finds them with a sequential depth-first
// search; here a lock-free union-find runs over all edges at once: every
// node starts as its own root, an edge hooks the larger of its two roots
// under the smaller with a compare-and-swap, and finds halve paths as they
// go.  Parents only ever decrease, so paths terminate and each component's
// root is its smallest node id: a label independent of the order of work.
//
// Each track is then triangulated by linear least squares in FP64: an
// observation (x, y) in a camera with rows p1, p2, p3 gives the equations
// (x p3 - p1) . (X, 1) = 0 and (y p3 - p2) . (X, 1) = 0.  The members of
// every track are gathered into lists (count, scan, scatter), and one thread
// per track sums its normal equations in registers and solves them in
// closed form.
#include <algorithm>
#include <cmath>


#include "sfm_internal.h"

namespace sfm {
namespace {

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0;
}

// Parent links are read and written as device-scope atomics: another CU's
// hook must not hide behind this CU's cached copy (a stale read is still safe,
// the compare-and-swap decides, but it costs retries).
__device__ __forceinline__ int32_t load_link(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_link(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) void uf_init_kernel(int32_t* parent, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    parent[i] = int32_t(i);
}

// Root of x, halving the path on the way (each write replaces a parent by
// one of its own ancestors, so concurrent finds and hooks stay consistent).
__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t x) {
  int32_t cur = load_link(&parent[x]);
  if (cur == x) return x;
  int32_t prev = x;
  int32_t next;
  while (cur > (next = load_link(&parent[cur]))) {
    store_link(&parent[prev], next);
    prev = cur;
    cur = next;
  }
  return cur;
}

__global__ __launch_bounds__(256) void uf_union_kernel(int32_t* parent, const int32_t* edges,
                                                       int64_t n_edges, int64_t n_nodes,
                                                       int32_t* err) {
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n_edges;
       k += int64_t(gridDim.x) * blockDim.x) {
    const int32_t u = edges[2 * k], v = edges[2 * k + 1];
    if (u < 0 || v < 0 || int64_t(u) >= n_nodes || int64_t(v) >= n_nodes) {
      *err = 1;
      continue;
    }
    int32_t ru = uf_find(parent, u), rv = uf_find(parent, v);
    while (ru != rv) {
      if (ru < rv) {
        const int32_t t = ru;
        ru = rv;
        rv = t;
      }
      // Hook the larger root under the smaller; a failed swap means it got a
      // parent meanwhile: find both roots again.
      const int32_t old = atomicCAS(&parent[ru], ru, rv);
      if (old == ru) break;
      ru = uf_find(parent, old);
      rv = uf_find(parent, rv);
    }
  }
}

// Root of x without writing: the labelling pass below must not use the
// halving find, whose writes (an ancestor read before another thread stored
// its node's root) could replace a finished label by a non-root ancestor.
__device__ __forceinline__ int32_t uf_root(const int32_t* parent, int32_t x) {
  int32_t cur = x, next;
  while (cur > (next = load_link(&parent[cur]))) cur = next;
  return cur;
}

// Final labels in place: every node points straight at its root.  Each
// thread writes only its own node, and only a root, so concurrent walks see
// either the old ancestor or the root and every label ends as the root.
__global__ __launch_bounds__(256) void uf_label_kernel(int32_t* parent, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    store_link(&parent[i], uf_root(parent, int32_t(i)));
}

// Observations per track: count per root, then (after a scan) each node's
// slot in its root's member list.
__global__ __launch_bounds__(256) void tri_count_kernel(const int32_t* label,
                                                        const int32_t* node_image,
                                                        int32_t n_images, int64_t n_nodes,
                                                        int32_t* cnt, int32_t* err) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_nodes;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t r = label[i], img = node_image[i];
    if (r < 0 || int64_t(r) >= n_nodes || img < 0 || img >= n_images) {
      *err = 1;
      continue;
    }
    atomicAdd(&cnt[r], 1);
  }
}

// Skips exactly the nodes the count pass skipped, so no list overflows.
__global__ __launch_bounds__(256) void tri_scatter_kernel(const int32_t* label,
                                                          const int32_t* node_image,
                                                          int32_t n_images, int64_t n_nodes,
                                                          const int32_t* start, int32_t* fill,
                                                          int32_t* members) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_nodes;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t r = label[i], img = node_image[i];
    if (r < 0 || int64_t(r) >= n_nodes || img < 0 || img >= n_images) continue;
    members[start[r] + atomicAdd(&fill[r], 1)] = int32_t(i);
  }
}

// Per root with at least two observations: the normal equations of its
// track summed in registers over its members (each observation (x, y) in
// camera P gives the rows x p3 - p1 and y p3 - p2 of A; M = sum of the
// first three columns' outer products, b = -sum a a4), then X = M^-1 b by
// the adjugate; NaN when M is singular (all rays through one centre) or
// the track has one observation.
__global__ __launch_bounds__(256) void tri_solve_kernel(
    const int32_t* label, const int32_t* node_image, const float* node_xy, const double* P,
    int32_t n_images, int64_t n_nodes, const int32_t* start, const int32_t* cnt,
    const int32_t* members, double* X, int32_t* n_obs) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_nodes;
       i += int64_t(gridDim.x) * blockDim.x) {
    if (label[i] != int32_t(i)) {
      n_obs[i] = 0;
      continue;
    }
    const int32_t m = cnt[i];
    n_obs[i] = m;
    if (m < 2) {
      X[3 * i] = X[3 * i + 1] = X[3 * i + 2] = NAN;
      continue;
    }
    double t[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t k = start[i], e = start[i] + m; k < e; ++k) {
      const int32_t j = members[k];
      const int32_t img = node_image[j];
      if (img < 0 || img >= n_images) continue;   // flagged by the count pass
      const double* p = P + 12 * int64_t(img);
      const double x = node_xy[2 * int64_t(j)], y = node_xy[2 * int64_t(j) + 1];
      double a[2][4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        a[0][c] = x * p[8 + c] - p[c];
        a[1][c] = y * p[8 + c] - p[4 + c];
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        t[0] += a[q][0] * a[q][0];
        t[1] += a[q][0] * a[q][1];
        t[2] += a[q][0] * a[q][2];
        t[3] += a[q][1] * a[q][1];
        t[4] += a[q][1] * a[q][2];
        t[5] += a[q][2] * a[q][2];
        t[6] -= a[q][0] * a[q][3];
        t[7] -= a[q][1] * a[q][3];
        t[8] -= a[q][2] * a[q][3];
      }
    }
    const double a = t[0], b = t[1], c = t[2], d = t[3], e = t[4], f = t[5];
    const double c00 = d * f - e * e, c01 = c * e - b * f, c02 = b * e - c * d;
    const double c11 = a * f - c * c, c12 = b * c - a * e, c22 = a * d - b * b;
    const double det = a * c00 + b * c01 + c * c02;
    const double scale = fabs(a) * fabs(d) * fabs(f) + 1e-300;
    if (!(fabs(det) > 1e-12 * scale)) {
      X[3 * i] = X[3 * i + 1] = X[3 * i + 2] = NAN;
      continue;
    }
    const double r0 = t[6], r1 = t[7], r2 = t[8];
    X[3 * i] = (c00 * r0 + c01 * r1 + c02 * r2) / det;
    X[3 * i + 1] = (c01 * r0 + c11 * r1 + c12 * r2) / det;
    X[3 * i + 2] = (c02 * r0 + c12 * r1 + c22 * r2) / det;
  }
}

int32_t blocks_for(int64_t n) {
  return int32_t(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65535)));
}

}  // namespace

// The label array is the union-find's parent array.
hipError_t launch_tracks(int64_t n_nodes, const int32_t* edges, int64_t n_edges, int32_t* label,
                         int32_t* err, hipStream_t st) {
  if (n_nodes <= 0) return hipSuccess;
  hipLaunchKernelGGL(uf_init_kernel, dim3(blocks_for(n_nodes)), dim3(256), 0, st, label, n_nodes);
  if (n_edges > 0)
    hipLaunchKernelGGL(uf_union_kernel, dim3(blocks_for(n_edges)), dim3(256), 0, st, label, edges,
                       n_edges, n_nodes, err);
  hipLaunchKernelGGL(uf_label_kernel, dim3(blocks_for(n_nodes)), dim3(256), 0, st, label, n_nodes);
  return hipGetLastError();
}

hipError_t triangulate_temp_bytes(int64_t n_nodes, size_t* bytes) {
  *bytes = scan_temp_bytes(n_nodes);
  return n_nodes > scan_limit() ? hipErrorInvalidValue : hipSuccess;
}

hipError_t launch_triangulate(int64_t n_nodes, const int32_t* label, const int32_t* node_image,
                              const float* node_xy, const double* P, int32_t n_images,
                              int32_t* ws, void* temp, size_t temp_bytes, double* X,
                              int32_t* n_obs, int32_t* err, hipStream_t st) {
  if (n_nodes <= 0) return hipSuccess;
  int32_t* cnt = ws;
  int32_t* start = ws + n_nodes;
  int32_t* fill = ws + 2 * n_nodes;
  int32_t* members = ws + 3 * n_nodes;
  const dim3 grid(blocks_for(n_nodes));
  hipLaunchKernelGGL(fill_i32_kernel, grid, dim3(256), 0, st, cnt, n_nodes);
  hipLaunchKernelGGL(fill_i32_kernel, grid, dim3(256), 0, st, fill, n_nodes);
  hipLaunchKernelGGL(tri_count_kernel, grid, dim3(256), 0, st, label, node_image, n_images,
                     n_nodes, cnt, err);
  if (temp_bytes < scan_temp_bytes(n_nodes)) return hipErrorInvalidValue;
  hipError_t e = launch_scan(cnt, start, n_nodes, false, static_cast<int32_t*>(temp), nullptr, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(tri_scatter_kernel, grid, dim3(256), 0, st, label, node_image, n_images,
                     n_nodes, start, fill, members);
  hipLaunchKernelGGL(tri_solve_kernel, grid, dim3(256), 0, st, label, node_image, node_xy, P,
                     n_images, n_nodes, start, cnt, members, X, n_obs);
  return hipGetLastError();
}

}  // namespace sfm
