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
// (x p3 - p1) . (X, 1) = 0 and (y p3 - p2) . (X, 1) = 0; the normal
// equations of X are summed per track and solved in closed form.
#include <algorithm>
#include <cmath>

#include "sfm_internal.h"

namespace sfm {
namespace {

__global__ __launch_bounds__(256) void fill_f64_kernel(double* p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
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

// Per observation: its two equations' contributions to the normal equations
// of its track (root r = label[i]): acc[10 r ..] = the upper triangle of
// M = sum a a^T over the first three coefficients (6), the right side
// sum -a a4 (3), and the number of observations.
__global__ __launch_bounds__(256) void tri_accumulate_kernel(
    const int32_t* label, const int32_t* node_image, const float* node_xy, const double* P,
    int32_t n_images, int64_t n_nodes, double* acc, int32_t* err) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_nodes;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t r = label[i], img = node_image[i];
    if (r < 0 || int64_t(r) >= n_nodes || img < 0 || img >= n_images) {
      *err = 1;
      continue;
    }
    const double* p = P + 12 * int64_t(img);
    const double x = node_xy[2 * i], y = node_xy[2 * i + 1];
    double a[2][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      a[0][c] = x * p[8 + c] - p[c];
      a[1][c] = y * p[8 + c] - p[4 + c];
    }
    double m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      m[0] += a[e][0] * a[e][0];
      m[1] += a[e][0] * a[e][1];
      m[2] += a[e][0] * a[e][2];
      m[3] += a[e][1] * a[e][1];
      m[4] += a[e][1] * a[e][2];
      m[5] += a[e][2] * a[e][2];
      m[6] -= a[e][0] * a[e][3];
      m[7] -= a[e][1] * a[e][3];
      m[8] -= a[e][2] * a[e][3];
    }
    double* t = acc + 10 * int64_t(r);
#pragma unroll
    for (int c = 0; c < 9; ++c) atomicAdd(&t[c], m[c]);
    atomicAdd(&t[9], 1.0);
  }
}

// Per root with at least two observations: X = M^-1 b by the adjugate; NaN
// when M is singular (all rays through one centre, or one observation).
__global__ __launch_bounds__(256) void tri_solve_kernel(const int32_t* label, const double* acc,
                                                        int64_t n_nodes, double* X,
                                                        int32_t* n_obs) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_nodes;
       i += int64_t(gridDim.x) * blockDim.x) {
    if (label[i] != int32_t(i)) {
      n_obs[i] = 0;
      continue;
    }
    const double* t = acc + 10 * i;
    const double a = t[0], b = t[1], c = t[2], d = t[3], e = t[4], f = t[5];
    const double c00 = d * f - e * e, c01 = c * e - b * f, c02 = b * e - c * d;
    const double c11 = a * f - c * c, c12 = b * c - a * e, c22 = a * d - b * b;
    const double det = a * c00 + b * c01 + c * c02;
    const int32_t n = int32_t(t[9]);
    n_obs[i] = n;
    const double scale = fabs(a) * fabs(d) * fabs(f) + 1e-300;
    if (n < 2 || !(fabs(det) > 1e-12 * scale)) {
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

hipError_t launch_triangulate(int64_t n_nodes, const int32_t* label, const int32_t* node_image,
                              const float* node_xy, const double* P, int32_t n_images,
                              double* acc, double* X, int32_t* n_obs, int32_t* err,
                              hipStream_t st) {
  if (n_nodes <= 0) return hipSuccess;
  const int64_t n_acc = 10 * n_nodes;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(blocks_for(n_acc)), dim3(256), 0, st, acc, n_acc);
  hipLaunchKernelGGL(tri_accumulate_kernel, dim3(blocks_for(n_nodes)), dim3(256), 0, st, label,
                     node_image, node_xy, P, n_images, n_nodes, acc, err);
  hipLaunchKernelGGL(tri_solve_kernel, dim3(blocks_for(n_nodes)), dim3(256), 0, st, label, acc,
                     n_nodes, X, n_obs);
  return hipGetLastError();
}

}  // namespace sfm
