// Staged matching of coarse features (Section 4): the pair's first stage
// matches a prefix of the query image's features against a prefix of the
// target image's, a second stage the next run of queries against the same
// targets.  Features are registered in decreasing scale, so a prefix is the
// highest-scale part of an image; a stage is the exhaustive matcher run on
// views that point into the registered arrays, and a merge kernel places each
// pair's rows of both stages one after the other in query order.
#include <algorithm>

#include "sfm_internal.h"

namespace sfm {
namespace {

__global__ __launch_bounds__(256) void make_views_kernel(const ImageDev* images,
                                                         const int32_t* spec, int32_t n_views,
                                                         ImageDev* views) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_views;
       i += gridDim.x * blockDim.x) {
    const int32_t img = spec[3 * i], first = spec[3 * i + 1], count = spec[3 * i + 2];
    ImageDev d = images[img];
    d.xy += 2 * int64_t(first);
    d.desc += 128 * int64_t(first);
    d.norm2 += first;
    d.n = count;
    views[i] = d;
  }
}

// One workgroup per pair: copy its first-stage rows, then its second-stage
// rows with query indices moved past the first stage's queries.
__global__ __launch_bounds__(256) void merge_stages_kernel(const StageMerge* merge,
                                                           int32_t n_pairs, StageRows one,
                                                           StageRows two, int32_t* oq,
                                                           int32_t* om, int32_t* od1,
                                                           int32_t* od2, int64_t* ocmp) {
  for (int32_t p = blockIdx.x; p < n_pairs; p += gridDim.x) {
    const StageMerge M = merge[p];
    for (int32_t i = threadIdx.x; i < M.n1; i += blockDim.x) {
      const int64_t s = M.src1 + i, d = M.dst + i;
      oq[d] = one.q[s];
      om[d] = one.m[s];
      od1[d] = one.d1[s];
      od2[d] = one.d2[s];
    }
    for (int32_t i = threadIdx.x; i < M.n2; i += blockDim.x) {
      const int64_t s = M.src2 + i, d = M.dst + M.n1 + i;
      oq[d] = two.q[s] + M.shift;
      om[d] = two.m[s];
      od1[d] = two.d1[s];
      od2[d] = two.d2[s];
    }
    if (threadIdx.x == 0 && ocmp) ocmp[p] = one.n_cmp[p] + (M.s2 >= 0 ? two.n_cmp[M.s2] : 0);
  }
}

int32_t grid_for(int64_t n, int64_t per) {
  return int32_t(std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, 65535)));
}

}  // namespace

hipError_t launch_make_views(const ImageDev* images, const int32_t* spec, int32_t n_views,
                             ImageDev* views, hipStream_t st) {
  if (n_views <= 0) return hipSuccess;
  hipLaunchKernelGGL(make_views_kernel, dim3(grid_for(n_views, 256)), dim3(256), 0, st, images,
                     spec, n_views, views);
  return hipGetLastError();
}

hipError_t launch_merge_stages(const StageMerge* merge, int32_t n_pairs, StageRows one,
                               StageRows two, int32_t* out_q, int32_t* out_m, int32_t* out_d1,
                               int32_t* out_d2, int64_t* out_cmp, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(merge_stages_kernel, dim3(grid_for(n_pairs, 1)), dim3(256), 0, st, merge,
                     n_pairs, one, two, out_q, out_m, out_d1, out_d2, out_cmp);
  return hipGetLastError();
}

}  // namespace sfm
