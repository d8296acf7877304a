// C ABI of libsfmgm: context, image registration, workspace and the launch
// sequences of the plain, batched and exhaustive forms.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sfm_gm.h"
#include "sfm_internal.h"

using namespace sfm;

// Scratch of sfm_guided_match_noalloc, one copy per GPU, held until the
// process ends.  In host code the name stands for a host-side shadow, never
// for device memory: host code uses the address hipGetSymbolAddress returns
// for the current device (ScratchDevice::ptr below).
static __device__ __align__(256) char scratch[SFM_NOALLOC_SCRATCH_BYTES];

// Writes offset[0] = 0: the output of a call without pairs.
__global__ void zero_offset_kernel(int64_t* offset) {
  if (threadIdx.x == 0) offset[0] = 0;
}

struct sfm_ctx {
  int32_t device = 0;
  int32_t group_tiles = kDefaultGroupTiles;          // query tiles per match workgroup
  int32_t features_per_bin = kDefaultFeaturesPerBin; // target features per bin of b
  size_t budget = 0;
  std::string last_error;
  std::mutex mu;

  // Registered images.
  int32_t n_images = 0;
  std::vector<int32_t> n_host;
  std::vector<float> bbox_host;        // 4 per image: min x, min y, max x, max y
  ImageDev* images_dev = nullptr;
  int32_t* norm2_dev = nullptr;
  int64_t* norm_off_dev = nullptr;

  // Workspace and its host staging.
  char* ws = nullptr;
  size_t ws_cap = 0;
  char* pinned = nullptr;
  size_t pinned_cap = 0;
  hipEvent_t staging_done = nullptr;   // last copy out of the pinned buffer
  hipEvent_t work_done = nullptr;      // end of the last matching call
  int32_t* err_dev = nullptr;
  char* noalloc_scratch = nullptr;     // this device's `scratch` (device address)
  unsigned long long* diag_dev = nullptr;   // sfm_band_error's two result words
  bool has_work = false;
  int32_t last_pairs = 0;              // pairs of the last matching call
  size_t last_counters = 0;            // workspace offset of its counters

  // Staged matching: view table, per-stage rows and merge plan.
  char* stage_buf = nullptr;
  size_t stage_cap = 0;

  // Phase timing: 4 events per record (start, after prepare, after match, end).
  bool profiling = false;
  std::vector<hipEvent_t> prof_events;
  std::vector<hipEvent_t> prof_pool;

  // Graph replay of the batched form (sfm_set_graph_replay, off by default):
  // the kernels of one launch layout are captured once the layout repeats
  // and replayed while it keeps repeating.
  bool graph_replay = false;
  std::vector<char> last_key;   // layout of the last batched call launched directly
  int32_t covis_method = 0;   // candidate images: 0 choose, 1 point histogram, 2 bit matrix
  double grid_group_px = 0.0; // grid search: query grouping distance (0 = off)
  int32_t grid_group_leader = 0;  // grouping against the group's first line
  int64_t last_groups = 0;    // query groups of the last grouped grid call
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  std::vector<char> graph_key;
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int fail(sfm_ctx* ctx, int status, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return status;
}

// The message is cut to the capacity last_error was given at creation, so
// this form never allocates.
int fail(sfm_ctx* ctx, int status, const char* msg) {
  if (ctx) ctx->last_error.assign(msg, strnlen(msg, ctx->last_error.capacity()));
  return status;
}

int hip_fail(sfm_ctx* ctx, hipError_t e, const char* what) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
  return fail(ctx, e == hipErrorOutOfMemory ? SFM_ENOMEM : SFM_EHIP, buf);
}

#define HIP_TRY(ctx, expr)                                   \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return hip_fail((ctx), _e, #expr); \
  } while (0)

// Sections of one call's workspace.
struct Layout {
  size_t pairs, F, order, items, geom, counters, wg_start, cand_x, cand_y, cand_nc, cand_j, bins,
      qrec, res, twin, groups, gcost, pcost, part, total, staged;
  int32_t wgs = 0;
  int64_t sum_na = 0, sum_nc = 0, sum_bins = 0, sum_blocks = 0, sum_groups = 0;
  int32_t max_na = 0, max_nb = 0;
};

int32_t bins_for(int32_t nb, int32_t features_per_bin) {
  return std::max<int32_t>(1, std::min<int32_t>(kMaxBins, nb / features_per_bin));
}

// n_items and n_part: the exhaustive form's work items (staged with the pair
// table) and partial results; 0 for the other forms.
Layout plan(const PairDesc* pd, size_t P, int32_t device, int32_t group_tiles,
            int64_t n_items = 0, int64_t n_part = 0) {
  Layout L;
  for (size_t k = 0; k < P; ++k) {
    const PairDesc& p = pd[k];
    L.sum_na += p.na;
    L.max_na = std::max(L.max_na, p.na);
    L.max_nb = std::max(L.max_nb, p.nb);
    L.sum_nc += p.nb + kCandPad;
    L.sum_bins += p.nbins + 1;
    L.sum_blocks += p.nblocks;
    L.sum_groups += p.ngroups;
  }
  size_t o = 0;
  L.pairs = o; o = align_up(o + P * sizeof(PairDesc));
  L.F = o; o = align_up(o + P * 9 * sizeof(double));
  L.order = o; o = align_up(o + P * sizeof(int32_t));
  L.items = o; o = align_up(o + size_t(n_items) * sizeof(int2));
  L.staged = o;
  L.geom = o; o = align_up(o + P * sizeof(PairGeom));
  L.counters = o; o = align_up(o + P * sizeof(PairCounters));
  L.wgs = match_workgroups(device, group_tiles, L.sum_groups);
  L.wg_start = o; o = align_up(o + size_t(L.wgs + 1) * sizeof(int32_t));
  L.cand_x = o; o = align_up(o + size_t(L.sum_nc) * sizeof(float));
  L.cand_y = o; o = align_up(o + size_t(L.sum_nc) * sizeof(float));
  L.cand_nc = o; o = align_up(o + size_t(L.sum_nc) * sizeof(uint32_t));
  L.cand_j = o; o = align_up(o + size_t(L.sum_nc) * sizeof(int32_t));
  L.bins = o; o = align_up(o + size_t(L.sum_bins) * sizeof(int32_t));
  L.qrec = o; o = align_up(o + size_t(L.sum_na) * sizeof(QueryRec));
  L.res = o; o = align_up(o + size_t(L.sum_na) * sizeof(QueryResult));
  L.twin = o; o = align_up(o + size_t(L.sum_blocks) * sizeof(int2));
  L.groups = o; o = align_up(o + size_t(L.sum_groups) * sizeof(TileGroup));
  L.gcost = o; o = align_up(o + size_t(L.sum_groups) * sizeof(int32_t));
  L.pcost = o; o = align_up(o + P * sizeof(long long));
  L.part = o; o = align_up(o + size_t(n_part) * sizeof(uint2));
  L.total = o;
  return L;
}

Layout plan(const std::vector<PairDesc>& pd, int32_t device, int32_t group_tiles,
            int64_t n_items = 0, int64_t n_part = 0) {
  return plan(pd.data(), pd.size(), device, group_tiles, n_items, n_part);
}

// The images pairs refer to: the registered ones, or views of them (a run of
// consecutive features of one image) built for a staged match.
struct ImageTable {
  const ImageDev* dev;   // device table
  const int32_t* n;      // host copy of the feature counts
  int32_t count;
};

ImageTable registered(const sfm_ctx* ctx) {
  return ImageTable{ctx->images_dev, ctx->n_host.data(), ctx->n_images};
}

// Fills pd[0 .. n_pairs) (room for n_pairs descriptors).
int describe_pairs(sfm_ctx* ctx, const ImageTable& tab, const sfm_pair* pairs, int32_t n_pairs,
                   bool ignore_band, PairDesc* pd) {
  if (n_pairs < 0) return fail(ctx, SFM_EINVAL, "n_pairs < 0");
  if (n_pairs > 0 && !pairs) return fail(ctx, SFM_EINVAL, "pairs is NULL");
  int64_t q = 0, c = 0, bo = 0, blk = 0, grp = 0;
  for (int32_t k = 0; k < n_pairs; ++k) {
    const sfm_pair& s = pairs[k];
    if (s.a < 0 || s.a >= tab.count || s.b < 0 || s.b >= tab.count) {
      char buf[128];
      snprintf(buf, sizeof buf, "pair %d: image index out of range (a=%d b=%d, %d registered)", k,
               s.a, s.b, tab.count);
      return fail(ctx, SFM_EINVAL, buf);
    }
    if (!ignore_band && !(s.band_px >= 0.0)) {
      char buf[96];
      snprintf(buf, sizeof buf, "pair %d: band_px must be >= 0 (got %g)", k, s.band_px);
      return fail(ctx, SFM_EINVAL, buf);
    }
    PairDesc& p = pd[k];
    memset(&p, 0, sizeof p);
    p.a = s.a;
    p.b = s.b;
    p.na = tab.n[s.a];
    p.nb = tab.n[s.b];
    p.nbins = ignore_band ? 1 : bins_for(p.nb, ctx->features_per_bin);
    p.nblocks = (p.na + kQueryTile - 1) / kQueryTile;
    p.ngroups = (p.nblocks + ctx->group_tiles - 1) / ctx->group_tiles;
    p.q_off = q;
    p.c_off = c;
    p.bin_off = bo;
    p.blk_off = blk;
    p.grp_off = grp;
    p.band = ignore_band ? INFINITY : s.band_px;
    p.ignore_band = ignore_band ? 1 : 0;
    q += p.na;
    c += p.nb + kCandPad;
    bo += p.nbins + 1;
    blk += p.nblocks;
    grp += p.ngroups;
  }
  if (blk > INT32_MAX / 2) return fail(ctx, SFM_ECAPACITY, "too many query tiles in one call");
  return SFM_OK;
}

int describe_pairs(sfm_ctx* ctx, const ImageTable& tab, const sfm_pair* pairs, int32_t n_pairs,
                   bool ignore_band, std::vector<PairDesc>& pd) {
  if (n_pairs < 0) return fail(ctx, SFM_EINVAL, "n_pairs < 0");
  pd.resize(size_t(n_pairs));
  return describe_pairs(ctx, tab, pairs, n_pairs, ignore_band, pd.data());
}

// A device workspace, its pinned staging buffer and their events: the
// context's own, or one of a server's slots (serve_space_create), which lets
// launches of different slots overlap on the device.
struct Space {
  char** ws;
  size_t* ws_cap;
  char** pinned;
  size_t* pinned_cap;
  hipEvent_t staging_done;   // last copy out of the pinned buffer
  hipEvent_t work_done;      // end of the last call on the workspace
  bool* has_work;
  size_t budget;
};

Space ctx_space(sfm_ctx* ctx) {
  return Space{&ctx->ws,          &ctx->ws_cap,    &ctx->pinned,   &ctx->pinned_cap,
               ctx->staging_done, ctx->work_done,  &ctx->has_work, ctx->budget};
}

int ensure_ws(sfm_ctx* ctx, const Space& sp, size_t bytes) {
  if (bytes > sp.budget) {
    char buf[160];
    snprintf(buf, sizeof buf, "workspace of %zu bytes exceeds the budget of %zu bytes", bytes,
             sp.budget);
    return fail(ctx, SFM_ECAPACITY, buf);
  }
  if (bytes <= *sp.ws_cap) return SFM_OK;
  if (*sp.has_work) HIP_TRY(ctx, hipEventSynchronize(sp.work_done));
  if (*sp.ws) HIP_TRY(ctx, hipFree(*sp.ws));
  *sp.ws = nullptr;
  *sp.ws_cap = 0;
  const size_t cap = std::min(sp.budget, std::max(bytes, bytes + bytes / 4));
  HIP_TRY(ctx, hipMalloc(sp.ws, cap));
  *sp.ws_cap = cap;
  return SFM_OK;
}

int ensure_pin(sfm_ctx* ctx, const Space& sp, size_t bytes) {
  if (bytes <= *sp.pinned_cap) return SFM_OK;
  HIP_TRY(ctx, hipEventSynchronize(sp.staging_done));
  if (*sp.pinned) HIP_TRY(ctx, hipHostFree(*sp.pinned));
  *sp.pinned = nullptr;
  *sp.pinned_cap = 0;
  const size_t cap = std::max<size_t>(bytes, 1 << 16);
  HIP_TRY(ctx, hipHostMalloc(reinterpret_cast<void**>(sp.pinned), cap, hipHostMallocDefault));
  *sp.pinned_cap = cap;
  return SFM_OK;
}

int ensure_workspace(sfm_ctx* ctx, size_t bytes) { return ensure_ws(ctx, ctx_space(ctx), bytes); }
int ensure_pinned(sfm_ctx* ctx, size_t bytes) { return ensure_pin(ctx, ctx_space(ctx), bytes); }

enum class Form { kBatched, kPlain, kExhaustive, kBandError };

sfm_options default_options() {
  sfm_options o;
  memset(&o, 0, sizeof o);
  o.ratio_num = 64;
  o.ratio_den = 100;
  o.recheck_margin_px = 1e-3;
  return o;
}

int check_options(sfm_ctx* ctx, const sfm_options& opt) {
  if (opt.ratio_den <= 0 || opt.ratio_num < 0)
    return fail(ctx, SFM_EINVAL, "ratio_den must be > 0 and ratio_num >= 0");
  if (!(opt.recheck_margin_px >= 0.0) || !std::isfinite(opt.recheck_margin_px))
    return fail(ctx, SFM_EINVAL, "recheck_margin_px must be finite and >= 0");
  return SFM_OK;
}

// Everything the batched form's kernels take: a graph captured for one Key
// is valid for every call with the same Key.
struct GraphKey {
  BatchView v;
  sfm_matches out;
  int32_t n_pairs, sum_groups, wgs, max_na;
  const int32_t* order;
};

// Enqueues the batched form's kernels on `st` by replaying the graph of this
// key, capturing (on a private stream) and instantiating it first when the
// key differs from the last one.  The staging copy stays outside the graph,
// so the host may prepare the next call while this one runs.
int replay_batched(sfm_ctx* ctx, const GraphKey& key, int32_t* am, int32_t* ad1, int32_t* ad2,
                   int32_t* ac, hipStream_t st) {
  const char* kb = reinterpret_cast<const char*>(&key);
  if (!ctx->graph || ctx->graph_key.size() != sizeof key ||
      memcmp(ctx->graph_key.data(), kb, sizeof key) != 0) {
    if (ctx->graph) HIP_TRY(ctx, hipGraphExecDestroy(ctx->graph));
    ctx->graph = nullptr;
    ctx->graph_key.clear();
    if (!ctx->cap_stream)
      HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = ctx->cap_stream;
    const BatchView& v = key.v;
    const sfm_matches& out = key.out;
    HIP_TRY(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const hipError_t e1 = launch_prepare(v, 0, key.n_pairs, 0, key.sum_groups, key.wgs, key.order,
                                         key.max_na, cs);
    const hipError_t e2 = launch_match(v, key.sum_groups > 0 ? key.wgs : 0, cs);
    const hipError_t e3 = launch_emit(v, 0, key.n_pairs, out.offset, out.query, out.match, out.d1,
                                      out.d2, out.n_comparisons, out.n_borderline, am, ad1, ad2, ac, cs);
    hipGraph_t g = nullptr;
    HIP_TRY(ctx, hipStreamEndCapture(cs, &g));
    const hipError_t ei = (e1 != hipSuccess)   ? e1
                          : (e2 != hipSuccess) ? e2
                          : (e3 != hipSuccess) ? e3
                                               : hipGraphInstantiate(&ctx->graph, g, nullptr,
                                                                     nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(ctx, ei);
    ctx->graph_key.assign(kb, kb + sizeof key);
  }
  HIP_TRY(ctx, hipGraphLaunch(ctx->graph, st));
  return SFM_OK;
}

// True when `key` is the captured graph's layout or the last directly
// launched batched call's.
bool key_repeats(const sfm_ctx* ctx, const GraphKey& key) {
  const char* kb = reinterpret_cast<const char*>(&key);
  const auto same = [&](const std::vector<char>& k) {
    return k.size() == sizeof key && memcmp(k.data(), kb, sizeof key) == 0;
  };
  return (ctx->graph && same(ctx->graph_key)) || same(ctx->last_key);
}

// Records an event on `st` when profiling is enabled.
hipError_t prof_mark(sfm_ctx* ctx, hipStream_t st) {
  if (!ctx->profiling) return hipSuccess;
  hipEvent_t e;
  if (!ctx->prof_pool.empty()) {
    e = ctx->prof_pool.back();
    ctx->prof_pool.pop_back();
  } else {
    const hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
  }
  ctx->prof_events.push_back(e);
  return hipEventRecord(e, st);
}

// Every pair's F must be finite and not all zero.
int check_F(sfm_ctx* ctx, const double* F, int32_t n_pairs) {
  if (n_pairs > 0 && !F) return fail(ctx, SFM_EINVAL, "F is NULL");
  for (int32_t k = 0; k < n_pairs; ++k) {
    bool nonzero = false;
    for (int t = 0; t < 9; ++t) {
      const double f = F[9 * size_t(k) + size_t(t)];
      if (!std::isfinite(f)) {
        char buf[64];
        snprintf(buf, sizeof buf, "pair %d: F is not finite", k);
        return fail(ctx, SFM_EINVAL, buf);
      }
      nonzero |= f != 0.0;
    }
    if (!nonzero) {
      char buf[64];
      snprintf(buf, sizeof buf, "pair %d: F is all zero", k);
      return fail(ctx, SFM_EINVAL, buf);
    }
  }
  return SFM_OK;
}

// Output checks of the matching forms.
int check_outputs(sfm_ctx* ctx, const sfm_matches* out, const Layout& L, const sfm_options& opt) {
  if (!out->offset) return fail(ctx, SFM_EINVAL, "out->offset is NULL");
  if (out->capacity < L.sum_na) {
    char buf[128];
    snprintf(buf, sizeof buf, "output capacity %lld < %lld queries", (long long)out->capacity,
             (long long)L.sum_na);
    return fail(ctx, SFM_ECAPACITY, buf);
  }
  if (L.sum_na > 0 && (!out->query || !out->match || !out->d1 || !out->d2))
    return fail(ctx, SFM_EINVAL, "output arrays are NULL");
  if (opt.emit_all && L.sum_na > 0 &&
      (!out->all_match || !out->all_d1 || !out->all_d2 || !out->all_count))
    return fail(ctx, SFM_EINVAL, "emit_all needs all_match, all_d1, all_d2 and all_count");
  return SFM_OK;
}

// The kernels' view of one call whose workspace sections (plan()) start at `ws`.
BatchView batch_view(const sfm_ctx* ctx, const ImageTable& tab, char* ws, const Layout& L,
                     int32_t n_pairs, const sfm_options& opt) {
  BatchView v;
  memset(&v, 0, sizeof v);   // padding too: graph keys compare the bytes
  v.images = tab.dev;
  v.pairs = reinterpret_cast<const PairDesc*>(ws + L.pairs);
  v.F = reinterpret_cast<const double*>(ws + L.F);
  v.geom = reinterpret_cast<PairGeom*>(ws + L.geom);
  v.counters = reinterpret_cast<PairCounters*>(ws + L.counters);
  v.cand_x = reinterpret_cast<float*>(ws + L.cand_x);
  v.cand_y = reinterpret_cast<float*>(ws + L.cand_y);
  v.cand_nc = reinterpret_cast<uint32_t*>(ws + L.cand_nc);
  v.cand_j = reinterpret_cast<int32_t*>(ws + L.cand_j);
  v.bin_start = reinterpret_cast<int32_t*>(ws + L.bins);
  v.qrec = reinterpret_cast<QueryRec*>(ws + L.qrec);
  v.res = reinterpret_cast<QueryResult*>(ws + L.res);
  v.twin = reinterpret_cast<int2*>(ws + L.twin);
  v.wg_start = reinterpret_cast<int32_t*>(ws + L.wg_start);
  v.gcost = reinterpret_cast<int32_t*>(ws + L.gcost);
  v.pcost = reinterpret_cast<long long*>(ws + L.pcost);
  v.err = ctx->err_dev;
  v.n_pairs = n_pairs;
  v.total_blocks = int32_t(L.sum_blocks);
  v.ratio_num = opt.ratio_num;
  v.ratio_den = opt.ratio_den;
  v.accept_single = opt.accept_single ? 1 : 0;
  v.keep_counts = opt.emit_all ? 1 : 0;
  v.group_tiles = ctx->group_tiles;
  v.max_na = L.max_na;
  v.max_nb = L.max_nb;
  v.margin = opt.recheck_margin_px;
  v.groups = reinterpret_cast<TileGroup*>(ws + L.groups);
  return v;
}

// Binning takes the largest pairs first, so small ones fill the tail; equal
// sizes keep the caller's order.  In place (std::sort allocates nothing).
void binning_order(const PairDesc* pd, int32_t n_pairs, int32_t* ord) {
  for (int32_t k = 0; k < n_pairs; ++k) ord[k] = k;
  std::sort(ord, ord + n_pairs, [&](int32_t x, int32_t y) {
    const int32_t sx = std::max(pd[x].na, pd[x].nb), sy = std::max(pd[y].na, pd[y].nb);
    return sx != sy ? sx > sy : x < y;
  });
}

// One matching call over the images of `tab`; the caller holds ctx->mu.
// kBandError runs the preparation and the FP32-accuracy diagnostic instead
// of matching (`out` is unused; diag receives the two result words).
int match_locked(sfm_ctx* ctx, const ImageTable& tab, const sfm_pair* pairs, int32_t n_pairs,
                 const double* F, const sfm_options* opt_in, const sfm_matches* out, void* stream,
                 Form form, unsigned long long* diag = nullptr, const Space* alt = nullptr) {
  const Space S = alt ? *alt : ctx_space(ctx);
  const bool diagnostic = form == Form::kBandError;
  sfm_matches none;
  memset(&none, 0, sizeof none);
  if (diagnostic) out = &none;
  if (!out) return fail(ctx, SFM_EINVAL, "out is NULL");
  sfm_options opt = default_options();
  if (opt_in) opt = *opt_in;
  int rc = check_options(ctx, opt);
  if (rc) return rc;
  const bool exhaustive = form == Form::kExhaustive;
  std::vector<PairDesc> pd;
  rc = describe_pairs(ctx, tab, pairs, n_pairs, exhaustive, pd);
  if (rc) return rc;
  if (!exhaustive && (rc = check_F(ctx, F, n_pairs))) return rc;
  int64_t n_items = 0, n_part = 0;
  if (exhaustive) {
    for (int32_t k = 0; k < n_pairs; ++k) {
      if (pd[size_t(k)].na > kExhaustiveMaxQueries || pd[size_t(k)].nb > kExhaustiveMaxTargets) {
        char buf[160];
        snprintf(buf, sizeof buf,
                 "pair %d: exhaustive matching takes at most %d queries and %d targets", k,
                 kExhaustiveMaxQueries, kExhaustiveMaxTargets);
        return fail(ctx, SFM_ECAPACITY, buf);
      }
    }
    exhaustive_plan(pd.data(), n_pairs, nullptr, &n_items, &n_part);
    if (n_items > INT32_MAX) return fail(ctx, SFM_ECAPACITY, "too many work items in one call");
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const Layout L = plan(pd, ctx->device, ctx->group_tiles, n_items, n_part);
  if (!diagnostic && (rc = check_outputs(ctx, out, L, opt))) return rc;
  if (diagnostic && opt.emit_all) return fail(ctx, SFM_EINVAL, "emit_all has no outputs here");

  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (n_pairs == 0) {
    if (!diagnostic) HIP_TRY(ctx, hipMemsetAsync(out->offset, 0, sizeof(int64_t), st));
    return SFM_OK;
  }
  if ((rc = ensure_ws(ctx, S, L.total))) return rc;
  if ((rc = ensure_pin(ctx, S, L.staged))) return rc;
  // Calls on one context are ordered: wait for the previous one on this stream.
  if (*S.has_work) HIP_TRY(ctx, hipStreamWaitEvent(st, S.work_done, 0));

  HIP_TRY(ctx, hipEventSynchronize(S.staging_done));
  memcpy((*S.pinned) + L.pairs, pd.data(), pd.size() * sizeof(PairDesc));
  if (exhaustive) {
    memset((*S.pinned) + L.F, 0, pd.size() * 9 * sizeof(double));
    exhaustive_plan(pd.data(), n_pairs, reinterpret_cast<int2*>((*S.pinned) + L.items), &n_items,
                    &n_part);
  } else {
    memcpy((*S.pinned) + L.F, F, pd.size() * 9 * sizeof(double));
  }
  binning_order(pd.data(), n_pairs, reinterpret_cast<int32_t*>((*S.pinned) + L.order));
  HIP_TRY(ctx, hipMemcpyAsync((*S.ws), (*S.pinned), L.staged, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipEventRecord(S.staging_done, st));

  const BatchView v = batch_view(ctx, tab, (*S.ws), L, n_pairs, opt);

  // The layout of a batched call, for graph replay.
  const bool replay = !alt && ctx->graph_replay && !ctx->profiling && form == Form::kBatched;
  GraphKey key;
  memset(&key, 0, sizeof key);
  if (replay) {
    key.v = v;
    key.out = *out;
    key.n_pairs = n_pairs;
    key.sum_groups = int32_t(L.sum_groups);
    key.wgs = L.wgs;
    for (const PairDesc& pp : pd) key.max_na = std::max(key.max_na, pp.na);
    key.order = reinterpret_cast<const int32_t*>((*S.ws) + L.order);
    if (!opt.emit_all) {
      key.out.all_match = key.out.all_d1 = key.out.all_d2 = key.out.all_count = nullptr;
    }
  }
  int32_t* am = opt.emit_all ? out->all_match : nullptr;
  int32_t* ad1 = opt.emit_all ? out->all_d1 : nullptr;
  int32_t* ad2 = opt.emit_all ? out->all_d2 : nullptr;
  int32_t* ac = opt.emit_all ? out->all_count : nullptr;
  if (diagnostic) {
    int32_t max_na = 0;
    for (const PairDesc& pp : pd) max_na = std::max(max_na, pp.na);
    HIP_TRY(ctx, hipMemsetAsync(diag, 0, 2 * sizeof(unsigned long long), st));
    HIP_TRY(ctx, launch_prepare(v, 0, n_pairs, 0, int32_t(L.sum_groups), L.wgs,
                                reinterpret_cast<const int32_t*>((*S.ws) + L.order), max_na, st));
    HIP_TRY(ctx, launch_band_error(v, L.sum_groups, diag, st));
  } else if (form == Form::kPlain) {
    for (int32_t p = 0; p < n_pairs; ++p) {
      HIP_TRY(ctx, prof_mark(ctx, st));
      const int32_t g0 = int32_t(pd[size_t(p)].grp_off), gn = pd[size_t(p)].ngroups;
      const int32_t wgs = match_workgroups(ctx->device, ctx->group_tiles, gn);
      HIP_TRY(ctx, launch_prepare(v, p, 1, g0, gn, wgs, nullptr, pd[size_t(p)].na, st));
      HIP_TRY(ctx, prof_mark(ctx, st));
      HIP_TRY(ctx, launch_match(v, gn > 0 ? wgs : 0, st));
      HIP_TRY(ctx, prof_mark(ctx, st));
      HIP_TRY(ctx, launch_emit(v, p, 1, out->offset, out->query, out->match, out->d1, out->d2,
                               out->n_comparisons, out->n_borderline, am, ad1, ad2, ac, st));
      HIP_TRY(ctx, prof_mark(ctx, st));
    }
  } else if (exhaustive) {
    // No preparation: the exhaustive kernels read the images directly and
    // leave the index in b (emission maps nothing).
    BatchView ve = v;
    ve.cand_j = nullptr;
    HIP_TRY(ctx, prof_mark(ctx, st));
    HIP_TRY(ctx, prof_mark(ctx, st));
    HIP_TRY(ctx, launch_exhaustive(ve, reinterpret_cast<const int2*>((*S.ws) + L.items), n_items,
                                   reinterpret_cast<uint2*>((*S.ws) + L.part), st));
    HIP_TRY(ctx, prof_mark(ctx, st));
    HIP_TRY(ctx, launch_emit(ve, 0, n_pairs, out->offset, out->query, out->match, out->d1,
                             out->d2, out->n_comparisons, out->n_borderline, am, ad1, ad2, ac,
                             st));
    HIP_TRY(ctx, prof_mark(ctx, st));
  } else if (replay && key_repeats(ctx, key)) {
    if ((rc = replay_batched(ctx, key, am, ad1, ad2, ac, st))) return rc;
  } else {
    // A layout seen for the first time launches directly; the next call with
    // the same layout is captured and replayed.
    if (replay) {
      const char* kb = reinterpret_cast<const char*>(&key);
      ctx->last_key.assign(kb, kb + sizeof key);
    }
    HIP_TRY(ctx, prof_mark(ctx, st));
    int32_t max_na = 0;
    for (const PairDesc& pp : pd) max_na = std::max(max_na, pp.na);
    HIP_TRY(ctx, launch_prepare(v, 0, n_pairs, 0, int32_t(L.sum_groups), L.wgs,
                                reinterpret_cast<const int32_t*>((*S.ws) + L.order), max_na, st));
    HIP_TRY(ctx, prof_mark(ctx, st));
    HIP_TRY(ctx, launch_match(v, L.sum_groups > 0 ? L.wgs : 0, st));
    HIP_TRY(ctx, prof_mark(ctx, st));
    HIP_TRY(ctx, launch_emit(v, 0, n_pairs, out->offset, out->query, out->match, out->d1,
                             out->d2, out->n_comparisons, out->n_borderline, am, ad1, ad2, ac,
                             st));
    HIP_TRY(ctx, prof_mark(ctx, st));
  }
  HIP_TRY(ctx, hipEventRecord(S.work_done, st));
  *S.has_work = true;
  // sfm_last_stats reads the counters from the context workspace only.
  ctx->last_pairs = alt ? 0 : n_pairs;
  ctx->last_counters = L.counters;
  return SFM_OK;
}

int run_match(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
              const sfm_options* opt, const sfm_matches* out, void* stream, Form form) {
  if (!ctx) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  return match_locked(ctx, registered(ctx), pairs, n_pairs, F, opt, out, stream, form);
}

// sfm_guided_match_noalloc: the batched form on the device's `scratch`
// array, with the pair table, F and binning order staged in a process-wide
// host buffer instead of the context's workspace and pinned buffer.

constexpr int kMaxScratchDevices = 64;
// plan()'s staged prefix (pairs, F, order) at the most pairs a call takes.
constexpr size_t kNoAllocStageBytes =
    3 * kAlign +
    size_t(SFM_NOALLOC_MAX_PAIRS) * (sizeof(PairDesc) + 9 * sizeof(double) + sizeof(int32_t));

struct ScratchDevice {
  char* ptr = nullptr;           // device address of this GPU's `scratch`
  hipEvent_t staged = nullptr;   // after the last staging copy issued on this GPU
  hipEvent_t done = nullptr;     // after the last call's kernels on this GPU
  bool has_done = false;
};
ScratchDevice g_scratch[kMaxScratchDevices];
std::mutex g_scratch_setup_mu;    // guards the set-up of g_scratch
std::mutex g_noalloc_mu;          // held for a whole call: g_stage, g_stage_device, has_done
alignas(kAlign) char g_stage[kNoAllocStageBytes];
int32_t g_stage_device = -1;      // GPU whose `staged` event guards g_stage

// Once per device, with that device current: the device address of its
// `scratch` and the device's two events.  *ptr is NULL for devices past
// kMaxScratchDevices (the entry point then reports SFM_EINVAL).
hipError_t scratch_setup(int32_t device, char** ptr) {
  *ptr = nullptr;
  if (device >= kMaxScratchDevices) return hipSuccess;
  std::lock_guard<std::mutex> lock(g_scratch_setup_mu);
  ScratchDevice& s = g_scratch[device];
  if (!s.ptr) {
    hipError_t e = hipSuccess;
    if (!s.staged && (e = hipEventCreateWithFlags(&s.staged, hipEventDisableTiming)) != hipSuccess)
      return e;
    if (!s.done && (e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess)
      return e;
    char* p = nullptr;
    if ((e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
    s.ptr = p;
  }
  *ptr = s.ptr;
  return hipSuccess;
}

// The caller holds ctx->mu.  Allocates nothing: no device, pinned or heap
// memory (error messages are cut to last_error's reserved capacity).
int noalloc_locked(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
                   const sfm_options* opt_in, const sfm_matches* out, void* stream) {
  if (!out) return fail(ctx, SFM_EINVAL, "out is NULL");
  sfm_options opt = default_options();
  if (opt_in) opt = *opt_in;
  int rc = check_options(ctx, opt);
  if (rc) return rc;
  if (!ctx->noalloc_scratch) return fail(ctx, SFM_EINVAL, "no scratch array on this device");
  if (n_pairs > SFM_NOALLOC_MAX_PAIRS) {
    char buf[128];
    snprintf(buf, sizeof buf, "%d pairs: sfm_guided_match_noalloc takes at most %d", n_pairs,
             SFM_NOALLOC_MAX_PAIRS);
    return fail(ctx, SFM_ECAPACITY, buf);
  }
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  // g_stage is free once the last staging copy out of it has run.
  if (g_stage_device >= 0) HIP_TRY(ctx, hipEventSynchronize(g_scratch[g_stage_device].staged));
  // plan() puts the pair table first, so it is described in place.
  PairDesc* pd = reinterpret_cast<PairDesc*>(g_stage);
  if ((rc = describe_pairs(ctx, registered(ctx), pairs, n_pairs, false, pd))) return rc;
  if ((rc = check_F(ctx, F, n_pairs))) return rc;
  const Layout L = plan(pd, size_t(n_pairs), ctx->device, ctx->group_tiles);
  if ((rc = check_outputs(ctx, out, L, opt))) return rc;
  if (L.pairs != 0 || L.staged > kNoAllocStageBytes)
    return fail(ctx, SFM_EINVAL, "staging layout does not fit the host buffer");
  if (L.total > SFM_NOALLOC_SCRATCH_BYTES) {
    char buf[160];
    snprintf(buf, sizeof buf,
             "the call needs %zu bytes of scratch; sfm_guided_match_noalloc has %zu", L.total,
             size_t(SFM_NOALLOC_SCRATCH_BYTES));
    return fail(ctx, SFM_ECAPACITY, buf);
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (n_pairs == 0) {
    hipLaunchKernelGGL(zero_offset_kernel, dim3(1), dim3(64), 0, st, out->offset);
    HIP_TRY(ctx, hipGetLastError());
    return SFM_OK;
  }
  ScratchDevice& sd = g_scratch[ctx->device];
  // Calls on one context, and all calls of this entry point on one GPU (they
  // share its scratch), run in the order they were made.
  if (ctx->has_work) HIP_TRY(ctx, hipStreamWaitEvent(st, ctx->work_done, 0));
  if (sd.has_done) HIP_TRY(ctx, hipStreamWaitEvent(st, sd.done, 0));

  char* ws = ctx->noalloc_scratch;
  memcpy(g_stage + L.F, F, size_t(n_pairs) * 9 * sizeof(double));
  binning_order(pd, n_pairs, reinterpret_cast<int32_t*>(g_stage + L.order));
  HIP_TRY(ctx, hipMemcpyAsync(ws, g_stage, L.staged, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipEventRecord(sd.staged, st));
  g_stage_device = ctx->device;

  // The geometry kernel zeroes the per-pair counters; every other section is
  // written before it is read, so nothing left by an earlier call is used.
  const BatchView v = batch_view(ctx, registered(ctx), ws, L, n_pairs, opt);
  int32_t max_na = 0;
  for (int32_t k = 0; k < n_pairs; ++k) max_na = std::max(max_na, pd[k].na);
  HIP_TRY(ctx, launch_prepare(v, 0, n_pairs, 0, int32_t(L.sum_groups), L.wgs,
                              reinterpret_cast<const int32_t*>(ws + L.order), max_na, st));
  HIP_TRY(ctx, launch_match(v, L.sum_groups > 0 ? L.wgs : 0, st));
  const bool ea = opt.emit_all != 0;
  HIP_TRY(ctx, launch_emit(v, 0, n_pairs, out->offset, out->query, out->match, out->d1, out->d2,
                           out->n_comparisons, out->n_borderline, ea ? out->all_match : nullptr,
                           ea ? out->all_d1 : nullptr, ea ? out->all_d2 : nullptr,
                           ea ? out->all_count : nullptr, st));
  HIP_TRY(ctx, hipEventRecord(sd.done, st));
  sd.has_done = true;
  HIP_TRY(ctx, hipEventRecord(ctx->work_done, st));
  ctx->has_work = true;
  ctx->last_pairs = 0;   // its counters sit in the shared scratch: no sfm_last_stats
  return SFM_OK;
}

}  // namespace

namespace sfm {
int32_t ctx_device(const sfm_ctx* ctx) { return ctx->device; }
int32_t ctx_n_images(const sfm_ctx* ctx) { return ctx->n_images; }
int32_t ctx_image_size(const sfm_ctx* ctx, int32_t image) {
  return image >= 0 && image < ctx->n_images ? ctx->n_host[size_t(image)] : 0;
}
// The per-pair terms of plan(), each section counted without its alignment
// (which ctx_call_bytes covers), so sums over pairs bound plan().total.
size_t ctx_request_bytes(const sfm_ctx* ctx, int32_t a, int32_t b) {
  const size_t na = size_t(ctx_image_size(ctx, a)), nb = size_t(ctx_image_size(ctx, b));
  const size_t nbins = size_t(bins_for(int32_t(nb), ctx->features_per_bin));
  const size_t nblocks = (na + kQueryTile - 1) / kQueryTile;
  const size_t ngroups = (nblocks + size_t(ctx->group_tiles) - 1) / size_t(ctx->group_tiles);
  return sizeof(PairDesc) + 9 * sizeof(double) + sizeof(int32_t) + sizeof(PairGeom) +
         sizeof(PairCounters) + sizeof(long long) +
         (nb + kCandPad) * (2 * sizeof(float) + sizeof(uint32_t) + sizeof(int32_t)) +
         (nbins + 1) * sizeof(int32_t) +
         na * (sizeof(QueryRec) + sizeof(QueryResult) + sizeof(int2)) +
         ngroups * (sizeof(TileGroup) + sizeof(int32_t));
}
// The alignment of plan()'s sections and the schedule table at its largest.
size_t ctx_call_bytes(const sfm_ctx* ctx) {
  const int32_t wgs = match_workgroups(ctx->device, ctx->group_tiles, int64_t(1) << 40);
  return 20 * kAlign + size_t(wgs + 1) * sizeof(int32_t);
}
size_t ctx_budget(const sfm_ctx* ctx) { return ctx->budget; }

struct ServeSpace {
  char* ws = nullptr;
  size_t ws_cap = 0;
  char* pinned = nullptr;
  size_t pinned_cap = 0;
  hipEvent_t staging_done = nullptr, work_done = nullptr;
  bool has_work = false;
  size_t budget = 0;
  int32_t device = 0;
};

void serve_space_destroy(ServeSpace* sp) {
  if (!sp) return;
  (void)hipSetDevice(sp->device);
  if (sp->has_work) (void)hipEventSynchronize(sp->work_done);
  if (sp->staging_done) (void)hipEventSynchronize(sp->staging_done);
  if (sp->ws) (void)hipFree(sp->ws);
  if (sp->pinned) (void)hipHostFree(sp->pinned);
  if (sp->staging_done) (void)hipEventDestroy(sp->staging_done);
  if (sp->work_done) (void)hipEventDestroy(sp->work_done);
  delete sp;
}

ServeSpace* serve_space_create(sfm_ctx* ctx, size_t budget) {
  if (hipSetDevice(ctx->device) != hipSuccess) return nullptr;
  ServeSpace* sp = new ServeSpace();
  sp->device = ctx->device;
  sp->budget = budget;
  if (hipEventCreateWithFlags(&sp->staging_done, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&sp->work_done, hipEventDisableTiming) != hipSuccess) {
    serve_space_destroy(sp);
    return nullptr;
  }
  return sp;
}

int serve_match(sfm_ctx* ctx, ServeSpace* sp, const sfm_pair* pairs, int32_t n_pairs,
                const double* F, const sfm_options* opt, const sfm_matches* out, hipStream_t st) {
  if (!ctx || !sp) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  const Space S{&sp->ws,          &sp->ws_cap,   &sp->pinned,   &sp->pinned_cap,
                sp->staging_done, sp->work_done, &sp->has_work, sp->budget};
  return match_locked(ctx, registered(ctx), pairs, n_pairs, F, opt, out, st, Form::kBatched,
                      nullptr, &S);
}
}  // namespace sfm

extern "C" {

const char* sfm_strerror(int status) {
  switch (status) {
    case SFM_OK: return "ok";
    case SFM_EINVAL: return "invalid argument";
    case SFM_ENOMEM: return "out of memory";
    case SFM_EHIP: return "HIP runtime error";
    case SFM_ECAPACITY: return "capacity exceeded";
    case SFM_EKERNEL: return "device error flag raised";
    case SFM_EBUSY: return "busy";
    case SFM_ETIMEOUT: return "timed out";
    case SFM_ENOTFOUND: return "not found";
    default: return "unknown status";
  }
}

int sfm_last_error(sfm_ctx* ctx, char* buf, size_t len) {
  if (!ctx || !buf || len == 0) return SFM_EINVAL;
  snprintf(buf, len, "%s", ctx->last_error.c_str());
  return SFM_OK;
}

int sfm_create(sfm_ctx** out, int32_t device, size_t budget) {
  if (!out) return SFM_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SFM_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return SFM_EHIP;
  sfm_ctx* ctx = new sfm_ctx();
  ctx->device = device;
  ctx->budget = budget ? budget : (size_t(8) << 30);
  ctx->last_error.reserve(255);
  if (hipEventCreateWithFlags(&ctx->staging_done, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->work_done, hipEventDisableTiming) != hipSuccess ||
      hipMalloc(&ctx->err_dev, sizeof(int32_t)) != hipSuccess ||
      hipMemset(ctx->err_dev, 0, sizeof(int32_t)) != hipSuccess ||
      scratch_setup(device, &ctx->noalloc_scratch) != hipSuccess) {
    sfm_destroy(ctx);
    return SFM_EHIP;
  }
  *out = ctx;
  return SFM_OK;
}

static void free_registration(sfm_ctx* ctx) {
  if (ctx->images_dev) (void)hipFree(ctx->images_dev);
  if (ctx->norm2_dev) (void)hipFree(ctx->norm2_dev);
  if (ctx->norm_off_dev) (void)hipFree(ctx->norm_off_dev);
  ctx->images_dev = nullptr;
  ctx->norm2_dev = nullptr;
  ctx->norm_off_dev = nullptr;
  ctx->n_images = 0;
  ctx->n_host.clear();
  ctx->bbox_host.clear();
}

int sfm_destroy(sfm_ctx* ctx) {
  if (!ctx) return SFM_EINVAL;
  server_release(ctx);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  free_registration(ctx);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->stage_buf) (void)hipFree(ctx->stage_buf);
  if (ctx->diag_dev) (void)hipFree(ctx->diag_dev);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->err_dev) (void)hipFree(ctx->err_dev);
  for (hipEvent_t e : ctx->prof_events) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
  if (ctx->staging_done) (void)hipEventDestroy(ctx->staging_done);
  if (ctx->work_done) (void)hipEventDestroy(ctx->work_done);
  if (ctx->graph) (void)hipGraphExecDestroy(ctx->graph);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
  return SFM_OK;
}

int sfm_register_images(sfm_ctx* ctx, const sfm_image* images, int32_t n_images) {
  if (!ctx) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (n_images < 0 || (n_images > 0 && !images)) return fail(ctx, SFM_EINVAL, "bad image list");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (ctx->has_work) HIP_TRY(ctx, hipEventSynchronize(ctx->work_done));
  free_registration(ctx);
  std::vector<ImageDev> host(static_cast<size_t>(n_images));
  std::vector<int64_t> off(size_t(n_images) + 1, 0);
  for (int32_t k = 0; k < n_images; ++k) {
    const sfm_image& s = images[k];
    if (s.n < 0 || (s.n > 0 && (!s.xy || !s.desc))) {
      char buf[64];
      snprintf(buf, sizeof buf, "image %d: bad pointers or size", k);
      return fail(ctx, SFM_EINVAL, buf);
    }
    off[size_t(k) + 1] = off[size_t(k)] + s.n;
  }
  if (n_images == 0) return SFM_OK;
  HIP_TRY(ctx, hipMalloc(&ctx->norm2_dev, std::max<size_t>(4, size_t(off.back()) * 4)));
  HIP_TRY(ctx, hipMalloc(&ctx->norm_off_dev, off.size() * sizeof(int64_t)));
  HIP_TRY(ctx, hipMalloc(&ctx->images_dev, host.size() * sizeof(ImageDev)));
  for (int32_t k = 0; k < n_images; ++k) {
    ImageDev& d = host[size_t(k)];
    memset(&d, 0, sizeof d);
    d.xy = images[k].xy;
    d.desc = images[k].desc;
    d.norm2 = ctx->norm2_dev + off[size_t(k)];
    d.n = images[k].n;
  }
  HIP_TRY(ctx, hipMemcpy(ctx->norm_off_dev, off.data(), off.size() * sizeof(int64_t),
                         hipMemcpyHostToDevice));
  HIP_TRY(ctx, hipMemcpy(ctx->images_dev, host.data(), host.size() * sizeof(ImageDev),
                         hipMemcpyHostToDevice));
  int32_t* bad = nullptr;
  HIP_TRY(ctx, hipMalloc(&bad, sizeof(int32_t)));
  hipError_t e = hipMemset(bad, 0, sizeof(int32_t));
  if (e == hipSuccess)
    e = launch_register(host.data(), ctx->images_dev, n_images, ctx->norm2_dev,
                        ctx->norm_off_dev, nullptr, bad, nullptr);
  int32_t bad_h = 0;
  if (e == hipSuccess) e = hipMemcpy(&bad_h, bad, sizeof(int32_t), hipMemcpyDeviceToHost);
  (void)hipFree(bad);
  if (e != hipSuccess) {
    free_registration(ctx);
    return hip_fail(ctx, e, "image registration");
  }
  if (bad_h) {
    free_registration(ctx);
    return fail(ctx, SFM_EINVAL, "a descriptor byte exceeds 127 or a keypoint is not finite");
  }
  e = hipMemcpy(host.data(), ctx->images_dev, host.size() * sizeof(ImageDev),
                hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    free_registration(ctx);
    return hip_fail(ctx, e, "image registration");
  }
  ctx->n_images = n_images;
  ctx->n_host.resize(size_t(n_images));
  ctx->bbox_host.resize(4 * size_t(n_images));
  for (int32_t k = 0; k < n_images; ++k) {
    ctx->n_host[size_t(k)] = images[k].n;
    for (int c = 0; c < 4; ++c) ctx->bbox_host[4 * size_t(k) + size_t(c)] = host[size_t(k)].bbox[c];
  }
  return SFM_OK;
}

int sfm_workspace_size(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, size_t* bytes) {
  if (!ctx || !bytes) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  std::vector<PairDesc> pd;
  const int rc = describe_pairs(ctx, registered(ctx), pairs, n_pairs, false, pd);
  if (rc) return rc;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  *bytes = plan(pd, ctx->device, ctx->group_tiles).total;
  return SFM_OK;
}

int sfm_guided_match(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
                     const sfm_options* opt, const sfm_matches* out, void* stream) {
  return run_match(ctx, pairs, n_pairs, F, opt, out, stream, Form::kBatched);
}

int sfm_guided_match_noalloc(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs,
                             const double* F, const sfm_options* opt, const sfm_matches* out,
                             void* stream) {
  if (!ctx) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  return noalloc_locked(ctx, pairs, n_pairs, F, opt, out, stream);
}

int sfm_guided_match_plain(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs,
                           const double* F, const sfm_options* opt, const sfm_matches* out,
                           void* stream) {
  return run_match(ctx, pairs, n_pairs, F, opt, out, stream, Form::kPlain);
}

int sfm_bruteforce_match(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
                         const sfm_options* opt, const sfm_matches* out, void* stream) {
  return run_match(ctx, pairs, n_pairs, F, opt, out, stream, Form::kExhaustive);
}

int sfm_band_error(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
                   double* max_err_px, int64_t* n_slots, void* stream) {
  if (!ctx) return SFM_EINVAL;
  if (!max_err_px || !n_slots) return fail(ctx, SFM_EINVAL, "output pointer is NULL");
  std::lock_guard<std::mutex> lock(ctx->mu);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (!ctx->diag_dev) HIP_TRY(ctx, hipMalloc(&ctx->diag_dev, 2 * sizeof(unsigned long long)));
  *max_err_px = 0.0;
  *n_slots = 0;
  const int rc = match_locked(ctx, registered(ctx), pairs, n_pairs, F, nullptr, nullptr, stream,
                              Form::kBandError, ctx->diag_dev);
  if (rc || n_pairs == 0) return rc;
  unsigned long long h[2] = {0, 0};
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(ctx, hipMemcpyAsync(h, ctx->diag_dev, sizeof h, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  double e;
  memcpy(&e, &h[0], sizeof e);
  *max_err_px = e;
  *n_slots = int64_t(h[1]);
  return SFM_OK;
}

int sfm_grid_match(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
                   const sfm_options* opt_in, const sfm_matches* out, void* stream) {
  if (!ctx) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (!out || !out->offset) return fail(ctx, SFM_EINVAL, "out or out->offset is NULL");
  sfm_options opt = default_options();
  if (opt_in) opt = *opt_in;
  if (const int orc = check_options(ctx, opt)) return orc;
  std::vector<PairDesc> pd;
  int rc = describe_pairs(ctx, registered(ctx), pairs, n_pairs, false, pd);
  if (rc) return rc;
  if ((rc = check_F(ctx, F, n_pairs))) return rc;
  const size_t P = size_t(n_pairs);
  std::vector<GridPair> gp(P);
  int64_t sum_na = 0, cells = 0, items = 0, max_cells = 0;
  for (size_t k = 0; k < P; ++k) {
    const sfm_pair& s = pairs[k];
    if (!(s.band_px > 0.0) || !std::isfinite(s.band_px)) {
      char buf[96];
      snprintf(buf, sizeof buf, "pair %zu: the grid needs a finite d > 0 (got %g)", k, s.band_px);
      return fail(ctx, SFM_EINVAL, buf);
    }
    GridPair& g = gp[k];
    memset(&g, 0, sizeof g);
    g.a = s.a;
    g.b = s.b;
    g.na = pd[k].na;
    g.nb = pd[k].nb;
    if (g.nb > kGridMaxTargets) {
      char buf[96];
      snprintf(buf, sizeof buf, "pair %zu: %d target features exceed the grid limit %d", k, g.nb,
               kGridMaxTargets);
      return fail(ctx, SFM_ECAPACITY, buf);
    }
    g.d = s.band_px;
    for (int c = 0; c < 4; ++c) g.box[c] = double(ctx->bbox_host[4 * size_t(s.b) + size_t(c)]);
    g.q_off = sum_na;
    g.item_off = items;
    const double two_d = 2.0 * g.d;
    for (int t = 0; t < 4; ++t) {
      const double sx = (t & 1) ? g.d : 0.0, sy = (t & 2) ? g.d : 0.0;
      const double fx0 = std::floor((g.box[0] - sx) / two_d), fx1 = std::floor((g.box[2] - sx) / two_d);
      const double fy0 = std::floor((g.box[1] - sy) / two_d), fy1 = std::floor((g.box[3] - sy) / two_d);
      const double ncx = fx1 - fx0 + 1.0, ncy = fy1 - fy0 + 1.0;
      if (!(ncx * ncy <= double(kGridMaxCells)) || std::fabs(fx0) > 1e9 || std::fabs(fy0) > 1e9) {
        char buf[128];
        snprintf(buf, sizeof buf, "pair %zu: d = %g makes more than %lld cells per grid", k, g.d,
                 (long long)kGridMaxCells);
        return fail(ctx, SFM_ECAPACITY, buf);
      }
      g.cx0[t] = int32_t(fx0);
      g.cy0[t] = int32_t(fy0);
      g.ncx[t] = int32_t(ncx);
      g.ncy[t] = int32_t(ncy);
      g.cell_off[t] = cells;
      cells += int64_t(ncx) * int64_t(ncy) + 1;
      max_cells = std::max(max_cells, int64_t(ncx) * int64_t(ncy));
    }
    sum_na += g.na;
    items += 4 * int64_t(g.nb);
  }
  if (out->capacity < sum_na) {
    char buf[128];
    snprintf(buf, sizeof buf, "output capacity %lld < %lld queries", (long long)out->capacity,
             (long long)sum_na);
    return fail(ctx, SFM_ECAPACITY, buf);
  }
  if (sum_na > 0 && (!out->query || !out->match || !out->d1 || !out->d2))
    return fail(ctx, SFM_EINVAL, "output arrays are NULL");
  if (opt.emit_all && sum_na > 0 &&
      (!out->all_match || !out->all_d1 || !out->all_d2 || !out->all_count))
    return fail(ctx, SFM_EINVAL, "emit_all needs all_match, all_d1, all_d2 and all_count");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (n_pairs == 0) {
    HIP_TRY(ctx, hipMemsetAsync(out->offset, 0, sizeof(int64_t), st));
    return SFM_OK;
  }
  // Workspace: staged part (grid pairs, pair descriptors, F), then tables.
  size_t o = 0;
  const size_t o_gp = o; o = align_up(o + P * sizeof(GridPair));
  const size_t o_pd = o; o = align_up(o + P * sizeof(PairDesc));
  const size_t o_F = o; o = align_up(o + P * 9 * sizeof(double));
  std::vector<int2> blocks;
  int32_t max_nb = 0, max_na = 0;
  for (size_t k = 0; k < P; ++k) {
    for (int32_t q0 = 0; q0 < gp[k].na; q0 += kGridQueriesPerBlock)
      blocks.push_back(make_int2(int32_t(k), q0));
    max_nb = std::max(max_nb, gp[k].nb);
    max_na = std::max(max_na, gp[k].na);
  }
  if (blocks.size() > size_t(INT32_MAX)) return fail(ctx, SFM_ECAPACITY, "too many queries");
  const size_t o_blk = o; o = align_up(o + std::max<size_t>(blocks.size(), 1) * sizeof(int2));
  const bool grouped = ctx->grid_group_px > 0.0 && sum_na > 0;
  if (grouped && sum_na > INT32_MAX / 4) return fail(ctx, SFM_ECAPACITY, "too many queries");
  const size_t N = size_t(sum_na);
  const size_t o_seg = o; o = align_up(o + 2 * P * sizeof(int32_t));
  const size_t staged = o;
  size_t temp_bytes = 0;
  if (grouped) HIP_TRY(ctx, grid_group_temp_bytes(int32_t(N), n_pairs, &temp_bytes));
  const size_t o_cross = o; o = align_up(o + (grouped ? N * 4 * sizeof(double) : 0));
  const size_t o_hit = o; o = align_up(o + (grouped ? N * sizeof(int32_t) : 0));
  const size_t o_val = o; o = align_up(o + (grouped ? 2 * N * sizeof(int32_t) : 0));
  const size_t o_sten = o; o = align_up(o + (grouped ? 3 * N * sizeof(int32_t) : 0));
  const size_t o_temp = o; o = align_up(o + temp_bytes);
  const size_t o_start = o; o = align_up(o + size_t(cells) * sizeof(int32_t));
  const size_t o_cur = o; o = align_up(o + size_t(cells) * sizeof(int32_t));
  const size_t o_items = o; o = align_up(o + size_t(std::max<int64_t>(items, 1)) * sizeof(int32_t));
  const size_t o_res = o; o = align_up(o + size_t(std::max<int64_t>(sum_na, 1)) * sizeof(QueryResult));
  const size_t o_cnt = o; o = align_up(o + P * sizeof(PairCounters));
  if ((rc = ensure_workspace(ctx, o))) return rc;
  if ((rc = ensure_pinned(ctx, staged))) return rc;
  if (ctx->has_work) HIP_TRY(ctx, hipStreamWaitEvent(st, ctx->work_done, 0));
  HIP_TRY(ctx, hipEventSynchronize(ctx->staging_done));
  memcpy(ctx->pinned + o_gp, gp.data(), P * sizeof(GridPair));
  memcpy(ctx->pinned + o_pd, pd.data(), P * sizeof(PairDesc));
  memcpy(ctx->pinned + o_F, F, P * 9 * sizeof(double));
  memcpy(ctx->pinned + o_blk, blocks.data(), blocks.size() * sizeof(int2));
  {
    int32_t* seg = reinterpret_cast<int32_t*>(ctx->pinned + o_seg);
    for (size_t k = 0; k < P; ++k) {
      seg[k] = int32_t(gp[k].q_off);
      seg[P + k] = int32_t(gp[k].q_off + gp[k].na);
    }
  }
  HIP_TRY(ctx, hipMemcpyAsync(ctx->ws, ctx->pinned, staged, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipEventRecord(ctx->staging_done, st));
  HIP_TRY(ctx, hipMemsetAsync(ctx->ws + o_cnt, 0, P * sizeof(PairCounters), st));

  GridView gv;
  memset(&gv, 0, sizeof gv);
  gv.images = ctx->images_dev;
  gv.pairs = reinterpret_cast<const GridPair*>(ctx->ws + o_gp);
  gv.F = reinterpret_cast<const double*>(ctx->ws + o_F);
  gv.cell_start = reinterpret_cast<int32_t*>(ctx->ws + o_start);
  gv.cursor = reinterpret_cast<int32_t*>(ctx->ws + o_cur);
  gv.items = reinterpret_cast<int32_t*>(ctx->ws + o_items);
  gv.blocks = reinterpret_cast<const int2*>(ctx->ws + o_blk);
  gv.bitmap_words = std::max(1, (max_nb + 31) / 32);
  gv.lds_cells = int32_t(std::min<int64_t>(max_cells, kGridLdsCells));
  gv.res = reinterpret_cast<QueryResult*>(ctx->ws + o_res);
  gv.counters = reinterpret_cast<PairCounters*>(ctx->ws + o_cnt);
  gv.err = ctx->err_dev;
  gv.n_pairs = n_pairs;
  gv.ratio_num = opt.ratio_num;
  gv.ratio_den = opt.ratio_den;
  gv.accept_single = opt.accept_single ? 1 : 0;
  gv.keep_counts = opt.emit_all ? 1 : 0;
  if (!grouped) {
    HIP_TRY(ctx, launch_grid(gv, int64_t(blocks.size()), st));
  } else {
    // Grouping (Section 6.2.2): sort, stencil and scan on the device; the
    // host reads the group count to size the last launch.
    HIP_TRY(ctx, launch_grid(gv, 0, st));
    GroupView g;
    memset(&g, 0, sizeof g);
    g.cross = reinterpret_cast<double*>(ctx->ws + o_cross);
    g.hit = reinterpret_cast<int32_t*>(ctx->ws + o_hit);
    g.val[0] = reinterpret_cast<int32_t*>(ctx->ws + o_val);
    g.val[1] = g.val[0] + N;
    g.seg_begin = reinterpret_cast<const int32_t*>(ctx->ws + o_seg);
    g.seg_end = g.seg_begin + P;
    g.stencil = reinterpret_cast<int32_t*>(ctx->ws + o_sten);
    g.gid = g.stencil + N;
    g.gstart = g.gid + N;
    g.temp = ctx->ws + o_temp;
    g.temp_bytes = temp_bytes;
    g.n = int32_t(N);
    g.tol2 = ctx->grid_group_px * ctx->grid_group_px;
    g.to_leader = ctx->grid_group_leader;
    HIP_TRY(ctx, launch_grid_group_prepare(gv, g, st));
    int32_t n_groups = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&n_groups, g.gid + (N - 1), sizeof(int32_t), hipMemcpyDeviceToHost,
                                st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    if (n_groups < 1 || size_t(n_groups) > N) return fail(ctx, SFM_EKERNEL, "bad group count");
    HIP_TRY(ctx, launch_grid_groups(gv, g, n_groups, st));
    ctx->last_groups = n_groups;
  }

  // Ordered emission reads only the pair descriptors, results and counters.
  BatchView v;
  memset(&v, 0, sizeof v);
  v.pairs = reinterpret_cast<const PairDesc*>(ctx->ws + o_pd);
  v.res = gv.res;
  v.counters = gv.counters;
  v.n_pairs = n_pairs;
  v.max_na = max_na;
  int32_t* am = opt.emit_all ? out->all_match : nullptr;
  int32_t* ad1 = opt.emit_all ? out->all_d1 : nullptr;
  int32_t* ad2 = opt.emit_all ? out->all_d2 : nullptr;
  int32_t* ac = opt.emit_all ? out->all_count : nullptr;
  HIP_TRY(ctx, launch_emit(v, 0, n_pairs, out->offset, out->query, out->match, out->d1, out->d2,
                           out->n_comparisons, out->n_borderline, am, ad1, ad2, ac, st));
  HIP_TRY(ctx, hipEventRecord(ctx->work_done, st));
  ctx->has_work = true;
  ctx->last_pairs = n_pairs;
  ctx->last_counters = o_cnt;
  return SFM_OK;
}

int sfm_set_grid_grouping(sfm_ctx* ctx, double px, int32_t to_leader) {
  if (!ctx) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (!(px >= 0.0) || !std::isfinite(px)) return fail(ctx, SFM_EINVAL, "px must be finite and >= 0");
  ctx->grid_group_px = px;
  ctx->grid_group_leader = to_leader ? 1 : 0;
  return SFM_OK;
}

int sfm_grid_groups(sfm_ctx* ctx, int64_t* n_groups) {
  if (!ctx || !n_groups) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  *n_groups = ctx->last_groups;
  return SFM_OK;
}

int sfm_preemptive_match(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs,
                         const sfm_preemptive_cfg* cfg_in, const sfm_options* opt_in,
                         const sfm_matches* out, int32_t* stages, void* stream) {
  if (!ctx) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  sfm_preemptive_cfg cfg = {10, 20, 4, 0, 1000, 0};
  if (cfg_in) cfg = *cfg_in;
  if (cfg.query_pct < 1 || cfg.query_pct > 100 || cfg.target_pct < 1 || cfg.target_pct > 100 ||
      cfg.min_matches < 0 || cfg.enough < 0 || cfg.small_image < 0)
    return fail(ctx, SFM_EINVAL,
                "cfg: query_pct and target_pct must be in 1..100, the counts >= 0");
  sfm_options opt = default_options();
  if (opt_in) opt = *opt_in;
  if (opt.emit_all) return fail(ctx, SFM_EINVAL, "emit_all is not available for staged matching");
  if (!out || !out->offset) return fail(ctx, SFM_EINVAL, "out or out->offset is NULL");
  if (n_pairs < 0 || n_pairs > INT32_MAX / 3 || (n_pairs > 0 && !pairs))
    return fail(ctx, SFM_EINVAL, "bad pair list");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);

  // Views per pair k: 3k = stage-1 queries, 3k+1 = targets, 3k+2 = stage-2 queries.
  const size_t P = size_t(n_pairs);
  std::vector<int32_t> spec(9 * P), vn(3 * P);
  std::vector<uint8_t> whole(P);
  int64_t cap1 = 0, cap2 = 0;
  for (size_t k = 0; k < P; ++k) {
    const sfm_pair& s = pairs[k];
    if (s.a < 0 || s.a >= ctx->n_images || s.b < 0 || s.b >= ctx->n_images) {
      char buf[128];
      snprintf(buf, sizeof buf, "pair %zu: image index out of range (a=%d b=%d, %d registered)",
               k, s.a, s.b, ctx->n_images);
      return fail(ctx, SFM_EINVAL, buf);
    }
    const int64_t na = ctx->n_host[size_t(s.a)], nb = ctx->n_host[size_t(s.b)];
    whole[k] = na < cfg.small_image || nb < cfg.small_image;
    const int64_t q = whole[k] ? na : (na * cfg.query_pct + 99) / 100;
    const int64_t r = whole[k] ? nb : (nb * cfg.target_pct + 99) / 100;
    const int64_t q2 = whole[k] ? 0 : std::min(q, na - q);
    const int32_t v[9] = {s.a, 0, int32_t(q), s.b, 0, int32_t(r), s.a, int32_t(q), int32_t(q2)};
    std::copy(v, v + 9, spec.begin() + 9 * k);
    vn[3 * k] = int32_t(q);
    vn[3 * k + 1] = int32_t(r);
    vn[3 * k + 2] = int32_t(q2);
    cap1 += q;
    cap2 += q2;
  }
  if (out->capacity < cap1 + cap2) {
    char buf[128];
    snprintf(buf, sizeof buf, "output capacity %lld < %lld queries", (long long)out->capacity,
             (long long)(cap1 + cap2));
    return fail(ctx, SFM_ECAPACITY, buf);
  }
  if (cap1 + cap2 > 0 && (!out->query || !out->match || !out->d1 || !out->d2))
    return fail(ctx, SFM_EINVAL, "output arrays are NULL");
  if (n_pairs == 0) {
    HIP_TRY(ctx, hipMemsetAsync(out->offset, 0, sizeof(int64_t), st));
    return SFM_OK;
  }

  // Stage buffer: views, spec, both stages' rows and counts, merge plan.
  size_t o = 0;
  const size_t o_views = o; o = align_up(o + 3 * P * sizeof(ImageDev));
  const size_t o_spec = o; o = align_up(o + 9 * P * sizeof(int32_t));
  const size_t o_merge = o; o = align_up(o + P * sizeof(StageMerge));
  size_t o_off[2], o_cmp[2], o_rows[2];
  const int64_t caps[2] = {cap1, cap2};
  for (int t = 0; t < 2; ++t) {
    o_off[t] = o; o = align_up(o + (P + 1) * sizeof(int64_t));
    o_cmp[t] = o; o = align_up(o + P * sizeof(int64_t));
    o_rows[t] = o; o = align_up(o + 4 * size_t(std::max<int64_t>(caps[t], 1)) * sizeof(int32_t));
  }
  if (o > ctx->budget) return fail(ctx, SFM_ECAPACITY, "staged matching exceeds the budget");
  if (o > ctx->stage_cap) {
    if (ctx->has_work) HIP_TRY(ctx, hipEventSynchronize(ctx->work_done));
    if (ctx->stage_buf) HIP_TRY(ctx, hipFree(ctx->stage_buf));
    ctx->stage_buf = nullptr;
    ctx->stage_cap = 0;
    HIP_TRY(ctx, hipMalloc(&ctx->stage_buf, o + o / 4));
    ctx->stage_cap = o + o / 4;
  }
  char* B = ctx->stage_buf;
  if (ctx->has_work) HIP_TRY(ctx, hipStreamWaitEvent(st, ctx->work_done, 0));
  ImageDev* views = reinterpret_cast<ImageDev*>(B + o_views);
  HIP_TRY(ctx, hipMemcpyAsync(B + o_spec, spec.data(), spec.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, launch_make_views(ctx->images_dev, reinterpret_cast<const int32_t*>(B + o_spec),
                                 int32_t(3 * P), views, st));
  const ImageTable tab{views, vn.data(), int32_t(3 * P)};
  sfm_matches so[2];
  StageRows rows[2];
  for (int t = 0; t < 2; ++t) {
    int32_t* r = reinterpret_cast<int32_t*>(B + o_rows[t]);
    const size_t c = size_t(std::max<int64_t>(caps[t], 1));
    memset(&so[t], 0, sizeof so[t]);
    so[t].query = r;
    so[t].match = r + c;
    so[t].d1 = r + 2 * c;
    so[t].d2 = r + 3 * c;
    so[t].capacity = caps[t];
    so[t].offset = reinterpret_cast<int64_t*>(B + o_off[t]);
    so[t].n_comparisons = reinterpret_cast<int64_t*>(B + o_cmp[t]);
    rows[t] = StageRows{so[t].query, so[t].match, so[t].d1, so[t].d2, so[t].n_comparisons};
  }

  // Stage 1 (or the whole pair), then the counts back on the host.
  std::vector<sfm_pair> sp(P);
  for (size_t k = 0; k < P; ++k) sp[k] = sfm_pair{int32_t(3 * k), int32_t(3 * k + 1), 0.0};
  int rc = match_locked(ctx, tab, sp.data(), n_pairs, nullptr, &opt, &so[0], stream,
                        Form::kExhaustive);
  if (rc) return rc;
  std::vector<int64_t> off1(P + 1), off2(P + 1, 0);
  HIP_TRY(ctx, hipMemcpyAsync(off1.data(), so[0].offset, (P + 1) * sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));

  // Stage 2 for the pairs whose first stage found more than min_matches.
  std::vector<int32_t> in2(P, -1);
  sp.clear();
  for (size_t k = 0; k < P; ++k) {
    const int64_t c = off1[k + 1] - off1[k];
    if (whole[k] || vn[3 * k + 2] == 0 || c <= cfg.min_matches || (cfg.enough > 0 && c >= cfg.enough))
      continue;
    in2[k] = int32_t(sp.size());
    sp.push_back(sfm_pair{int32_t(3 * k + 2), int32_t(3 * k + 1), 0.0});
  }
  if (!sp.empty()) {
    rc = match_locked(ctx, tab, sp.data(), int32_t(sp.size()), nullptr, &opt, &so[1], stream,
                      Form::kExhaustive);
    if (rc) return rc;
    HIP_TRY(ctx, hipMemcpyAsync(off2.data(), so[1].offset, (sp.size() + 1) * sizeof(int64_t),
                                hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
  }

  // Merge: each pair's stage-1 rows, then its stage-2 rows.
  std::vector<StageMerge> plan_h(P);
  std::vector<int64_t> final_off(P + 1, 0);
  for (size_t k = 0; k < P; ++k) {
    StageMerge& m = plan_h[k];
    m.src1 = off1[k];
    m.n1 = int32_t(off1[k + 1] - off1[k]);
    m.s2 = in2[k];
    m.src2 = m.s2 >= 0 ? off2[size_t(m.s2)] : 0;
    m.n2 = m.s2 >= 0 ? int32_t(off2[size_t(m.s2) + 1] - off2[size_t(m.s2)]) : 0;
    m.shift = vn[3 * k];
    m.dst = final_off[k];
    final_off[k + 1] = final_off[k] + m.n1 + m.n2;
    if (stages) stages[k] = whole[k] ? 0 : (m.s2 >= 0 ? 2 : 1);
  }
  HIP_TRY(ctx, hipMemcpyAsync(B + o_merge, plan_h.data(), P * sizeof(StageMerge),
                              hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(out->offset, final_off.data(), (P + 1) * sizeof(int64_t),
                              hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, launch_merge_stages(reinterpret_cast<const StageMerge*>(B + o_merge), n_pairs,
                                   rows[0], rows[1], out->query, out->match, out->d1, out->d2,
                                   out->n_comparisons, st));
  HIP_TRY(ctx, hipEventRecord(ctx->work_done, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  int32_t flag = 0;
  HIP_TRY(ctx, hipMemcpy(&flag, ctx->err_dev, sizeof flag, hipMemcpyDeviceToHost));
  if (flag) {
    HIP_TRY(ctx, hipMemset(ctx->err_dev, 0, sizeof(int32_t)));
    return fail(ctx, SFM_EKERNEL, "a kernel raised the device error flag");
  }
  return SFM_OK;
}

int sfm_set_profiling(sfm_ctx* ctx, int32_t enable) {
  if (!ctx) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  ctx->profiling = enable != 0;
  return SFM_OK;
}

int sfm_phase_times(sfm_ctx* ctx, double ms[3], int64_t* n_records) {
  if (!ctx || !ms) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  ms[0] = ms[1] = ms[2] = 0.0;
  const size_t n = ctx->prof_events.size() / 4;
  if (!ctx->prof_events.empty()) HIP_TRY(ctx, hipEventSynchronize(ctx->prof_events.back()));
  for (size_t r = 0; r < n; ++r) {
    for (int k = 0; k < 3; ++k) {
      float t = 0.0f;
      HIP_TRY(ctx, hipEventElapsedTime(&t, ctx->prof_events[4 * r + k],
                                       ctx->prof_events[4 * r + k + 1]));
      ms[k] += t;
    }
  }
  for (hipEvent_t e : ctx->prof_events) ctx->prof_pool.push_back(e);
  ctx->prof_events.clear();
  if (n_records) *n_records = int64_t(n);
  return SFM_OK;
}

int sfm_last_stats(sfm_ctx* ctx, int64_t out[5]) {
  if (!ctx || !out) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  out[0] = out[1] = out[2] = out[3] = out[4] = 0;
  if (!ctx->has_work || ctx->last_pairs == 0) return SFM_OK;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipEventSynchronize(ctx->work_done));
  std::vector<PairCounters> c(size_t(ctx->last_pairs));
  HIP_TRY(ctx, hipMemcpy(c.data(), ctx->ws + ctx->last_counters, c.size() * sizeof(PairCounters),
                         hipMemcpyDeviceToHost));
  for (const PairCounters& k : c) {
    out[0] += int64_t(k.comparisons);
    out[1] += int64_t(k.elements);
    out[2] += k.ties;
    out[3] += k.accepted;
    out[4] += int64_t(k.borderline);
  }
  return SFM_OK;
}

int sfm_sync(sfm_ctx* ctx, void* stream) {
  if (!ctx) return SFM_EINVAL;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  int32_t flag = 0;
  HIP_TRY(ctx, hipMemcpy(&flag, ctx->err_dev, sizeof flag, hipMemcpyDeviceToHost));
  if (flag) {
    HIP_TRY(ctx, hipMemset(ctx->err_dev, 0, sizeof(int32_t)));
    return fail(ctx, SFM_EKERNEL, "a kernel raised the device error flag");
  }
  return SFM_OK;
}

int sfm_set_tuning(sfm_ctx* ctx, int32_t group_tiles, int32_t features_per_bin) {
  if (!ctx) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (group_tiles != 4 && group_tiles != 8)
    return fail(ctx, SFM_EINVAL, "group_tiles must be 4 or 8");
  if (features_per_bin < 1 || features_per_bin > 1024)
    return fail(ctx, SFM_EINVAL, "features_per_bin must be in 1..1024");
  ctx->group_tiles = group_tiles;
  ctx->features_per_bin = features_per_bin;
  return SFM_OK;
}

int sfm_candidate_images(sfm_ctx* ctx, const int32_t* vis_off, const int32_t* vis_pts,
                         int64_t nnz, int32_t n_images, int32_t n_points, int32_t threshold,
                         int32_t top_k, const sfm_candidates* out, void* stream) {
  if (!ctx) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (!out) return fail(ctx, SFM_EINVAL, "out is NULL");
  if (n_images < 0 || n_images > kMaxCovisImages)
    return fail(ctx, SFM_EINVAL, "n_images must be in 0..4096");
  if (n_points < 0 || int64_t(n_points) + 1 > scan_limit())
    return fail(ctx, SFM_EINVAL, "n_points out of range");
  if (nnz < 0 || nnz > INT32_MAX) return fail(ctx, SFM_EINVAL, "nnz must be in 0..2^31-1");
  if (threshold < 0 || top_k < 0) return fail(ctx, SFM_EINVAL, "threshold and top_k must be >= 0");
  if (n_images > 0 && (!vis_off || !out->n_cand))
    return fail(ctx, SFM_EINVAL, "vis_off and n_cand are required");
  if (nnz > 0 && !vis_pts) return fail(ctx, SFM_EINVAL, "vis_pts is NULL");
  if (n_images > 0 && top_k > 0 && (!out->cand || !out->n_shared))
    return fail(ctx, SFM_EINVAL, "cand and n_shared are required");
  if (out->pairs && !out->n_pairs) return fail(ctx, SFM_EINVAL, "pairs needs n_pairs");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const size_t np1 = size_t(n_points) + 1, ni1 = size_t(n_images) + 1;
  const size_t words = (size_t(n_images) + 31) / 32;
  const size_t pwords = (size_t(n_points) + 31) / 32;
  const size_t nsums = (std::max(np1, ni1) + 8191) / 8192 + 1;
  // The two exact methods: observers per point and an LDS histogram per image
  // (work ~ sum over points of observers^2, at least nnz^2 / n_points), or
  // the bit-matrix product (n^2 / 2 pairs of pwords words, ~20x cheaper per
  // unit).  Dense visibility favours the product, short tracks the histogram.
  bool use_gram = ctx->covis_method == 2;
  if (ctx->covis_method == 0 && n_images > 0 && n_points > 0) {
    const double hist = double(nnz) * double(nnz) / double(n_points);
    const double prod = double(n_images) * double(n_images) * double(pwords) / 2.0 / 20.0;
    use_gram = prod < hist;
  }
  size_t o = 0;
  const size_t o_count = o; o = align_up(o + np1 * 4);
  const size_t o_off = o; o = align_up(o + np1 * 4);
  const size_t o_cursor = o; o = align_up(o + np1 * 4);
  const size_t o_imgs = o; o = align_up(o + (use_gram ? 1 : std::max<size_t>(size_t(nnz), 1)) * 4);
  const size_t o_sums = o; o = align_up(o + nsums * 4);
  const size_t o_rc = o; o = align_up(o + ni1 * 4);
  const size_t o_ro = o; o = align_up(o + ni1 * 4);
  const size_t o_bits = o; o = align_up(o + std::max<size_t>(size_t(n_images) * words, 1) * 4);
  const size_t o_bitset = o;
  o = align_up(o + (use_gram ? std::max<size_t>(size_t(n_images) * pwords, 1) : 1) * 4);
  const size_t o_gram = o;
  o = align_up(o + (use_gram ? std::max<size_t>(size_t(n_images) * size_t(n_images), 1) : 1) * 4);
  int rc = ensure_workspace(ctx, o);
  if (rc) return rc;
  if (ctx->has_work) HIP_TRY(ctx, hipStreamWaitEvent(st, ctx->work_done, 0));
  CovisArgs a;
  a.vis_off = vis_off;
  a.vis_pts = vis_pts;
  a.nnz = nnz;
  a.n_images = n_images;
  a.n_points = n_points;
  a.threshold = threshold;
  a.top_k = top_k;
  a.pt_count = reinterpret_cast<int32_t*>(ctx->ws + o_count);
  a.pt_off = reinterpret_cast<int32_t*>(ctx->ws + o_off);
  a.cursor = reinterpret_cast<int32_t*>(ctx->ws + o_cursor);
  a.pt_imgs = reinterpret_cast<int32_t*>(ctx->ws + o_imgs);
  a.sums = reinterpret_cast<int32_t*>(ctx->ws + o_sums);
  a.row_count = reinterpret_cast<int32_t*>(ctx->ws + o_rc);
  a.row_off = reinterpret_cast<int32_t*>(ctx->ws + o_ro);
  a.bits = reinterpret_cast<uint32_t*>(ctx->ws + o_bits);
  a.bitset = reinterpret_cast<uint32_t*>(ctx->ws + o_bitset);
  a.gram = use_gram ? reinterpret_cast<int32_t*>(ctx->ws + o_gram) : nullptr;
  a.cand = out->cand;
  a.n_shared = out->n_shared;
  a.n_cand = out->n_cand;
  a.pairs = out->pairs;
  a.n_pairs = out->n_pairs;
  a.err = ctx->err_dev;
  HIP_TRY(ctx, launch_candidates(a, st));
  HIP_TRY(ctx, hipEventRecord(ctx->work_done, st));
  ctx->has_work = true;
  ctx->last_pairs = 0;
  return SFM_OK;
}

int sfm_tracks(sfm_ctx* ctx, int64_t n_nodes, const int32_t* edges, int64_t n_edges,
               int32_t* label, void* stream) {
  if (!ctx) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (n_nodes < 0 || n_nodes > INT32_MAX) return fail(ctx, SFM_EINVAL, "n_nodes out of range");
  if (n_edges < 0) return fail(ctx, SFM_EINVAL, "n_edges < 0");
  if (n_nodes > 0 && !label) return fail(ctx, SFM_EINVAL, "label is NULL");
  if (n_edges > 0 && !edges) return fail(ctx, SFM_EINVAL, "edges is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (ctx->has_work) HIP_TRY(ctx, hipStreamWaitEvent(st, ctx->work_done, 0));
  HIP_TRY(ctx, launch_tracks(n_nodes, edges, n_edges, label, ctx->err_dev, st));
  HIP_TRY(ctx, hipEventRecord(ctx->work_done, st));
  ctx->has_work = true;
  ctx->last_pairs = 0;
  return SFM_OK;
}

int sfm_triangulate(sfm_ctx* ctx, int64_t n_nodes, const int32_t* label, const int32_t* node_image,
                    const float* node_xy, const double* P, int32_t n_images, double* X,
                    int32_t* n_obs, void* stream) {
  if (!ctx) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (n_nodes < 0 || n_nodes > INT32_MAX) return fail(ctx, SFM_EINVAL, "n_nodes out of range");
  if (n_images < 0) return fail(ctx, SFM_EINVAL, "n_images < 0");
  if (n_nodes > 0 && (!label || !node_image || !node_xy || !X || !n_obs || (n_images > 0 && !P)))
    return fail(ctx, SFM_EINVAL, "a pointer is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  size_t temp_bytes = 0;
  HIP_TRY(ctx, triangulate_temp_bytes(n_nodes, &temp_bytes));
  const size_t lists = align_up(size_t(std::max<int64_t>(n_nodes, 1)) * 4 * sizeof(int32_t));
  int rc = ensure_workspace(ctx, lists + align_up(temp_bytes));
  if (rc) return rc;
  if (ctx->has_work) HIP_TRY(ctx, hipStreamWaitEvent(st, ctx->work_done, 0));
  HIP_TRY(ctx, launch_triangulate(n_nodes, label, node_image, node_xy, P, n_images,
                                  reinterpret_cast<int32_t*>(ctx->ws), ctx->ws + lists, temp_bytes,
                                  X, n_obs, ctx->err_dev, st));
  HIP_TRY(ctx, hipEventRecord(ctx->work_done, st));
  ctx->has_work = true;
  ctx->last_pairs = 0;
  return SFM_OK;
}

int sfm_set_covis_method(sfm_ctx* ctx, int32_t method) {
  if (!ctx) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (method < 0 || method > 2) return fail(ctx, SFM_EINVAL, "method must be 0, 1 or 2");
  ctx->covis_method = method;
  return SFM_OK;
}

int sfm_set_graph_replay(sfm_ctx* ctx, int32_t enable) {
  if (!ctx) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  ctx->graph_replay = enable != 0;
  ctx->last_key.clear();
  if (!ctx->graph_replay && ctx->graph) {
    if (ctx->has_work) HIP_TRY(ctx, hipEventSynchronize(ctx->work_done));
    HIP_TRY(ctx, hipGraphExecDestroy(ctx->graph));
    ctx->graph = nullptr;
    ctx->graph_key.clear();
  }
  return SFM_OK;
}

int sfm_get_tuning(sfm_ctx* ctx, int32_t* group_tiles, int32_t* features_per_bin) {
  if (!ctx || !group_tiles || !features_per_bin) return SFM_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  *group_tiles = ctx->group_tiles;
  *features_per_bin = ctx->features_per_bin;
  return SFM_OK;
}

int sfm_autotune(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
                 const sfm_options* opt, void* stream, int32_t repeats, double* ms_out) {
  if (!ctx) return SFM_EINVAL;
  if (repeats < 1) return fail(ctx, SFM_EINVAL, "repeats must be >= 1");
  static const int32_t kTiles[2] = {4, 8};
  static const int32_t kFpb[3] = {4, 8, 16};
  int64_t rows = 0;
  for (int32_t k = 0; k < n_pairs && pairs; ++k) {
    if (pairs[k].a < 0 || pairs[k].a >= ctx->n_images) return fail(ctx, SFM_EINVAL, "bad pair");
    rows += ctx->n_host[size_t(pairs[k].a)];
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // Scratch outputs for the trial runs.
  const size_t r4 = size_t(std::max<int64_t>(rows, 1)) * sizeof(int32_t);
  int32_t *q = nullptr, *m = nullptr, *d1 = nullptr, *d2 = nullptr;
  int64_t* off = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = SFM_OK;
  if (hipMalloc(&q, r4) != hipSuccess || hipMalloc(&m, r4) != hipSuccess ||
      hipMalloc(&d1, r4) != hipSuccess || hipMalloc(&d2, r4) != hipSuccess ||
      hipMalloc(&off, size_t(n_pairs + 1) * sizeof(int64_t)) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = fail(ctx, SFM_ENOMEM, "autotune scratch allocation failed");
  sfm_matches out;
  memset(&out, 0, sizeof out);
  out.query = q; out.match = m; out.d1 = d1; out.d2 = d2;
  out.offset = off; out.capacity = rows;
  int32_t keep_t, keep_f;
  {
    std::lock_guard<std::mutex> lock(ctx->mu);
    keep_t = ctx->group_tiles;
    keep_f = ctx->features_per_bin;
  }
  auto set = [&](int32_t t, int32_t f) {
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->group_tiles = t;
    ctx->features_per_bin = f;
  };
  double best = INFINITY;
  int32_t best_t = keep_t, best_f = keep_f;
  for (int ti = 0; ti < 2 && rc == SFM_OK; ++ti) {
    for (int fi = 0; fi < 3 && rc == SFM_OK; ++fi) {
      set(kTiles[ti], kFpb[fi]);
      // One untimed run sizes the workspace for this configuration.
      rc = run_match(ctx, pairs, n_pairs, F, opt, &out, stream, Form::kBatched);
      if (rc) break;
      if (hipEventRecord(e0, st) != hipSuccess) { rc = SFM_EHIP; break; }
      for (int32_t r = 0; r < repeats && rc == SFM_OK; ++r)
        rc = run_match(ctx, pairs, n_pairs, F, opt, &out, stream, Form::kBatched);
      if (rc) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = SFM_EHIP;
        break;
      }
      const double per = double(ms) / repeats;
      if (ms_out) ms_out[3 * ti + fi] = per;
      if (per < best) { best = per; best_t = kTiles[ti]; best_f = kFpb[fi]; }
    }
  }
  if (st) (void)hipStreamSynchronize(st); else (void)hipDeviceSynchronize();
  if (rc == SFM_OK)
    set(best_t, best_f);
  else
    set(keep_t, keep_f);
  if (q) (void)hipFree(q);
  if (m) (void)hipFree(m);
  if (d1) (void)hipFree(d1);
  if (d2) (void)hipFree(d2);
  if (off) (void)hipFree(off);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}

// Tuning cache: a JSON object, one entry per line,
//   "KEY": {"group_tiles": T, "features_per_bin": F, "ms": X},
// written by sfm_autotune_cached and read back by later calls.
static std::string tune_key(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  int64_t q = 0, c = 0;
  double band = 0.0;
  for (int32_t k = 0; k < n_pairs; ++k) {
    q += ctx->n_host[size_t(pairs[k].a)];
    c += ctx->n_host[size_t(pairs[k].b)];
    band += std::isfinite(pairs[k].band_px) ? pairs[k].band_px : 0.0;
  }
  const int qb = int(std::floor(std::log2(double(q) + 1.0)));
  const int fb = int(std::floor(std::log2(double(c) / std::max(1, n_pairs) + 1.0)));
  const int bb = int(std::lround(2.0 * std::log2(band / std::max(1, n_pairs) + 1e-9)));
  char buf[256];
  snprintf(buf, sizeof buf, "%s|cu%d|q%d|f%d|b%d", arch.c_str(), cus, qb, fb, bb);
  return buf;
}

static std::vector<std::string> tune_cache_lines(const char* path) {
  std::vector<std::string> lines;
  FILE* f = fopen(path, "r");
  if (!f) return lines;
  char buf[1024];
  while (fgets(buf, sizeof buf, f)) {
    std::string l(buf);
    while (!l.empty() && (l.back() == '\n' || l.back() == '\r' || l.back() == ',')) l.pop_back();
    if (l.find("\"group_tiles\"") != std::string::npos) lines.push_back(l);
  }
  fclose(f);
  return lines;
}

static bool tune_entry(const std::string& line, std::string* key, int32_t* t, int32_t* fpb) {
  const size_t k0 = line.find('"'), k1 = line.find('"', k0 + 1);
  const size_t pt = line.find("\"group_tiles\":"), pf = line.find("\"features_per_bin\":");
  if (k0 == std::string::npos || k1 == std::string::npos || pt == std::string::npos ||
      pf == std::string::npos)
    return false;
  *key = line.substr(k0 + 1, k1 - k0 - 1);
  *t = int32_t(strtol(line.c_str() + pt + 14, nullptr, 10));
  *fpb = int32_t(strtol(line.c_str() + pf + 19, nullptr, 10));
  return true;
}

int sfm_autotune_cached(sfm_ctx* ctx, const sfm_pair* pairs, int32_t n_pairs, const double* F,
                        const sfm_options* opt, void* stream, int32_t repeats,
                        const char* cache_path, double* ms_out, int32_t* from_cache) {
  if (!ctx || !cache_path || !from_cache) return SFM_EINVAL;
  if (n_pairs < 1 || !pairs) return fail(ctx, SFM_EINVAL, "autotuning needs at least one pair");
  for (int32_t k = 0; k < n_pairs; ++k)
    if (pairs[k].a < 0 || pairs[k].a >= ctx->n_images || pairs[k].b < 0 ||
        pairs[k].b >= ctx->n_images)
      return fail(ctx, SFM_EINVAL, "bad pair");
  *from_cache = 0;
  const std::string key = tune_key(ctx, pairs, n_pairs);
  std::vector<std::string> lines = tune_cache_lines(cache_path);
  for (const std::string& l : lines) {
    std::string k;
    int32_t t = 0, fpb = 0;
    if (tune_entry(l, &k, &t, &fpb) && k == key) {
      const int rc = sfm_set_tuning(ctx, t, fpb);
      if (rc == SFM_OK) *from_cache = 1;
      return rc;
    }
  }
  double ms[6];
  int rc = sfm_autotune(ctx, pairs, n_pairs, F, opt, stream, repeats, ms);
  if (rc) return rc;
  if (ms_out) memcpy(ms_out, ms, sizeof ms);
  int32_t t = 0, fpb = 0;
  sfm_get_tuning(ctx, &t, &fpb);
  const double best = ms[3 * (t == 8 ? 1 : 0) + (fpb == 4 ? 0 : fpb == 8 ? 1 : 2)];
  char entry[512];
  snprintf(entry, sizeof entry,
           "  \"%s\": {\"group_tiles\": %d, \"features_per_bin\": %d, \"ms\": %.4f}", key.c_str(), t,
           fpb, best);
  lines.push_back(entry);
  const std::string tmp = std::string(cache_path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return fail(ctx, SFM_EINVAL, std::string("cannot write the tuning cache ") + tmp);
  fputs("{\n", f);
  for (size_t k = 0; k < lines.size(); ++k) {
    std::string l = lines[k];
    if (l.compare(0, 2, "  ") != 0) l = "  " + l.substr(l.find('"'));
    fputs(l.c_str(), f);
    fputs(k + 1 < lines.size() ? ",\n" : "\n", f);
  }
  fputs("}\n", f);
  fclose(f);
  if (rename(tmp.c_str(), cache_path) != 0)
    return fail(ctx, SFM_EINVAL, std::string("cannot replace the tuning cache ") + cache_path);
  return SFM_OK;
}

}  // extern "C"
