// C ABI of the OFV estimator: argument validation, workspace management and
// the coarse-to-fine schedule of the pipeline (section "Live-Optical Flow
// Velocimetry", arXiv 2509.25924, six-step list).  Every compute entry point
// validates all arguments on the host first, then only enqueues kernels on
// the handle's stream: no allocation, no synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "ofv.h"
#include "ofv_stages.h"
#include "ofv_internal.h"
#include "ofv_adj.h"

using namespace ofv;

namespace {

constexpr int64_t kPitchAlign = 64;      // elements; 256 B rows for float32 planes
// Kernels address a plane with 32-bit byte offsets and 24-bit row products:
// every plane stays below 2 GiB and every pitch below 2^24 elements.
constexpr int64_t kMaxPlaneBytes = int64_t{1} << 31;
constexpr int64_t kMaxPitch = int64_t{1} << 24;
constexpr size_t kSlabAlign = 256;        // bytes

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

thread_local std::string g_create_error;

}  // namespace

struct ofv_ctx {
  int device = -1;  // -1: validation-only handle (no device resources)
  int num_cus = 256;  // compute units of the device (sizes band launches)
  hipStream_t stream = nullptr;
  int max_w = 0, max_h = 0, max_batch = 0;
  // level geometry of the largest frame; planes of smaller frames reuse it
  int lw[OFV_MAX_LEVELS] = {}, lh[OFV_MAX_LEVELS] = {};
  int64_t lpitch[OFV_MAX_LEVELS] = {};
  int64_t img_off[OFV_MAX_LEVELS] = {};   // element offset of level l inside a frame slab
  size_t frame_bytes = 0;                  // one frame's pyramid slab (sized for float32)
  size_t flow_bytes = 0;                   // one flow ping-pong buffer (2 planes of level 0)
  size_t slot_bytes = 0;                   // one pair: 2 slabs + 2 flow buffers
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // per-workgroup pixel counts of ofv_derived at the end of the workspace
  unsigned int* derived_counts = nullptr;
  // streaming (ofv_stream_push): slab of slot 0 holding the last pushed frame's pyramid
  bool stream_valid = false;
  int stream_slab = 0;
  int stream_w = 0, stream_h = 0;
  ofv_params stream_params{};
  std::string err;
  // work decomposition of the Gauss-Newton kernel: tuned table, forced choice
  struct TuneKey {
    int kr, storage, mode, w, hgt, n;
    bool operator<(const TuneKey& o) const {
      return std::tie(kr, storage, mode, w, hgt, n) < std::tie(o.kr, o.storage, o.mode, o.w, o.hgt, o.n);
    }
  };
  struct Choice {
    int variant, tile_h;
  };
  std::map<TuneKey, Choice> tuned;
  int forced_variant = -1;  // -1: tuned table, else the heuristic
  int forced_tile_h = 0;
  // event capture around Gauss-Newton launches (ofv_autotune only)
  bool capture = false;
  std::vector<hipEvent_t> events;
  size_t events_used = 0;
  struct Rec {
    TuneKey key;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  // backward workspace (ofv_reserve_backward): saved iterates, scratch planes, image-gradient pyramids
  float* bw = nullptr;
  size_t bw_bytes = 0;
  int bw_levels = 0, bw_iters = 0, bw_pairs = 0;
  bool bw_store_all = false;
  // the forward whose iterates (and pyramids) the workspace holds: a backward
  // with OFV_FLAG_SAVED_FORWARD on the same inputs skips its own forward
  struct SavedForward {
    bool valid = false;
    int n = 0;
    ofv_params params{};
    std::vector<ofv_image> f0, f1;
    std::vector<const float*> init;
  } saved_fw;
};

namespace {

ofv_status fail(ofv_ctx* h, ofv_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (h) h->err = buf; else g_create_error = buf;
  return s;
}

bool fault_injected(const char* what) {
  const char* e = std::getenv("OFV_FAULT_INJECT");
  return e && std::strstr(e, what) != nullptr;
}

// The library's only synchronisation points (ofv_destroy, ofv_autotune, a
// reserve_backward that replaces a smaller reservation) go through this;
// OFV_FAULT_INJECT=sync makes each report a device error.
hipError_t sync_stream(hipStream_t s) {
  if (fault_injected("sync")) return hipErrorLaunchFailure;
  return hipStreamSynchronize(s);
}

// Makes the handle's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (dev < 0) return;
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) changed = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

size_t pixel_bytes(int type) { return type == OFV_PIX_U8 ? 1 : (type == OFV_PIX_U16 ? 2 : 4); }
size_t storage_bytes(int st) { return st == OFV_STORE_F32 ? 4 : 2; }

// Byte range [lo, hi) touched by an image.
void image_range(const ofv_image* f, uintptr_t& lo, uintptr_t& hi) {
  lo = reinterpret_cast<uintptr_t>(f->data);
  hi = lo + (static_cast<uint64_t>(f->height - 1) * static_cast<uint64_t>(f->pitch) + f->width) *
                pixel_bytes(f->type);
}

bool overlap(uintptr_t a0, uintptr_t a1, uintptr_t b0, uintptr_t b1) { return a0 < b1 && b0 < a1; }

ofv_status check_image(ofv_ctx* h, const ofv_image* f, const char* name) {
  if (!f) return fail(h, OFV_ERR_INVALID_ARG, "%s is NULL", name);
  if (!f->data) return fail(h, OFV_ERR_INVALID_ARG, "%s->data is NULL", name);
  if (f->width < 1 || f->height < 1)
    return fail(h, OFV_ERR_INVALID_ARG, "%s has size %dx%d (must be >= 1x1)", name, f->width, f->height);
  if (f->pitch < f->width)
    return fail(h, OFV_ERR_INVALID_ARG, "%s pitch %lld < width %d", name, (long long)f->pitch, f->width);
  if (f->type == OFV_PIX_U8) {
    if (f->bit_depth < 1 || f->bit_depth > 8)
      return fail(h, OFV_ERR_INVALID_ARG, "%s: bit_depth %d invalid for U8 (1..8)", name, f->bit_depth);
  } else if (f->type == OFV_PIX_U16) {
    if (f->bit_depth < 1 || f->bit_depth > 16)
      return fail(h, OFV_ERR_INVALID_ARG, "%s: bit_depth %d invalid for U16 (1..16)", name, f->bit_depth);
  } else if (f->type != OFV_PIX_F32) {
    return fail(h, OFV_ERR_INVALID_ARG, "%s: unknown pixel type %d", name, f->type);
  }
  if (f->pitch >= kMaxPitch ||
      f->pitch * static_cast<int64_t>(f->height) * static_cast<int64_t>(pixel_bytes(f->type)) >= kMaxPlaneBytes)
    return fail(h, OFV_ERR_UNSUPPORTED, "%s: pitch of 2^24 elements or more, or 2 GiB or more", name);
  return OFV_OK;
}

ofv_status check_params(ofv_ctx* h, const ofv_params* p) {
  if (!p) return fail(h, OFV_ERR_INVALID_ARG, "params is NULL");
  if (p->num_levels < 1 || p->num_levels > OFV_MAX_LEVELS)
    return fail(h, OFV_ERR_INVALID_ARG, "num_levels %d outside 1..%d", p->num_levels, OFV_MAX_LEVELS);
  if (p->kernel_radius < 1) return fail(h, OFV_ERR_INVALID_ARG, "kernel_radius %d < 1", p->kernel_radius);
  if (p->kernel_radius > OFV_MAX_KERNEL_RADIUS)
    return fail(h, OFV_ERR_UNSUPPORTED, "kernel_radius %d > %d", p->kernel_radius, OFV_MAX_KERNEL_RADIUS);
  if (p->iterations < 1) return fail(h, OFV_ERR_INVALID_ARG, "iterations %d < 1", p->iterations);
  if (p->norm_radius < 0 || p->norm_radius > OFV_MAX_NORM_RADIUS)
    return fail(h, OFV_ERR_INVALID_ARG, "norm_radius %d outside 0..%d", p->norm_radius, OFV_MAX_NORM_RADIUS);
  if (!std::isfinite(p->norm_eps) || p->norm_eps < 0.0f)
    return fail(h, OFV_ERR_INVALID_ARG, "norm_eps must be finite and >= 0");
  if (!std::isfinite(p->reg_rel) || p->reg_rel < 0.0f || !std::isfinite(p->reg_abs) || p->reg_abs < 0.0f)
    return fail(h, OFV_ERR_INVALID_ARG, "reg_rel and reg_abs must be finite and >= 0");
  if (p->storage < OFV_STORE_F32 || p->storage > OFV_STORE_BF16)
    return fail(h, OFV_ERR_INVALID_ARG, "unknown storage %d", p->storage);
  if (p->flags & ~(OFV_FLAG_FORWARD_ADDITIVE | OFV_FLAG_INCREMENT_UPDATE | OFV_FLAG_NO_FP64_FALLBACK |
                   OFV_FLAG_STORE_ALL | OFV_FLAG_SAVE_ITERATES | OFV_FLAG_SAVED_FORWARD))
    return fail(h, OFV_ERR_INVALID_ARG, "unknown flags 0x%x", p->flags);
  return OFV_OK;
}

ofv_status check_handle(ofv_ctx* h) {
  if (!h) return OFV_ERR_INVALID_ARG;
  h->err.clear();
  return OFV_OK;
}

ofv_status device_error(ofv_ctx* h, hipError_t e, const char* where) {
  return fail(h, OFV_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

// ------------------------------------------------------------------ per-pair geometry and buffers

struct PairPlan {
  const ofv_image* f[2];
  const float* init;
  float* out;
  int lw[OFV_MAX_LEVELS], lh[OFV_MAX_LEVELS];
  char* slot;
  int slab[2] = {0, 1};          // pyramid slab of the slot that holds frame k
  bool built[2] = {false, false};  // frame k's pyramid is already in its slab (streaming)
};

void level_dims(int w, int hgt, int levels, int* lw, int* lh) {
  lw[0] = w;
  lh[0] = hgt;
  for (int l = 1; l < levels; ++l) {
    lw[l] = (lw[l - 1] + 1) / 2;
    lh[l] = (lh[l - 1] + 1) / 2;
  }
}

char* img_plane(const ofv_ctx* h, const PairPlan& pp, int frame, int level, size_t ts) {
  return pp.slot + pp.slab[frame] * h->frame_bytes + static_cast<size_t>(h->img_off[level]) * ts;
}

float* flow_buf(const ofv_ctx* h, const PairPlan& pp, int which) {
  return reinterpret_cast<float*>(pp.slot + 2 * h->frame_bytes + which * h->flow_bytes);
}

int choose_tile_h(int64_t strips_total, int64_t rows_max) {
  // Enough workgroups to cover 256 CUs several times, without making the
  // vertical halo (2 KR + 2 rows per tile) dominate.
  if (const char* e = std::getenv("OFV_TILE_H")) {
    int v = std::atoi(e);
    if (v >= 4 && v <= 1024) return v;
  }
  int th = 64;
  while (th > 16 && strips_total * ((rows_max + th - 1) / th) < 2048) th /= 2;
  return th;
}

// Work decomposition of the Gauss-Newton kernel for one launch group:
// OFV_GN_VARIANT in the environment, then a choice forced on the handle, then
// the handle's tuned table, then the default: from 3 Mi pixels per launch
// (enough to give every CU several strips) the band march for windows of
// KR >= 8 and the strip march below (measured on MI355X: at 5120 x 4096,
// KR 10 the band takes 229 us against 296 us for the strip march and more
// for every tile shape, in both the direct and the up-sampling flow mode;
// on 16 or 64 pairs of 2048^2 at KR 4 the strip march leads at 2048^2 and
// the band trails it), 64 x 16 tiles below 3 Mi pixels.  Levels one pixel
// wide or high always take the strip march.
void pick_gn_choice(const ofv_ctx* h, const ofv_ctx::TuneKey& key, int64_t strips, int64_t rows_max, int64_t pixels,
                    bool degenerate, int& variant, int& tile_h) {
  tile_h = choose_tile_h(strips, rows_max);
  if (degenerate) {  // a level of one row or one column: the tile kernels need 2 x 2 pixels
    variant = GN_MARCH;
    return;
  }
  if (const char* e = std::getenv("OFV_GN_VARIANT")) {
    if (!std::strcmp(e, "march")) { variant = GN_MARCH; return; }
    if (!std::strcmp(e, "tile64x32") || !std::strcmp(e, "tile32")) { variant = GN_TILE_64x32; return; }
    if (!std::strcmp(e, "tile64x16") || !std::strcmp(e, "tile16")) { variant = GN_TILE_64x16; return; }
    if (!std::strcmp(e, "tile32x16")) { variant = GN_TILE_32x16; return; }
    if (!std::strcmp(e, "tile16x16")) { variant = GN_TILE_16x16; return; }
    if (!std::strcmp(e, "tile64x64")) { variant = GN_TILE_64x64; return; }
    if (!std::strcmp(e, "tile64x32w")) { variant = GN_TILE_64x32W; return; }
    if (!std::strcmp(e, "tile64x16w")) { variant = GN_TILE_64x16W; return; }
    if (!std::strcmp(e, "tile16x16w")) { variant = GN_TILE_16x16W; return; }
    if (!std::strcmp(e, "tile32x16w")) { variant = GN_TILE_32x16W; return; }
    if (!std::strcmp(e, "tile32x32w")) { variant = GN_TILE_32x32W; return; }
    if (!std::strcmp(e, "band")) { variant = GN_BAND4; tile_h = 0; return; }
  }
  if (h->forced_variant >= 0) {
    variant = h->forced_variant;
    if (h->forced_tile_h > 0) tile_h = h->forced_tile_h;
    else if (variant == GN_BAND4) tile_h = 0;
    return;
  }
  auto it = h->tuned.find(key);
  if (it != h->tuned.end()) {
    variant = it->second.variant;
    tile_h = it->second.tile_h;
    return;
  }
  variant = pixels >= (int64_t{3} << 20) ? (key.kr >= 8 ? GN_BAND4 : GN_MARCH) : GN_TILE_64x16;
  if (variant == GN_BAND4) tile_h = 0;
}

// pick_gn_choice, then for the band decomposition without a tile height of
// its own (forced or tuned; 0 = none) the one from the occupancy query over
// the jobs of one launch (job j: band_strips[j] strips of band_rows[j] rows).
void pick_gn(const ofv_ctx* h, const ofv_ctx::TuneKey& key, int64_t strips, int64_t rows_max, int64_t pixels,
             bool degenerate, int& variant, int& tile_h, const int64_t* band_strips, const int64_t* band_rows,
             int band_jobs) {
  pick_gn_choice(h, key, strips, rows_max, pixels, degenerate, variant, tile_h);
  if (variant != GN_BAND4 || tile_h > 0) return;
  const int per_cu = std::max(1, gn_band_per_cu(key.kr, key.storage, key.mode));
  tile_h = gn_band_tile_h(band_strips, band_rows, band_jobs, static_cast<int64_t>(per_cu) * h->num_cus, key.kr);
}

hipEvent_t next_event(ofv_ctx* h) {
  if (h->events_used == h->events.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->events.push_back(e);
  }
  return h->events[h->events_used++];
}

// Launches jobs in chunks of kMaxJobs; `fill` writes job i into args and
// returns its block count.
template <typename Args, typename Fill, typename Launch>
ofv_status run_chunked(ofv_ctx* h, int njobs, Args& args, Fill fill, Launch launch, const char* what) {
  for (int base = 0; base < njobs; base += kMaxJobs) {
    const int cnt = std::min(kMaxJobs, njobs - base);
    args.njobs = cnt;
    int blocks = 0;
    for (int i = 0; i < cnt; ++i) {
      args.job[i].tile_start = blocks;
      blocks += fill(base + i, args.job[i]);
    }
    if (blocks == 0) continue;
    hipError_t e = launch(args, blocks);
    if (e != hipSuccess) return device_error(h, e, what);
  }
  return OFV_OK;
}

// Runs fill(job_index, job) for chunks of at most kMaxJobs jobs and launches each chunk.
template <typename Args, typename Fill, typename Launch>
ofv_status run_jobs(ofv_ctx* h, int njobs, Args& args, Fill fill, Launch launch, const char* what) {
  for (int base = 0; base < njobs; base += kMaxJobs) {
    const int cnt = std::min(kMaxJobs, njobs - base);
    args.njobs = cnt;
    for (int i = 0; i < cnt; ++i) fill(base + i, args.job[i]);
    hipError_t e = launch(args);
    if (e != hipSuccess) return device_error(h, e, what);
  }
  return OFV_OK;
}

// How far run_pipeline goes: the whole estimator, the pyramids only, or the
// pyramids and the initial field's restriction (everything before step 3).
enum PipeStop { PIPE_FULL = 0, PIPE_PYRAMID = 1, PIPE_NO_GN = 2 };

// save (optional): per (pair j, level l, iteration k) at index (j * L + l) *
// IT + k, the u plane that receives that iteration's output (v plane
// lpitch[l] * lh[l] further); the last iteration of level 0 writes the
// pair's flow_out instead where it has one.
ofv_status run_pipeline(ofv_ctx* h, int n, PairPlan* pp, const ofv_params* p, float* const* save = nullptr,
                        PipeStop stop = PIPE_FULL) {
  // any run rewrites the slabs of the slots it uses: a retained streaming frame
  // and a saved forward are gone
  h->stream_valid = false;
  h->saved_fw.valid = false;
  const int L = p->num_levels;
  // estimator variants other than the symmetric estimator's consistent update
  // run on the generic kernels, which read them at run time
  const bool generic = (p->flags & (OFV_FLAG_FORWARD_ADDITIVE | OFV_FLAG_INCREMENT_UPDATE)) != 0;
  const uint32_t est = ((p->flags & OFV_FLAG_FORWARD_ADDITIVE) ? EST_FORWARD_ADDITIVE : 0u) |
                       ((p->flags & OFV_FLAG_INCREMENT_UPDATE) ? EST_INCREMENT : 0u) |
                       ((p->flags & OFV_FLAG_NO_FP64_FALLBACK) ? EST_NO_FP64 : 0u);
  const int kr = p->kernel_radius;
  const int it = p->iterations;
  const int st = p->storage;
  const size_t ts = storage_bytes(st);
  hipStream_t s = h->stream;

  // frames whose pyramid is still to be built: (pair, frame)
  std::vector<std::pair<int, int>> fj;
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < 2; ++k)
      if (!pp[j].built[k]) fj.emplace_back(j, k);
  const int nf = static_cast<int>(fj.size());
  // Step 1: normalisation of both frames of every pair -> level 0.
  {
    NormArgs na{};
    na.nr = p->norm_radius;
    na.eps = p->norm_eps;
    na.storage = st;
    auto fill = [&](int i, NormJob& J) {
      const PairPlan& q = pp[fj[i].first];
      const ofv_image* f = q.f[fj[i].second];
      J.in = f->data;
      J.in_pitch = f->pitch;
      J.type = f->type;
      J.bits = f->bit_depth;
      J.w = f->width;
      J.h = f->height;
      J.out = img_plane(h, q, fj[i].second, 0, ts);
      J.out_pitch = h->lpitch[0];
      return ((J.w + kNormTW - 1) / kNormTW) * ((J.h + kNormTH - 1) / kNormTH);
    };
    ofv_status r = run_chunked(h, nf, na, fill,
                               [&](const NormArgs& a, int b) { return launch_normalize(a, b, s); }, "normalize");
    if (r != OFV_OK) return r;
  }
  // Step 2: pyramid levels 1..L-1 of both frames, up to three levels per
  // launch; launches over 16 Mi input pixels or more build one level each
  // (there the three-level workgroups, which stage their finest region with
  // the halo of all three levels, 2x the owned pixels, run at half the
  // single-level kernel's rate: 5120 x 4096 float32 plane 56 us in one
  // launch, 45 us in three; below 4 Mi pixels the one launch wins).
  for (int l = 1; l < L;) {
    int64_t lpx = 0;  // input pixels of this launch
    for (const auto& f : fj) lpx += static_cast<int64_t>(pp[f.first].lw[l - 1]) * pp[f.first].lh[l - 1];
    const int nlev = lpx >= kReduceSingleLevelPixels ? 1 : std::min(kMaxReduceLevels, L - l);
    ofv_status r = OFV_OK;
    if (nlev == 1) {
      ReduceArgs ra{};
      ra.storage = st;
      ra.scale = 1.0f;
      auto fill = [&](int i, ReduceJob& J) {
        const PairPlan& q = pp[fj[i].first];
        J.in = img_plane(h, q, fj[i].second, l - 1, ts);
        J.out = img_plane(h, q, fj[i].second, l, ts);
        J.in_pitch = h->lpitch[l - 1];
        J.out_pitch = h->lpitch[l];
        J.w = q.lw[l - 1];
        J.h = q.lh[l - 1];
        return static_cast<int>(reduce_blocks(q.lw[l], q.lh[l]));
      };
      r = run_chunked(h, nf, ra, fill, [&](const ReduceArgs& a, int b) { return launch_reduce(a, b, s); },
                      "reduce");
    } else {
      ReduceMArgs ra{};
      ra.storage = st;
      int64_t px = 0;  // input pixels of the launches
      for (const auto& f : fj) px += static_cast<int64_t>(pp[f.first].lw[l - 1]) * pp[f.first].lh[l - 1];
      const bool small = reduce_multi_small(nlev, px);
      int tw = 0, th = 0;
      reduce_multi_tile(nlev, small, tw, th);
      auto fill = [&](int i, ReduceMJob& J) {
        const PairPlan& q = pp[fj[i].first];
        J.in = img_plane(h, q, fj[i].second, l - 1, ts);
        J.in_pitch = h->lpitch[l - 1];
        for (int k = 0; k < nlev; ++k) {
          J.out[k] = img_plane(h, q, fj[i].second, l + k, ts);
          J.out_pitch[k] = h->lpitch[l + k];
        }
        J.w = q.lw[l - 1];
        J.h = q.lh[l - 1];
        const int d = l + nlev - 1;  // deepest level of the launch
        return ((q.lw[d] + tw - 1) / tw) * ((q.lh[d] + th - 1) / th);
      };
      r = run_chunked(h, nf, ra, fill,
                      [&](const ReduceMArgs& a, int b) { return launch_reduce_multi(a, nlev, small, b, s); },
                      "reduce");
    }
    if (r != OFV_OK) return r;
    l += nlev;
  }
  if (stop == PIPE_PYRAMID) return OFV_OK;
  // Initial flow: restricted to the coarsest level by REDUCE / 2 (pairs that have one).
  std::vector<int> cur(n, -1);  // flow buffer holding the current field, -1 = zero field
  std::vector<int> with_init;
  for (int j = 0; j < n; ++j)
    if (pp[j].init) with_init.push_back(j);
  if (!with_init.empty()) {
    const int ni = static_cast<int>(with_init.size());
    if (L == 1) {
      // copy, so that flow_init may alias flow_out
      for (int j : with_init) {
        const int w = pp[j].lw[0], hh = pp[j].lh[0];
        float* dst = flow_buf(h, pp[j], 1);
        for (int c = 0; c < 2; ++c) {
          hipError_t e = hipMemcpy2DAsync(dst + c * h->lpitch[0] * h->lh[0], h->lpitch[0] * sizeof(float),
                                          pp[j].init + static_cast<int64_t>(c) * w * hh, w * sizeof(float),
                                          w * sizeof(float), hh, hipMemcpyDeviceToDevice, s);
          if (e != hipSuccess) return device_error(h, e, "flow_init copy");
        }
        cur[j] = 1;
      }
    } else {
      for (int l = 1; l < L; ++l) {
        ReduceArgs ra{};
        ra.storage = ST_F32;
        ra.scale = 0.5f;
        auto fill = [&](int i, ReduceJob& J) {
          const PairPlan& q = pp[with_init[i / 2]];
          const int c = i % 2;
          if (l == 1) {
            J.in = q.init + static_cast<int64_t>(c) * q.lw[0] * q.lh[0];
            J.in_pitch = q.lw[0];
          } else {
            J.in = flow_buf(h, q, (l - 1) & 1) + c * h->lpitch[l - 1] * h->lh[l - 1];
            J.in_pitch = h->lpitch[l - 1];
          }
          J.out = flow_buf(h, q, l & 1) + c * h->lpitch[l] * h->lh[l];
          J.out_pitch = h->lpitch[l];
          J.w = q.lw[l - 1];
          J.h = q.lh[l - 1];
          return static_cast<int>(reduce_blocks(q.lw[l], q.lh[l]));
        };
        ofv_status r = run_chunked(h, 2 * ni, ra, fill,
                                   [&](const ReduceArgs& a, int b) { return launch_reduce(a, b, s); },
                                   "restrict flow_init");
        if (r != OFV_OK) return r;
      }
      for (int j : with_init) cur[j] = (L - 1) & 1;
    }
  }
  if (stop == PIPE_NO_GN) return OFV_OK;
  // Steps 3-6: Gauss-Newton iterations, coarse to fine; the up-sampling of
  // step 4 is fused into the first iteration of every finer level and the
  // last level-0 iteration writes the caller's buffer.
  const int tx = gn_tile_w(kr);
  for (int l = L - 1; l >= 0; --l) {
    int64_t strips = 0, rows_max = 0;
    for (int j = 0; j < n; ++j) {
      strips += (pp[j].lw[l] + tx - 1) / tx;
      rows_max = std::max<int64_t>(rows_max, pp[j].lh[l]);
    }
    for (int k = 0; k < it; ++k) {
      const bool final_iter = (l == 0 && k == it - 1);
      GnArgs ga{};
      ga.reg_rel = p->reg_rel;
      ga.reg_abs = p->reg_abs;
      ga.est = est;
      std::vector<int> next(n);
      // the input-flow mode is a compile-time property of the kernel: group pairs by it
      auto mode_of = [&](int j) {
        if (k == 0 && l < L - 1) return static_cast<int>(FLOW_UPSAMPLE);
        return static_cast<int>(cur[j] < 0 ? FLOW_ZERO : FLOW_DIRECT);
      };
      // levels thinner than 2 pixels go to the march in a launch of their own,
      // so the decomposition of every other pair does not depend on them
      for (int gk = 0; gk < 2 * (FLOW_UPSAMPLE + 1); ++gk) {
        const int mode = gk >> 1;
        const bool thin = gk & 1;
        std::vector<int> group;
        for (int j = 0; j < n; ++j)
          if (mode_of(j) == mode && (pp[j].lw[l] < 2 || pp[j].lh[l] < 2) == thin) group.push_back(j);
        if (group.empty()) continue;
        ofv_ctx::TuneKey key{kr, st, mode, 0, 0, static_cast<int>(group.size())};
        for (int j : group) {
          key.w = std::max(key.w, pp[j].lw[l]);
          key.hgt = std::max(key.hgt, pp[j].lh[l]);
        }
        int variant = 0, tile_h = 0, tw = 0, th = 0;
        int64_t pixels = 0;
        for (int j : group) pixels += static_cast<int64_t>(pp[j].lw[l]) * pp[j].lh[l];
        // the band's tile height from the jobs of the group's largest launch (the first kMaxJobs)
        int64_t bs[kMaxJobs], br[kMaxJobs];
        const int bj = std::min<int>(kMaxJobs, static_cast<int>(group.size()));
        for (int gi = 0; gi < bj; ++gi) {
          bs[gi] = (pp[group[gi]].lw[l] + tx - 1) / tx;
          br[gi] = pp[group[gi]].lh[l];
        }
        pick_gn(h, key, strips, rows_max, pixels, thin, variant, tile_h, bs, br, bj);
        if (generic && variant == GN_BAND4) {  // the band has no generic-estimator build: the strip march
          variant = GN_MARCH;
          tile_h = choose_tile_h(strips, rows_max);
        }
        if (generic && variant != GN_MARCH) variant = GN_TILE_16x16;   // the generic estimator's tiles
        gn_tile_dims(variant, kr, tile_h, tw, th);
        ga.tile_h = tile_h;
        auto fill = [&](int gi, GnJob& J) {
          const int j = group[gi];
          const PairPlan& q = pp[j];
          J.p0 = img_plane(h, q, 0, l, ts);
          J.p1 = img_plane(h, q, 1, l, ts);
          J.img_pitch = h->lpitch[l];
          J.w = q.lw[l];
          J.h = q.lh[l];
          J.cw = l + 1 < L ? q.lw[l + 1] : 0;
          J.ch = l + 1 < L ? q.lh[l + 1] : 0;
          J.mode = mode;
          if (mode == FLOW_UPSAMPLE) {
            const float* src = flow_buf(h, q, cur[j]);
            J.in_u = src;
            J.in_v = src + h->lpitch[l + 1] * h->lh[l + 1];
            J.in_pitch = h->lpitch[l + 1];
          } else if (mode == FLOW_ZERO) {
            J.in_u = J.in_v = nullptr;
            J.in_pitch = 0;
          } else {
            const float* src = flow_buf(h, q, cur[j]);
            J.in_u = src;
            J.in_v = src + h->lpitch[l] * h->lh[l];
            J.in_pitch = h->lpitch[l];
          }
          if (save) {
            // every iteration reads its predecessor's saved output and writes its own slot
            if (mode == FLOW_UPSAMPLE) {
              J.in_u = save[(j * L + l + 1) * it + it - 1];
              J.in_v = J.in_u + h->lpitch[l + 1] * h->lh[l + 1];
            } else if (mode == FLOW_DIRECT && k >= 1) {
              J.in_u = save[(j * L + l) * it + k - 1];
              J.in_v = J.in_u + h->lpitch[l] * h->lh[l];
              J.in_pitch = h->lpitch[l];
            }
            if (final_iter && q.out) {
              // the adjoint never reads the last output: it goes to the caller's buffer
              J.out_u = q.out;
              J.out_v = q.out + static_cast<int64_t>(q.lw[0]) * q.lh[0];
              J.out_pitch = q.lw[0];
            } else {
              J.out_u = save[(j * L + l) * it + k];
              J.out_v = J.out_u + h->lpitch[l] * h->lh[l];
              J.out_pitch = h->lpitch[l];
            }
            next[j] = 0;
          } else if (final_iter) {
            J.out_u = q.out;
            J.out_v = q.out + static_cast<int64_t>(q.lw[0]) * q.lh[0];
            J.out_pitch = q.lw[0];
            next[j] = -2;
          } else {
            const int nb = cur[j] == 0 ? 1 : 0;
            float* dst = flow_buf(h, q, nb);
            J.out_u = dst;
            J.out_v = dst + h->lpitch[l] * h->lh[l];
            J.out_pitch = h->lpitch[l];
            next[j] = nb;
          }
          return static_cast<int>(((q.lw[l] + tw - 1) / tw) * ((q.lh[l] + th - 1) / th));
        };
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        if (h->capture) {
          ev0 = next_event(h);
          ev1 = next_event(h);
          if (!ev0 || !ev1) return fail(h, OFV_ERR_DEVICE, "hipEventCreate failed while tuning");
          (void)hipEventRecord(ev0, s);
        }
        ofv_status r = run_chunked(h, static_cast<int>(group.size()), ga, fill,
                                   [&](const GnArgs& a, int b) { return launch_gn(a, kr, st, mode, variant, b, s, generic); },
                                   "gauss-newton iteration");
        if (r != OFV_OK) return r;
        if (h->capture) {
          (void)hipEventRecord(ev1, s);
          h->recs.push_back({key, ev0, ev1});
        }
      }
      cur = next;
    }
  }
  return OFV_OK;
}

ofv_status validate_pair(ofv_ctx* h, const ofv_image* f0, const ofv_image* f1, const float* init,
                         const float* out, int idx) {
  char n0[32], n1[32];
  snprintf(n0, sizeof n0, "frame0[%d]", idx);
  snprintf(n1, sizeof n1, "frame1[%d]", idx);
  ofv_status r = check_image(h, f0, n0);
  if (r != OFV_OK) return r;
  r = check_image(h, f1, n1);
  if (r != OFV_OK) return r;
  if (f0->width != f1->width || f0->height != f1->height)
    return fail(h, OFV_ERR_INVALID_ARG, "pair %d: frame sizes differ (%dx%d vs %dx%d)", idx, f0->width,
                f0->height, f1->width, f1->height);
  if (!out) return fail(h, OFV_ERR_INVALID_ARG, "flow_out[%d] is NULL", idx);
  if (f0->width > h->max_w || f0->height > h->max_h)
    return fail(h, OFV_ERR_CAPACITY, "pair %d: %dx%d exceeds the handle's %dx%d", idx, f0->width, f0->height,
                h->max_w, h->max_h);
  const uintptr_t o0 = reinterpret_cast<uintptr_t>(out);
  const uintptr_t o1 = o0 + 2ull * f0->width * f0->height * sizeof(float);
  uintptr_t a0, a1;
  image_range(f0, a0, a1);
  if (overlap(o0, o1, a0, a1)) return fail(h, OFV_ERR_INVALID_ARG, "flow_out[%d] overlaps frame0", idx);
  image_range(f1, a0, a1);
  if (overlap(o0, o1, a0, a1)) return fail(h, OFV_ERR_INVALID_ARG, "flow_out[%d] overlaps frame1", idx);
  if (init && init != out) {
    const uintptr_t i0 = reinterpret_cast<uintptr_t>(init);
    if (overlap(o0, o1, i0, i0 + (o1 - o0)))
      return fail(h, OFV_ERR_INVALID_ARG, "flow_init[%d] partially overlaps flow_out", idx);
  }
  return OFV_OK;
}

// Level-0 scratch planes of one pair: dL/dA and the solve's direct gradient
// (7), three gradient fields in rotation (6), the input field of a level's
// first iteration (2).
constexpr int kBwScratchPlanes = 15;

// Floats of one pair's backward workspace: the output field of every
// (level, iteration); in store-all mode also, per (level, iteration), the
// five window sums and Gx, Gy, b, and per level the first iteration's input
// field; the scratch planes.  The image-gradient pyramids of all pairs
// follow the pair blocks, contiguous, so one fill clears them.
struct BwLayout {
  size_t saved = 0, record = 0, scratch = 0, pair = 0, gpyr = 0;
};

BwLayout bw_layout(const ofv_ctx* h, int levels, int iters, bool store_all) {
  BwLayout b;
  for (int l = 0; l < levels; ++l) {
    const size_t pl = static_cast<size_t>(h->lpitch[l]) * h->lh[l];
    b.saved += static_cast<size_t>(iters) * 2 * pl;
    if (store_all) b.record += (static_cast<size_t>(iters) * 8 + 2) * pl;
  }
  b.scratch = kBwScratchPlanes * static_cast<size_t>(h->lpitch[0]) * h->lh[0];
  b.pair = b.saved + b.record + b.scratch;
  b.gpyr = h->frame_bytes / 2;  // two float32 pyramid slabs (frame_bytes is one slab in bytes)
  return b;
}

size_t bw_total_bytes(const ofv_ctx* h, int levels, int iters, int pairs, bool store_all) {
  const BwLayout b = bw_layout(h, levels, iters, store_all);
  return (b.pair + b.gpyr) * static_cast<size_t>(pairs) * sizeof(float);
}

// Addresses in the reserved backward workspace (offsets from the reserved
// levels and iterations, so they do not depend on the call's).
struct BwView {
  const ofv_ctx* h;
  BwLayout lay;
  explicit BwView(const ofv_ctx* c) : h(c), lay(bw_layout(c, c->bw_levels, c->bw_iters, c->bw_store_all)) {}
  size_t plane(int l) const { return static_cast<size_t>(h->lpitch[l]) * h->lh[l]; }
  float* pair(int j) const { return h->bw + static_cast<size_t>(j) * lay.pair; }
  float* saved(int j, int l, int k) const {
    size_t o = 0;
    for (int i = 0; i < l; ++i) o += static_cast<size_t>(h->bw_iters) * 2 * plane(i);
    return pair(j) + o + static_cast<size_t>(k) * 2 * plane(l);
  }
  float* rec_level(int j, int l) const {
    size_t o = lay.saved;
    for (int i = 0; i < l; ++i) o += (static_cast<size_t>(h->bw_iters) * 8 + 2) * plane(i);
    return pair(j) + o;
  }
  float* rec(int j, int l, int k) const { return rec_level(j, l) + static_cast<size_t>(k) * 8 * plane(l); }
  float* rec_in(int j, int l) const { return rec_level(j, l) + static_cast<size_t>(h->bw_iters) * 8 * plane(l); }
  float* scratch(int j, int q) const {
    return pair(j) + lay.saved + lay.record + static_cast<size_t>(q) * h->lpitch[0] * h->lh[0];
  }
  float* gpyr_all() const { return h->bw + static_cast<size_t>(h->bw_pairs) * lay.pair; }
  float* gpyr(int j, int f, int l) const {
    return gpyr_all() + static_cast<size_t>(j) * lay.gpyr + static_cast<size_t>(f) * (h->frame_bytes / 4) +
           h->img_off[l];
  }
};

// One batched backward (or saving forward) call: the pairs, their levels and
// where their fields live in the backward workspace.
struct BwPlan {
  ofv_ctx* h;
  int n, L, IT, kr;
  const ofv_params* params;
  bool store_all;
  BwView bv;
  std::vector<PairPlan> pp;
  hipStream_t s;
  int sp0, plane0;

  BwPlan(ofv_ctx* c, int npairs, const ofv_params* p)
      : h(c), n(npairs), L(p->num_levels), IT(p->iterations), kr(p->kernel_radius), params(p),
        store_all((p->flags & OFV_FLAG_STORE_ALL) != 0), bv(c), pp(npairs), s(c->stream),
        sp0(static_cast<int>(c->lpitch[0])), plane0(static_cast<int>(c->lpitch[0] * c->lh[0])) {}

  int lp(int l) const { return static_cast<int>(h->lpitch[l]); }
  int lplane(int l) const { return static_cast<int>(h->lpitch[l] * h->lh[l]); }
  // the restricted initial field (coarsest level), in the pair's flow buffer
  float* init_field(int j) const { return flow_buf(h, pp[j], L == 1 ? 1 : (L - 1) & 1); }

  struct Field {
    float* u;
    int pitch;  // row pitch
    int vstep;  // v plane = u + vstep
  };
  // input field of the first iteration of a level: up-sampled (levels above
  // the coarsest), the restricted initial field, or zero
  Field vin0(int j, int l) const {
    if (l == L - 1 && pp[j].init) return {init_field(j), lp(l), lplane(l)};
    if (store_all) return {bv.rec_in(j, l), lp(l), lplane(l)};
    return {bv.scratch(j, 13), lp(l), lplane(l)};
  }

  // fills the first iteration's input planes of level l (up-sampling or zeros), one launch
  ofv_status prepare_vin0(int l) {
    AuxArgs ua{};
    int mw = 0, mh = 0;
    std::vector<int> js;
    for (int j = 0; j < n; ++j) {
      if (l == L - 1 && pp[j].init) continue;
      js.push_back(j);
      mw = std::max(mw, pp[j].lw[l]);
      mh = std::max(mh, pp[j].lh[l]);
    }
    const bool up = l < L - 1;
    return run_jobs(h, static_cast<int>(js.size()), ua, [&](int i, AuxJob& J) {
      const int j = js[i];
      if (up) {
        J.in0 = bv.saved(j, l + 1, IT - 1);
        J.in1 = J.in0 + lplane(l + 1);
        J.ip = lp(l + 1);
        J.cw = pp[j].lw[l + 1];
        J.ch = pp[j].lh[l + 1];
      }
      const Field f = vin0(j, l);
      J.out0 = f.u;
      J.out1 = f.u + f.vstep;
      J.op = f.pitch;
      J.w = pp[j].lw[l];
      J.h = pp[j].lh[l];
    }, [&](const AuxArgs& a) { return up ? launch_upsample_batch(a, mw, mh, s) : launch_zero_fields(a, mw, mh, s); },
                    up ? "up-sampling" : "fill");
  }

  // The forward, keeping each iteration's output in the workspace (the last
  // of level 0 goes to the pair's flow_out where it has one); store-all: the
  // recording iterations, which also keep each iteration's sums and Gx, Gy, b.
  ofv_status forward() {
    if (!store_all) {
      std::vector<float*> save(static_cast<size_t>(n) * L * IT);
      for (int j = 0; j < n; ++j)
        for (int l = 0; l < L; ++l)
          for (int k = 0; k < IT; ++k) save[(static_cast<size_t>(j) * L + l) * IT + k] = bv.saved(j, l, k);
      return run_pipeline(h, n, pp.data(), params, save.data());
    }
    ofv_status r = run_pipeline(h, n, pp.data(), params, nullptr, PIPE_NO_GN);
    if (r != OFV_OK) return r;
    for (int l = L - 1; l >= 0; --l) {
      r = prepare_vin0(l);
      if (r != OFV_OK) return r;
      int64_t px = 0;
      for (int j = 0; j < n; ++j) px += static_cast<int64_t>(pp[j].lw[l]) * pp[j].lh[l];
      const int ty = adj_tile_h(px);
      for (int k = 0; k < IT; ++k) {
        AdjArgs aa{};
        aa.reg_rel = params->reg_rel;
        aa.reg_abs = params->reg_abs;
        aa.no_fp64 = (params->flags & OFV_FLAG_NO_FP64_FALLBACK) ? 1 : 0;
        int blocks = 0;
        r = run_jobs(h, n, aa, [&](int j, AdjJob& J) {
          if ((j % kMaxJobs) == 0) blocks = 0;
          J = AdjJob{};
          J.p0 = reinterpret_cast<const float*>(img_plane(h, pp[j], 0, l, 4));
          J.p1 = reinterpret_cast<const float*>(img_plane(h, pp[j], 1, l, 4));
          J.ip = lp(l);
          if (k == 0) {
            const Field f = vin0(j, l);
            J.vu = f.u;
            J.vv = f.u + f.vstep;
            J.vp = f.pitch;
          } else {
            J.vu = bv.saved(j, l, k - 1);
            J.vv = J.vu + lplane(l);
            J.vp = lp(l);
          }
          if (l == 0 && k == IT - 1 && pp[j].out) {
            J.ou = pp[j].out;
            J.ov = pp[j].out + static_cast<int64_t>(pp[j].lw[0]) * pp[j].lh[0];
            J.op = pp[j].lw[0];
          } else {
            J.ou = bv.saved(j, l, k);
            J.ov = J.ou + lplane(l);
            J.op = lp(l);
          }
          J.st = bv.rec(j, l, k);
          J.stp = lp(l);
          J.sts = lplane(l);
          J.w = pp[j].lw[l];
          J.h = pp[j].lh[l];
          J.tile_start = blocks;
          blocks += adj_sums_blocks(J.w, J.h, ty);
        }, [&](const AdjArgs& a) { return launch_adj_sums(a, kr, ADJ_RECORD, ty, blocks, s); }, "recording iteration");
        if (r != OFV_OK) return r;
      }
    }
    return OFV_OK;
  }
};

// Flags that do not change what a forward computes or keeps.
constexpr uint32_t kSaveFlags = OFV_FLAG_SAVE_ITERATES | OFV_FLAG_SAVED_FORWARD;

bool same_image(const ofv_image& a, const ofv_image& b) {
  return a.data == b.data && a.width == b.width && a.height == b.height && a.pitch == b.pitch && a.type == b.type &&
         a.bit_depth == b.bit_depth;
}

bool same_params(const ofv_params& a, const ofv_params& b) {
  return a.num_levels == b.num_levels && a.kernel_radius == b.kernel_radius && a.iterations == b.iterations &&
         a.norm_radius == b.norm_radius && a.norm_eps == b.norm_eps && a.reg_rel == b.reg_rel &&
         a.reg_abs == b.reg_abs && a.storage == b.storage && (a.flags & ~kSaveFlags) == (b.flags & ~kSaveFlags);
}

void record_saved_forward(ofv_ctx* h, int n, const ofv_image* f0, const ofv_image* f1, const float* const* init,
                          const ofv_params* p) {
  auto& sf = h->saved_fw;
  sf.valid = true;
  sf.n = n;
  sf.params = *p;
  sf.f0.assign(f0, f0 + n);
  sf.f1.assign(f1, f1 + n);
  sf.init.assign(n, nullptr);
  for (int j = 0; j < n; ++j) sf.init[j] = init ? init[j] : nullptr;
}

bool saved_forward_matches(const ofv_ctx* h, int n, const ofv_image* f0, const ofv_image* f1,
                           const float* const* init, const ofv_params* p) {
  const auto& sf = h->saved_fw;
  if (!sf.valid || sf.n != n || !same_params(sf.params, *p)) return false;
  for (int j = 0; j < n; ++j)
    if (!same_image(sf.f0[j], f0[j]) || !same_image(sf.f1[j], f1[j]) || sf.init[j] != (init ? init[j] : nullptr))
      return false;
  return true;
}

// A forward that saves its iterates for the adjoint (OFV_FLAG_SAVE_ITERATES):
// the adjoint's estimator and storage, and a reservation that holds them.
ofv_status check_saving(ofv_ctx* h, int n, const ofv_params* p) {
  if (p->flags & (OFV_FLAG_FORWARD_ADDITIVE | OFV_FLAG_INCREMENT_UPDATE))
    return fail(h, OFV_ERR_UNSUPPORTED, "the adjoint covers the symmetric estimator's consistent update only");
  if (p->storage != OFV_STORE_F32) return fail(h, OFV_ERR_UNSUPPORTED, "the adjoint needs F32 storage");
  const bool sa = (p->flags & OFV_FLAG_STORE_ALL) != 0;
  if (!h->bw || p->num_levels > h->bw_levels || p->iterations > h->bw_iters || n > h->bw_pairs ||
      (sa && !h->bw_store_all))
    return fail(h, OFV_ERR_CAPACITY,
                "backward workspace holds %d levels x %d iterations x %d pairs%s; call ofv_reserve_backward_ex",
                h->bw_levels, h->bw_iters, h->bw_pairs, h->bw_store_all ? " (store-all)" : "");
  return OFV_OK;
}

ofv_status compute_common(ofv_ctx* h, int n, const ofv_image* f0, const ofv_image* f1, const ofv_params* p,
                          const float* const* init, float* const* out) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (n < 1) return fail(h, OFV_ERR_INVALID_ARG, "batch size %d < 1", n);
  if (!f0 || !f1 || !out) return fail(h, OFV_ERR_INVALID_ARG, "frame or flow_out array is NULL");
  ofv_status r = check_params(h, p);
  if (r != OFV_OK) return r;
  if (n > h->max_batch) return fail(h, OFV_ERR_CAPACITY, "batch %d exceeds max_batch %d", n, h->max_batch);
  for (int j = 0; j < n; ++j) {
    r = validate_pair(h, &f0[j], &f1[j], init ? init[j] : nullptr, out[j], j);
    if (r != OFV_OK) return r;
  }
  for (int j = 0; j < n; ++j) {
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(out[j]);
    const uintptr_t a1 = a0 + 2ull * f0[j].width * f0[j].height * sizeof(float);
    for (int i = 0; i < n; ++i) {
      if (i == j) continue;
      const uintptr_t b0 = reinterpret_cast<uintptr_t>(out[i]);
      const uintptr_t b1 = b0 + 2ull * f0[i].width * f0[i].height * sizeof(float);
      if (overlap(a0, a1, b0, b1)) return fail(h, OFV_ERR_INVALID_ARG, "flow_out[%d] overlaps flow_out[%d]", j, i);
      uintptr_t c0, c1;
      image_range(&f0[i], c0, c1);
      if (overlap(a0, a1, c0, c1)) return fail(h, OFV_ERR_INVALID_ARG, "flow_out[%d] overlaps frame0[%d]", j, i);
      image_range(&f1[i], c0, c1);
      if (overlap(a0, a1, c0, c1)) return fail(h, OFV_ERR_INVALID_ARG, "flow_out[%d] overlaps frame1[%d]", j, i);
    }
  }
  const bool save = (p->flags & OFV_FLAG_SAVE_ITERATES) != 0;
  if (save) {
    r = check_saving(h, n, p);
    if (r != OFV_OK) return r;
  }
  if (fault_injected("launch")) return fail(h, OFV_ERR_DEVICE, "injected launch failure");
  if (h->device < 0) return fail(h, OFV_ERR_UNSUPPORTED, "validation-only handle (created with device -1)");
  DeviceGuard g(h->device);
  std::vector<PairPlan> pp(n);
  for (int j = 0; j < n; ++j) {
    pp[j].f[0] = &f0[j];
    pp[j].f[1] = &f1[j];
    pp[j].init = init ? init[j] : nullptr;
    pp[j].out = out[j];
    pp[j].slot = h->ws + static_cast<size_t>(j) * h->slot_bytes;
    level_dims(f0[j].width, f0[j].height, p->num_levels, pp[j].lw, pp[j].lh);
  }
  if (!save) return run_pipeline(h, n, pp.data(), p);
  BwPlan bp(h, n, p);
  bp.pp = pp;
  r = bp.forward();
  if (r == OFV_OK) record_saved_forward(h, n, f0, f1, init, p);
  return r;
}

// Workspace layout of a handle for pairs up to w x hgt: level sizes and
// pitches, each level's offset in a frame's pyramid slab (sized for float32
// planes), and the bytes of one pair's slot (two slabs, two flow buffers).
void set_geometry(ofv_ctx* h, int w, int hgt, int batch) {
  h->max_w = w;
  h->max_h = hgt;
  h->max_batch = batch;
  level_dims(w, hgt, OFV_MAX_LEVELS, h->lw, h->lh);
  int64_t off = 0;
  for (int l = 0; l < OFV_MAX_LEVELS; ++l) {
    h->lpitch[l] = round_up(h->lw[l], kPitchAlign);
    h->img_off[l] = off;
    off += h->lpitch[l] * h->lh[l];
  }
  h->frame_bytes = round_up(off * 4, kSlabAlign);
  h->flow_bytes = round_up(2 * h->lpitch[0] * h->lh[0] * 4, kSlabAlign);
  h->slot_bytes = 2 * h->frame_bytes + 2 * h->flow_bytes;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

void ofv_default_params(ofv_params* p) {
  if (!p) return;
  p->num_levels = 3;
  p->kernel_radius = 4;
  p->iterations = 3;
  p->norm_radius = 1;
  p->norm_eps = 1e-4f;
  p->reg_rel = 1e-3f;
  p->reg_abs = 1e-9f;
  p->storage = OFV_STORE_F32;
  p->flags = 0;
}

const char* ofv_status_string(ofv_status s) {
  switch (s) {
    case OFV_OK: return "ok";
    case OFV_ERR_INVALID_ARG: return "invalid argument";
    case OFV_ERR_UNSUPPORTED: return "unsupported";
    case OFV_ERR_CAPACITY: return "exceeds workspace capacity";
    case OFV_ERR_OUT_OF_MEMORY: return "out of device memory";
    case OFV_ERR_DEVICE: return "device error";
  }
  return "unknown status";
}

const char* ofv_last_error(ofv_handle h) { return h ? h->err.c_str() : g_create_error.c_str(); }

ofv_status ofv_create(ofv_handle* out, int device, int max_width, int max_height, int max_batch, void* stream) {
  g_create_error.clear();
  if (!out) return fail(nullptr, OFV_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (max_width < 1 || max_height < 1 || max_batch < 1)
    return fail(nullptr, OFV_ERR_INVALID_ARG, "max sizes must be >= 1 (got %dx%d, batch %d)", max_width, max_height,
                max_batch);
  if (device < -1) return fail(nullptr, OFV_ERR_INVALID_ARG, "device %d < -1", device);
  if (round_up(max_width, kPitchAlign) >= kMaxPitch ||
      static_cast<int64_t>(round_up(max_width, kPitchAlign)) * max_height * 4 >= kMaxPlaneBytes)
    return fail(nullptr, OFV_ERR_UNSUPPORTED, "a %dx%d float plane would reach 2 GiB", max_width, max_height);
  ofv_ctx* h = new (std::nothrow) ofv_ctx();
  if (!h) return fail(nullptr, OFV_ERR_OUT_OF_MEMORY, "host allocation failed");
  h->device = device;
  h->stream = static_cast<hipStream_t>(stream);
  set_geometry(h, max_width, max_height, max_batch);
  h->ws_bytes = h->slot_bytes * static_cast<size_t>(max_batch) + kDerivedMaxBlocks * sizeof(unsigned int);
  if (device >= 0) {
    if (fault_injected("alloc")) {
      delete h;
      return fail(nullptr, OFV_ERR_OUT_OF_MEMORY, "injected allocation failure");
    }
    DeviceGuard g(device);
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess || cur != device) {
      delete h;
      return fail(nullptr, OFV_ERR_DEVICE, "cannot select device %d: %s", device,
                  hipGetErrorString(e != hipSuccess ? e : hipErrorInvalidDevice));
    }
    e = hipMalloc(reinterpret_cast<void**>(&h->ws), h->ws_bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      const size_t h_bytes_tmp = h->ws_bytes;
      delete h;
      return fail(nullptr, OFV_ERR_OUT_OF_MEMORY, "hipMalloc(%zu bytes): %s", h_bytes_tmp, hipGetErrorString(e));
    }
    h->derived_counts = reinterpret_cast<unsigned int*>(h->ws + h->slot_bytes * static_cast<size_t>(max_batch));
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
      h->num_cus = cus;
  }
  *out = h;
  return OFV_OK;
}

ofv_status ofv_set_stream(ofv_handle h, void* stream) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  h->stream = static_cast<hipStream_t>(stream);
  return OFV_OK;
}

ofv_status ofv_workspace_bytes(ofv_handle h, size_t* bytes) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (!bytes) return fail(h, OFV_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = h->ws_bytes;
  return OFV_OK;
}

ofv_status ofv_compute_flow(ofv_handle h, const ofv_image* frame0, const ofv_image* frame1,
                            const ofv_params* params, float* flow_out) {
  return compute_common(h, 1, frame0, frame1, params, nullptr, &flow_out);
}

ofv_status ofv_compute_flow_ex(ofv_handle h, const ofv_image* frame0, const ofv_image* frame1,
                               const ofv_params* params, const float* flow_init, float* flow_out) {
  return compute_common(h, 1, frame0, frame1, params, &flow_init, &flow_out);
}

ofv_status ofv_compute_flow_batch(ofv_handle h, int n, const ofv_image* frame0, const ofv_image* frame1,
                                  const ofv_params* params, const float* const* flow_init,
                                  float* const* flow_out) {
  return compute_common(h, n, frame0, frame1, params, flow_init, flow_out);
}

// ------------------------------------------------------------------ no-allocation entry point

// Device scratch of ofv_compute_flow_static: the two pyramid slabs and the
// two flow ping-pong buffers of one pair.  Each device the library runs on
// holds its own copy until the process ends.  In host code `scratch` is
// only a stand-in for the symbol: its device address comes from
// hipGetSymbolAddress, once per device.
static constexpr size_t kStaticScratchBytes = size_t{48} << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxStaticDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxStaticDevices] = {};

// Device address of `scratch` on the current device `dev`.
hipError_t static_scratch(int dev, char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

ofv_status static_fail(ofv_ctx* c, ofv_status s) {
  g_create_error = c->err;
  return s;
}

}  // namespace

ofv_status ofv_compute_flow_static(const ofv_image* frame0, const ofv_image* frame1, const ofv_params* params,
                                   float* flow_out, void* stream) {
  g_create_error.clear();
  ofv_ctx c;  // host-side plan of the call: it owns no device memory
  ofv_status r = check_params(&c, params);
  if (r != OFV_OK) return static_fail(&c, r);
  if (params->flags & OFV_FLAG_SAVE_ITERATES)
    return static_fail(&c, fail(&c, OFV_ERR_UNSUPPORTED, "saved iterates live in a handle's backward workspace"));
  r = check_image(&c, frame0, "frame0");
  if (r != OFV_OK) return static_fail(&c, r);
  r = check_image(&c, frame1, "frame1");
  if (r != OFV_OK) return static_fail(&c, r);
  set_geometry(&c, frame0->width, frame0->height, 1);
  if (c.slot_bytes > kStaticScratchBytes)
    return static_fail(&c, fail(&c, OFV_ERR_CAPACITY,
                                "%dx%d needs %zu bytes of scratch; the static scratch holds %zu (about 1.5 Mi pixels)",
                                frame0->width, frame0->height, c.slot_bytes, kStaticScratchBytes));
  r = validate_pair(&c, frame0, frame1, nullptr, flow_out, 0);
  if (r != OFV_OK) return static_fail(&c, r);
  if (fault_injected("launch")) return static_fail(&c, fail(&c, OFV_ERR_DEVICE, "injected launch failure"));
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return static_fail(&c, device_error(&c, e, "hipGetDevice"));
  if (dev < 0 || dev >= kMaxStaticDevices)
    return static_fail(&c, fail(&c, OFV_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxStaticDevices));
  e = static_scratch(dev, &c.ws);
  if (e != hipSuccess) return static_fail(&c, device_error(&c, e, "hipGetSymbolAddress(scratch)"));
  c.device = dev;
  c.stream = static_cast<hipStream_t>(stream);
  c.ws_bytes = kStaticScratchBytes;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
    c.num_cus = cus;
  PairPlan pp{};
  pp.f[0] = frame0;
  pp.f[1] = frame1;
  pp.init = nullptr;
  pp.out = flow_out;
  pp.slot = c.ws;
  level_dims(frame0->width, frame0->height, params->num_levels, pp.lw, pp.lh);
  r = run_pipeline(&c, 1, &pp, params);
  return r == OFV_OK ? OFV_OK : static_fail(&c, r);
}

// ------------------------------------------------------------------ adjoint


ofv_status ofv_backward_workspace_bytes(ofv_handle h, int max_levels, int max_iterations, int max_pairs,
                                        uint32_t mode, size_t* bytes) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (!bytes) return fail(h, OFV_ERR_INVALID_ARG, "bytes is NULL");
  if (max_levels < 1 || max_levels > OFV_MAX_LEVELS)
    return fail(h, OFV_ERR_INVALID_ARG, "max_levels %d outside 1..%d", max_levels, OFV_MAX_LEVELS);
  if (max_iterations < 1 || max_iterations > 64)
    return fail(h, OFV_ERR_INVALID_ARG, "max_iterations %d outside 1..64", max_iterations);
  if (max_pairs < 1 || max_pairs > h->max_batch)
    return fail(h, OFV_ERR_INVALID_ARG, "max_pairs %d outside 1..%d (the handle's max_batch)", max_pairs,
                h->max_batch);
  if (mode & ~OFV_BACKWARD_STORE_ALL) return fail(h, OFV_ERR_INVALID_ARG, "unknown mode 0x%x", mode);
  *bytes = bw_total_bytes(h, max_levels, max_iterations, max_pairs, (mode & OFV_BACKWARD_STORE_ALL) != 0);
  return OFV_OK;
}

ofv_status ofv_reserve_backward_ex(ofv_handle h, int max_levels, int max_iterations, int max_pairs, uint32_t mode) {
  size_t bytes = 0;
  ofv_status r = ofv_backward_workspace_bytes(h, max_levels, max_iterations, max_pairs, mode, &bytes);
  if (r != OFV_OK) return r;
  if (h->device < 0) return fail(h, OFV_ERR_UNSUPPORTED, "validation-only handle (created with device -1)");
  const bool store_all = (mode & OFV_BACKWARD_STORE_ALL) != 0;
  if (h->bw && max_levels <= h->bw_levels && max_iterations <= h->bw_iters && max_pairs <= h->bw_pairs &&
      (!store_all || h->bw_store_all))
    return OFV_OK;
  // grow to cover the previous reservation too
  if (h->bw) {
    max_levels = std::max(max_levels, h->bw_levels);
    max_iterations = std::max(max_iterations, h->bw_iters);
    max_pairs = std::max(max_pairs, h->bw_pairs);
    const bool sa = store_all || h->bw_store_all;
    bytes = bw_total_bytes(h, max_levels, max_iterations, max_pairs, sa);
    mode = sa ? OFV_BACKWARD_STORE_ALL : 0u;
  }
  DeviceGuard g(h->device);
  if (h->bw) {
    h->saved_fw.valid = false;
    if (sync_stream(h->stream) != hipSuccess || hipFree(h->bw) != hipSuccess)
      return fail(h, OFV_ERR_DEVICE, "releasing the previous backward workspace failed");
    h->bw = nullptr;
    h->bw_bytes = 0;
    h->bw_levels = h->bw_iters = h->bw_pairs = 0;
    h->bw_store_all = false;
  }
  if (fault_injected("alloc")) return fail(h, OFV_ERR_OUT_OF_MEMORY, "injected allocation failure");
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&h->bw), bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    h->bw = nullptr;
    return fail(h, OFV_ERR_OUT_OF_MEMORY, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
  }
  h->bw_bytes = bytes;
  h->bw_levels = max_levels;
  h->bw_iters = max_iterations;
  h->bw_pairs = max_pairs;
  h->bw_store_all = (mode & OFV_BACKWARD_STORE_ALL) != 0;
  return OFV_OK;
}

ofv_status ofv_reserve_backward(ofv_handle h, int max_levels, int max_iterations) {
  return ofv_reserve_backward_ex(h, max_levels, max_iterations, 1, 0u);
}

namespace {

ofv_status backward_common(ofv_ctx* h, int n, const ofv_image* f0, const ofv_image* f1, const ofv_params* params,
                           const float* const* init, const float* const* gflow, float* const* gf0,
                           float* const* gf1, float* const* ginit) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (n < 1) return fail(h, OFV_ERR_INVALID_ARG, "batch size %d < 1", n);
  if (!f0 || !f1 || !gflow) return fail(h, OFV_ERR_INVALID_ARG, "frame or grad_flow array is NULL");
  ofv_status r = check_params(h, params);
  if (r != OFV_OK) return r;
  if (params->flags & (OFV_FLAG_FORWARD_ADDITIVE | OFV_FLAG_INCREMENT_UPDATE))
    return fail(h, OFV_ERR_UNSUPPORTED, "the adjoint covers the symmetric estimator's consistent update only");
  if (params->storage != OFV_STORE_F32) return fail(h, OFV_ERR_UNSUPPORTED, "the adjoint needs F32 storage");
  if (n > h->max_batch) return fail(h, OFV_ERR_CAPACITY, "batch %d exceeds max_batch %d", n, h->max_batch);
  // every input range, then every output range: outputs may overlap nothing
  std::vector<std::pair<uintptr_t, uintptr_t>> rng;
  for (int j = 0; j < n; ++j) {
    r = check_image(h, &f0[j], "frame0");
    if (r != OFV_OK) return r;
    r = check_image(h, &f1[j], "frame1");
    if (r != OFV_OK) return r;
    if (f0[j].width != f1[j].width || f0[j].height != f1[j].height)
      return fail(h, OFV_ERR_INVALID_ARG, "pair %d: frame sizes differ", j);
    if (f0[j].width > h->max_w || f0[j].height > h->max_h)
      return fail(h, OFV_ERR_CAPACITY, "pair %d: %dx%d exceeds the handle's %dx%d", j, f0[j].width, f0[j].height,
                  h->max_w, h->max_h);
    if (!gflow[j]) return fail(h, OFV_ERR_INVALID_ARG, "pair %d: grad_flow is NULL", j);
    if (ginit && ginit[j] && !(init && init[j]))
      return fail(h, OFV_ERR_INVALID_ARG, "pair %d: grad_flow_init needs flow_init", j);
    const uintptr_t n1 = static_cast<uintptr_t>(f0[j].width) * f0[j].height * sizeof(float);
    uintptr_t a0, a1;
    image_range(&f0[j], a0, a1);
    rng.emplace_back(a0, a1);
    image_range(&f1[j], a0, a1);
    rng.emplace_back(a0, a1);
    const uintptr_t gf = reinterpret_cast<uintptr_t>(gflow[j]);
    rng.emplace_back(gf, gf + 2 * n1);
    if (init && init[j]) {
      const uintptr_t fi = reinterpret_cast<uintptr_t>(init[j]);
      rng.emplace_back(fi, fi + 2 * n1);
    }
  }
  const size_t nin = rng.size();
  for (int j = 0; j < n; ++j) {
    const uintptr_t n1 = static_cast<uintptr_t>(f0[j].width) * f0[j].height * sizeof(float);
    const float* outs[3] = {gf0 ? gf0[j] : nullptr, gf1 ? gf1[j] : nullptr, ginit ? ginit[j] : nullptr};
    const uintptr_t len[3] = {n1, n1, 2 * n1};
    for (int i = 0; i < 3; ++i) {
      if (!outs[i]) continue;
      const uintptr_t o0 = reinterpret_cast<uintptr_t>(outs[i]);
      for (size_t k = 0; k < rng.size(); ++k)
        if (overlap(o0, o0 + len[i], rng[k].first, rng[k].second))
          return fail(h, OFV_ERR_INVALID_ARG, "pair %d: gradient output %d overlaps %s", j, i,
                      k < nin ? "an input" : "another gradient output");
      rng.emplace_back(o0, o0 + len[i]);
    }
  }
  const int L = params->num_levels, IT = params->iterations;
  const bool store_all = (params->flags & OFV_FLAG_STORE_ALL) != 0;
  r = check_saving(h, n, params);
  if (r != OFV_OK) return r;
  if (fault_injected("launch")) return fail(h, OFV_ERR_DEVICE, "injected launch failure");
  if (h->device < 0) return fail(h, OFV_ERR_UNSUPPORTED, "validation-only handle (created with device -1)");
  DeviceGuard g(h->device);
  hipStream_t s = h->stream;
  const BwView bv(h);
  const int kr = params->kernel_radius;
  const int sp0 = static_cast<int>(h->lpitch[0]);
  const int plane0 = static_cast<int>(h->lpitch[0] * h->lh[0]);

  BwPlan bp(h, n, params);
  for (int j = 0; j < n; ++j) {
    PairPlan& q = bp.pp[j];
    q.f[0] = &f0[j];
    q.f[1] = &f1[j];
    q.init = init ? init[j] : nullptr;
    q.out = nullptr;
    q.slot = h->ws + static_cast<size_t>(j) * h->slot_bytes;
    level_dims(f0[j].width, f0[j].height, L, q.lw, q.lh);
  }
  std::vector<PairPlan>& pp = bp.pp;
  auto lp = [&](int l) { return bp.lp(l); };
  auto lplane = [&](int l) { return bp.lplane(l); };
  using Field = BwPlan::Field;
  auto vin0 = [&](int j, int l) { return bp.vin0(j, l); };

  // ---- forward, keeping each iteration's output (store-all: and its record),
  // unless the handle holds the saved forward of exactly these inputs
  if (!((params->flags & OFV_FLAG_SAVED_FORWARD) && saved_forward_matches(h, n, f0, f1, init, params))) {
    r = bp.forward();
    if (r != OFV_OK) return r;
    record_saved_forward(h, n, f0, f1, init, params);
  }

  // ---- backward
  hipError_t e = launch_fill(bv.gpyr_all(), static_cast<int64_t>(bv.lay.gpyr) * n, 0.0f, s);
  if (e != hipSuccess) return device_error(h, e, "fill");
  // gradient fields in rotation: scratch planes 7 + 2i (u) and 8 + 2i (v); -1 = the caller's grad_flow
  auto gbuf = [&](int j, int i) { return bv.scratch(j, 7 + 2 * i); };
  int gcur = -1;
  for (int l = 0; l < L; ++l) {
    int64_t lpx = 0;
    for (int j = 0; j < n; ++j) lpx += static_cast<int64_t>(pp[j].lw[l]) * pp[j].lh[l];
    const int ty = adj_tile_h(lpx);
    for (int k = IT - 1; k >= 0; --k) {
      if (k == 0 && !store_all) {
        r = bp.prepare_vin0(l);
        if (r != OFV_OK) return r;
      }
      const int gnext = (gcur + 1 + 3) % 3;
      AdjArgs aa{};
      aa.reg_rel = params->reg_rel;
      aa.reg_abs = params->reg_abs;
      aa.no_fp64 = 0;
      auto fill = [&](int j, AdjJob& J) {
        J = AdjJob{};
        J.p0 = reinterpret_cast<const float*>(img_plane(h, pp[j], 0, l, 4));
        J.p1 = reinterpret_cast<const float*>(img_plane(h, pp[j], 1, l, 4));
        J.ip = lp(l);
        if (k == 0) {
          const Field f = vin0(j, l);
          J.vu = f.u;
          J.vv = f.u + f.vstep;
          J.vp = f.pitch;
        } else {
          J.vu = bv.saved(j, l, k - 1);
          J.vv = J.vu + lplane(l);
          J.vp = lp(l);
        }
        if (gcur < 0) {
          J.gu = gflow[j];
          J.gv = gflow[j] + static_cast<int64_t>(f0[j].width) * f0[j].height;
          J.gp = f0[j].width;
        } else {
          J.gu = gbuf(j, gcur);
          J.gv = J.gu + plane0;
          J.gp = sp0;
        }
        J.gA = bv.scratch(j, 0);
        J.sp = sp0;
        J.ps = plane0;
        if (store_all) {
          J.st = bv.rec(j, l, k);
          J.stp = lp(l);
          J.sts = lplane(l);
        }
        J.ou = gbuf(j, gnext);
        J.ov = J.ou + plane0;
        J.op = sp0;
        J.gP0 = bv.gpyr(j, 0, l);
        J.gP1 = bv.gpyr(j, 1, l);
        J.w = pp[j].lw[l];
        J.h = pp[j].lh[l];
      };
      int blocks = 0;
      r = run_jobs(h, n, aa, [&](int j, AdjJob& J) {
        if ((j % kMaxJobs) == 0) blocks = 0;
        fill(j, J);
        J.tile_start = blocks;
        blocks += store_all ? adj_point_blocks(J.w, J.h) : adj_sums_blocks(J.w, J.h, ty);
      }, [&](const AdjArgs& a) {
        return store_all ? launch_adj_solve_stored(a, blocks, s) : launch_adj_sums(a, kr, ADJ_SOLVE, ty, blocks, s);
      }, "solve adjoint");
      if (r != OFV_OK) return r;
      r = run_jobs(h, n, aa, [&](int j, AdjJob& J) {
        if ((j % kMaxJobs) == 0) blocks = 0;
        fill(j, J);
        J.tile_start = blocks;
        blocks += adj_scatter_blocks(J.w, J.h, ty);
      }, [&](const AdjArgs& a) { return launch_adj_scatter(a, kr, store_all, ty, blocks, s); }, "warp adjoint");
      if (r != OFV_OK) return r;
      gcur = gnext;
    }
    if (l < L - 1) {
      // gradient w.r.t. the coarser level's last output: transpose of the up-sampling
      const int gacc = (gcur + 1) % 3;
      AuxArgs ua{};
      int mw = 0, mh = 0;
      for (int j = 0; j < n; ++j) mw = std::max(mw, pp[j].lw[l + 1]), mh = std::max(mh, pp[j].lh[l + 1]);
      r = run_jobs(h, n, ua, [&](int j, AuxJob& J) {
        J.in0 = gbuf(j, gcur);
        J.in1 = J.in0 + plane0;
        J.ip = sp0;
        J.w = pp[j].lw[l];
        J.h = pp[j].lh[l];
        J.out0 = gbuf(j, gacc);
        J.out1 = J.out0 + plane0;
        J.op = sp0;
        J.cw = pp[j].lw[l + 1];
        J.ch = pp[j].lh[l + 1];
      }, [&](const AuxArgs& a) { return launch_upsample_adj(a, mw, mh, s); }, "up-sampling adjoint");
      if (r != OFV_OK) return r;
      gcur = gacc;
    }
  }
  // gbuf(j, gcur): gradient w.r.t. the coarsest level's input field = the restricted initial field
  std::vector<int> wi;
  for (int j = 0; j < n; ++j)
    if (ginit && ginit[j]) wi.push_back(j);
  if (!wi.empty()) {
    if (L == 1) {
      for (int j : wi)
        for (int c = 0; c < 2; ++c) {
          e = hipMemcpy2DAsync(ginit[j] + static_cast<int64_t>(c) * f0[j].width * f0[j].height,
                               f0[j].width * sizeof(float), gbuf(j, gcur) + c * plane0, sp0 * sizeof(float),
                               f0[j].width * sizeof(float), f0[j].height, hipMemcpyDeviceToDevice, s);
          if (e != hipSuccess) return device_error(h, e, "copy");
        }
    } else {
      int cur = gcur;
      for (int l = L - 1; l >= 1; --l) {
        const bool last = (l == 1);
        const int tgt = (cur + 1) % 3;
        AuxArgs ra{};
        ra.scale = 0.5f;
        ra.accumulate = 0;
        int mw = 0, mh = 0;
        for (int j : wi) mw = std::max(mw, pp[j].lw[l - 1]), mh = std::max(mh, pp[j].lh[l - 1]);
        const int nw = static_cast<int>(wi.size());
        r = run_jobs(h, 2 * nw, ra, [&](int i, AuxJob& J) {
          const int j = wi[i / 2], c = i % 2;
          J.in0 = gbuf(j, cur) + c * plane0;
          J.ip = sp0;
          J.cw = pp[j].lw[l];
          J.ch = pp[j].lh[l];
          J.w = pp[j].lw[l - 1];
          J.h = pp[j].lh[l - 1];
          if (last) {
            J.out0 = ginit[j] + static_cast<int64_t>(c) * f0[j].width * f0[j].height;
            J.op = f0[j].width;
          } else {
            J.out0 = gbuf(j, tgt) + c * plane0;
            J.op = sp0;
          }
        }, [&](const AuxArgs& a) { return launch_reduce_adj(a, mw, mh, s); }, "restriction adjoint");
        if (r != OFV_OK) return r;
        cur = tgt;
      }
    }
  }
  // image-gradient pyramids: REDUCE transposed, coarse to fine, both frames of every pair
  for (int l = L - 1; l >= 1; --l) {
    AuxArgs ra{};
    ra.scale = 1.0f;
    ra.accumulate = 1;
    int mw = 0, mh = 0;
    for (int j = 0; j < n; ++j) mw = std::max(mw, pp[j].lw[l - 1]), mh = std::max(mh, pp[j].lh[l - 1]);
    r = run_jobs(h, 2 * n, ra, [&](int i, AuxJob& J) {
      const int j = i / 2, f = i % 2;
      J.in0 = bv.gpyr(j, f, l);
      J.ip = lp(l);
      J.cw = pp[j].lw[l];
      J.ch = pp[j].lh[l];
      J.out0 = bv.gpyr(j, f, l - 1);
      J.op = lp(l - 1);
      J.w = pp[j].lw[l - 1];
      J.h = pp[j].lh[l - 1];
    }, [&](const AuxArgs& a) { return launch_reduce_adj(a, mw, mh, s); }, "pyramid adjoint");
    if (r != OFV_OK) return r;
  }
  // normalisation (and intensity scaling) transposed, every requested frame gradient
  std::vector<std::pair<int, int>> nf;
  for (int j = 0; j < n; ++j) {
    if (gf0 && gf0[j]) nf.emplace_back(j, 0);
    if (gf1 && gf1[j]) nf.emplace_back(j, 1);
  }
  if (!nf.empty()) {
    NormAdjArgs na{};
    na.nr = params->norm_radius;
    na.eps = params->norm_eps;
    int mw = 0, mh = 0;
    for (const auto& q : nf) mw = std::max(mw, f0[q.first].width), mh = std::max(mh, f0[q.first].height);
    r = run_jobs(h, static_cast<int>(nf.size()), na, [&](int i, NormAdjJob& J) {
      const int j = nf[i].first, f = nf[i].second;
      const ofv_image* fr = f == 0 ? &f0[j] : &f1[j];
      J.f = ImageIn{fr->data, fr->pitch, fr->width, fr->height, fr->type, fr->bit_depth};
      J.gN = bv.gpyr(j, f, 0);
      J.gp = lp(0);
      J.gF = f == 0 ? gf0[j] : gf1[j];
      J.fp = fr->width;
    }, [&](const NormAdjArgs& a) { return launch_norm_adj(a, mw, mh, s); }, "normalisation adjoint");
    if (r != OFV_OK) return r;
  }
  return OFV_OK;
}

}  // namespace

ofv_status ofv_compute_flow_backward(ofv_handle h, const ofv_image* frame0, const ofv_image* frame1,
                                     const ofv_params* params, const float* flow_init, const float* grad_flow,
                                     float* grad_frame0, float* grad_frame1, float* grad_flow_init) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (!frame0 || !frame1) return fail(h, OFV_ERR_INVALID_ARG, "frame0 or frame1 is NULL");
  if (!grad_flow) return fail(h, OFV_ERR_INVALID_ARG, "grad_flow is NULL");
  if (grad_flow_init && !flow_init) return fail(h, OFV_ERR_INVALID_ARG, "grad_flow_init needs flow_init");
  return backward_common(h, 1, frame0, frame1, params, &flow_init, &grad_flow, &grad_frame0, &grad_frame1,
                         &grad_flow_init);
}

ofv_status ofv_compute_flow_backward_batch(ofv_handle h, int n, const ofv_image* frames0, const ofv_image* frames1,
                                           const ofv_params* params, const float* const* flow_init,
                                           const float* const* grad_flow, float* const* grad_frame0,
                                           float* const* grad_frame1, float* const* grad_flow_init) {
  return backward_common(h, n, frames0, frames1, params, flow_init, grad_flow, grad_frame0, grad_frame1,
                         grad_flow_init);
}

ofv_status ofv_destroy(ofv_handle h) {
  if (!h) return OFV_OK;
  ofv_status r = OFV_OK;
  // a validation-only handle has no stream to drain, but an injected sync failure is reported all the same
  if (h->device < 0 && fault_injected("sync")) r = OFV_ERR_DEVICE;
  if (h->device >= 0) {
    DeviceGuard g(h->device);
    if (sync_stream(h->stream) != hipSuccess) r = OFV_ERR_DEVICE;
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    if (h->bw && hipFree(h->bw) != hipSuccess) r = OFV_ERR_DEVICE;
    if (h->ws && hipFree(h->ws) != hipSuccess) r = OFV_ERR_DEVICE;
  }
  delete h;
  return r;
}

// ------------------------------------------------------------------ time-resolved streaming

ofv_status ofv_stream_reset(ofv_handle h) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  h->stream_valid = false;
  return OFV_OK;
}

ofv_status ofv_stream_push(ofv_handle h, const ofv_image* frame, const ofv_params* params, const float* flow_init,
                           float* flow_out, int* produced) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (!frame || !produced) return fail(h, OFV_ERR_INVALID_ARG, "frame or produced is NULL");
  *produced = 0;
  ofv_status r = check_params(h, params);
  if (r != OFV_OK) return r;
  if (params->flags & OFV_FLAG_SAVE_ITERATES)
    return fail(h, OFV_ERR_UNSUPPORTED, "the streaming call does not save iterates");
  r = validate_pair(h, frame, frame, flow_init, flow_out, 0);
  if (r != OFV_OK) return r;
  const ofv_params& p = *params;
  const bool have = h->stream_valid;
  if (have) {
    const ofv_params& q = h->stream_params;
    if (frame->width != h->stream_w || frame->height != h->stream_h)
      return fail(h, OFV_ERR_INVALID_ARG, "frame is %dx%d, the retained frame %dx%d (ofv_stream_reset first)",
                  frame->width, frame->height, h->stream_w, h->stream_h);
    if (p.num_levels != q.num_levels || p.norm_radius != q.norm_radius || p.norm_eps != q.norm_eps ||
        p.storage != q.storage)
      return fail(h, OFV_ERR_INVALID_ARG,
                  "num_levels, norm_radius, norm_eps and storage must match the retained frame (ofv_stream_reset first)");
  }
  if (fault_injected("launch")) return fail(h, OFV_ERR_DEVICE, "injected launch failure");
  if (h->device < 0) return fail(h, OFV_ERR_UNSUPPORTED, "validation-only handle (created with device -1)");
  DeviceGuard g(h->device);
  PairPlan pp;
  pp.f[0] = nullptr;  // the retained frame: its pyramid is in slab stream_slab
  pp.f[1] = frame;
  pp.init = flow_init;
  pp.out = flow_out;
  pp.slot = h->ws;
  level_dims(frame->width, frame->height, p.num_levels, pp.lw, pp.lh);
  const int new_slab = have ? 1 - h->stream_slab : 0;
  pp.slab[0] = h->stream_slab;
  pp.slab[1] = new_slab;
  pp.built[0] = true;
  r = run_pipeline(h, 1, &pp, params, nullptr, have ? PIPE_FULL : PIPE_PYRAMID);
  if (r != OFV_OK) return r;
  h->stream_valid = true;
  h->stream_slab = new_slab;
  h->stream_w = frame->width;
  h->stream_h = frame->height;
  h->stream_params = p;
  *produced = have ? 1 : 0;
  return OFV_OK;
}

// ------------------------------------------------------------------ live derived quantities

void ofv_default_derived_params(ofv_derived_params* p) {
  if (!p) return;
  p->dx = 1.0f;
  p->dz = 1.0f;
  p->dt = 1.0f;
  p->streamwise_sign = 1;
}

ofv_status ofv_derived(ofv_handle h, const float* flow, int width, int height, int64_t pitch, const uint8_t* mask,
                       int64_t mask_pitch, const ofv_derived_params* params, float* vorticity, int64_t vort_pitch,
                       const float* probe_xy, int n_probes, float* probe_uv, double* area) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (!flow) return fail(h, OFV_ERR_INVALID_ARG, "flow is NULL");
  if (!params) return fail(h, OFV_ERR_INVALID_ARG, "params is NULL");
  if (width < 1 || height < 1) return fail(h, OFV_ERR_INVALID_ARG, "size %dx%d invalid", width, height);
  if (pitch < width) return fail(h, OFV_ERR_INVALID_ARG, "pitch < width");
  if (mask && mask_pitch < width) return fail(h, OFV_ERR_INVALID_ARG, "mask_pitch < width");
  if (vorticity && vort_pitch < width) return fail(h, OFV_ERR_INVALID_ARG, "vort_pitch < width");
  const ofv_derived_params& p = *params;
  for (float q : {p.dx, p.dz, p.dt})
    if (!std::isfinite(q) || !(q > 0.0f)) return fail(h, OFV_ERR_INVALID_ARG, "dx, dz and dt must be finite and > 0");
  if (p.streamwise_sign != 1 && p.streamwise_sign != -1)
    return fail(h, OFV_ERR_INVALID_ARG, "streamwise_sign %d is not +1 or -1", p.streamwise_sign);
  if (n_probes < 0 || n_probes > (1 << 20)) return fail(h, OFV_ERR_INVALID_ARG, "n_probes %d outside 0..2^20", n_probes);
  if (n_probes > 0 && (!probe_xy || !probe_uv)) return fail(h, OFV_ERR_INVALID_ARG, "probe arrays are NULL");
  if (2 * pitch * static_cast<int64_t>(height) * 4 >= 2 * kMaxPlaneBytes ||
      (vorticity && vort_pitch * static_cast<int64_t>(height) * 4 >= kMaxPlaneBytes))
    return fail(h, OFV_ERR_UNSUPPORTED, "planes of 2 GiB or more");
  const uintptr_t f0 = reinterpret_cast<uintptr_t>(flow);
  const uintptr_t f1 = f0 + static_cast<uintptr_t>(2 * pitch * static_cast<int64_t>(height) * 4);
  if (vorticity) {
    const uintptr_t o0 = reinterpret_cast<uintptr_t>(vorticity);
    if (overlap(o0, o0 + static_cast<uintptr_t>(vort_pitch * static_cast<int64_t>(height) * 4), f0, f1))
      return fail(h, OFV_ERR_INVALID_ARG, "vorticity overlaps the flow");
  }
  if (n_probes > 0) {
    const uintptr_t o0 = reinterpret_cast<uintptr_t>(probe_uv);
    if (overlap(o0, o0 + static_cast<uintptr_t>(n_probes) * 8, f0, f1))
      return fail(h, OFV_ERR_INVALID_ARG, "probe_uv overlaps the flow");
  }
  if (area) {
    const uintptr_t o0 = reinterpret_cast<uintptr_t>(area);
    if (overlap(o0, o0 + sizeof(double), f0, f1)) return fail(h, OFV_ERR_INVALID_ARG, "area overlaps the flow");
  }
  if (!vorticity && !area && n_probes == 0) return OFV_OK;  // nothing requested
  if (fault_injected("launch")) return fail(h, OFV_ERR_DEVICE, "injected launch failure");
  if (h->device < 0) return fail(h, OFV_ERR_UNSUPPORTED, "validation-only handle (created with device -1)");
  DeviceGuard g(h->device);
  DerivedArgs a{};
  a.u = flow;
  a.v = flow + pitch * static_cast<int64_t>(height);
  a.pitch = pitch;
  a.w = width;
  a.h = height;
  a.mask = mask;
  a.mask_pitch = mask_pitch;
  a.cx = static_cast<float>((static_cast<double>(p.dz) / p.dx) / p.dt);
  a.cy = static_cast<float>((static_cast<double>(p.dx) / p.dz) / p.dt);
  a.sign = p.streamwise_sign;
  a.ntiles = ((width + kDerivedTW - 1) / kDerivedTW) * ((height + kDerivedTH - 1) / kDerivedTH);
  a.omega = vorticity;
  a.omega_pitch = vort_pitch;
  a.probe_xy = probe_xy;
  a.probe_uv = probe_uv;
  a.n_probes = n_probes;
  a.su = static_cast<float>(static_cast<double>(p.dx) / p.dt);
  a.sv = static_cast<float>(static_cast<double>(p.dz) / p.dt);
  a.partial = area ? h->derived_counts : nullptr;
  a.area = area;
  a.dx = p.dx;
  a.dz = p.dz;
  const int nblocks = std::max(1, std::min(kDerivedMaxBlocks, std::max(a.ntiles, (n_probes + 255) / 256)));
  const hipError_t e = launch_derived(a, nblocks, h->stream);
  return e == hipSuccess ? OFV_OK : device_error(h, e, "derived");
}

// ------------------------------------------------------------------ work-decomposition tuning

ofv_status ofv_set_gn_variant(ofv_handle h, int variant, int tile_h) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (variant < -1 || variant >= kGnVariants) return fail(h, OFV_ERR_INVALID_ARG, "unknown variant %d", variant);
  if (tile_h != 0 && (tile_h < 4 || tile_h > 1024)) return fail(h, OFV_ERR_INVALID_ARG, "tile_h %d outside 4..1024", tile_h);
  h->forced_variant = variant;
  h->forced_tile_h = tile_h;
  return OFV_OK;
}

namespace {

// Times every candidate decomposition on the n pairs (one batch call per
// run, so the launch groups and their keys are the batch's) and records the
// fastest per key in the handle.
ofv_status autotune_impl(ofv_handle h, int n, const ofv_image* frame0, const ofv_image* frame1,
                         const ofv_params* params, float* const* flow_out, int repeats) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (repeats < 1 || repeats > 1000) return fail(h, OFV_ERR_INVALID_ARG, "repeats %d outside 1..1000", repeats);
  if (params && (params->flags & (OFV_FLAG_FORWARD_ADDITIVE | OFV_FLAG_INCREMENT_UPDATE)))
    return fail(h, OFV_ERR_UNSUPPORTED, "the autotuner times the symmetric estimator's decompositions");
  if (params && (params->flags & OFV_FLAG_SAVE_ITERATES))
    return fail(h, OFV_ERR_UNSUPPORTED, "the autotuner times forward calls that save no iterates");
  // validate exactly like a compute call (the validation-only handle stops there)
  ofv_status r = compute_common(h, n, frame0, frame1, params, nullptr, flow_out);
  if (r != OFV_OK) return r;
  DeviceGuard g(h->device);
  struct Cand {
    int variant, tile_h;
  };
  // tile variants ignore tile_h (their tile height is fixed); it is recorded as their height.  The band
  // takes the occupancy-derived height (0) and three fixed ones: taller tiles than one round of resident
  // workgroups gives halve the vertical halo at the cost of idle slots
  const Cand cands[] = {{GN_TILE_16x16, 16},  {GN_TILE_16x16W, 16}, {GN_TILE_32x16, 16}, {GN_TILE_32x16W, 16},
                        {GN_TILE_64x16, 16},  {GN_TILE_64x32, 32},  {GN_TILE_64x16W, 16}, {GN_TILE_64x32W, 32},
                        {GN_TILE_32x32W, 32}, {GN_TILE_64x64, 64},  {GN_MARCH, 16},       {GN_MARCH, 32},
                        {GN_MARCH, 64},       {GN_BAND4, 0},       {GN_BAND4, 64},      {GN_BAND4, 128},
                        {GN_BAND4, 256}};
  constexpr int nc = static_cast<int>(sizeof(cands) / sizeof(cands[0]));
  // launch times per (level key, candidate); the candidates take turns within every
  // repeat, so that slow drifts of the clock affect them alike
  std::map<ofv_ctx::TuneKey, std::vector<std::vector<float>>> samples;
  const int saved_v = h->forced_variant, saved_t = h->forced_tile_h;
  for (int k = -1; k < repeats && r == OFV_OK; ++k) {  // k = -1: warm-up of every candidate
    for (int ci = 0; ci < nc && r == OFV_OK; ++ci) {
      h->forced_variant = cands[ci].variant;
      h->forced_tile_h = cands[ci].tile_h;
      h->capture = k >= 0;
      h->events_used = 0;
      h->recs.clear();
      r = compute_common(h, n, frame0, frame1, params, nullptr, flow_out);
      h->capture = false;
      if (r != OFV_OK) break;
      if (k < 0) continue;
      if (sync_stream(h->stream) != hipSuccess) {
        r = fail(h, OFV_ERR_DEVICE, "synchronisation failed while tuning");
        break;
      }
      for (const auto& rec : h->recs) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, rec.a, rec.b) != hipSuccess) ms = 1e30f;
        auto& v = samples[rec.key];
        if (v.empty()) v.resize(nc);
        v[ci].push_back(ms);
      }
    }
  }
  // per level key: the candidate with the lowest median launch time
  std::map<ofv_ctx::TuneKey, std::pair<float, ofv_ctx::Choice>> best;
  for (auto& kv : samples) {
    for (int ci = 0; ci < nc; ++ci) {
      std::vector<float>& v = kv.second[ci];
      if (v.empty()) continue;
      std::sort(v.begin(), v.end());
      const float med = v[v.size() / 2];
      auto it = best.find(kv.first);
      if (it == best.end() || med < it->second.first)
        best[kv.first] = {med, ofv_ctx::Choice{cands[ci].variant, cands[ci].tile_h}};
    }
  }
  h->forced_variant = saved_v;
  h->forced_tile_h = saved_t;
  h->recs.clear();
  if (r != OFV_OK) return r;
  for (const auto& kv : best) h->tuned[kv.first] = kv.second.second;
  return OFV_OK;
}

}  // namespace

ofv_status ofv_autotune(ofv_handle h, const ofv_image* frame0, const ofv_image* frame1, const ofv_params* params,
                        float* flow_out, int repeats) {
  return autotune_impl(h, 1, frame0, frame1, params, &flow_out, repeats);
}

ofv_status ofv_autotune_batch(ofv_handle h, int n, const ofv_image* frame0, const ofv_image* frame1,
                              const ofv_params* params, float* const* flow_out, int repeats) {
  return autotune_impl(h, n, frame0, frame1, params, flow_out, repeats);
}

ofv_status ofv_tuning_export(ofv_handle h, char* buf, size_t cap, size_t* needed) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  std::ostringstream os;
  for (const auto& kv : h->tuned)
    os << kv.first.kr << ' ' << kv.first.storage << ' ' << kv.first.mode << ' ' << kv.first.w << ' '
       << kv.first.hgt << ' ' << kv.first.n << ' ' << kv.second.variant << ' ' << kv.second.tile_h << '\n';
  const std::string txt = os.str();
  if (needed) *needed = txt.size() + 1;
  if (!buf) return OFV_OK;
  if (cap < txt.size() + 1) return fail(h, OFV_ERR_CAPACITY, "buffer of %zu bytes, %zu needed", cap, txt.size() + 1);
  std::memcpy(buf, txt.c_str(), txt.size() + 1);
  return OFV_OK;
}

ofv_status ofv_tuning_import(ofv_handle h, const char* text) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (!text) return fail(h, OFV_ERR_INVALID_ARG, "text is NULL");
  std::istringstream is(text);
  std::map<ofv_ctx::TuneKey, ofv_ctx::Choice> add;
  std::string row;
  int line = 0;
  while (std::getline(is, row)) {
    ++line;
    if (row.find_first_not_of(" \t\r") == std::string::npos) continue;   // blank line
    std::istringstream ls(row);
    ofv_ctx::TuneKey k{};
    ofv_ctx::Choice c{};
    std::string rest;
    // eight integers and nothing after them
    if (!(ls >> k.kr >> k.storage >> k.mode >> k.w >> k.hgt >> k.n >> c.variant >> c.tile_h) || (ls >> rest))
      return fail(h, OFV_ERR_INVALID_ARG, "tuning line %d is malformed", line);
    // band entries record tile height 0 (sized at every launch from the occupancy) or 4..1024
    if (c.variant < GN_MARCH || c.variant >= kGnVariants ||
        ((c.tile_h < 4 || c.tile_h > 1024) && !(c.variant == GN_BAND4 && c.tile_h == 0)))
      return fail(h, OFV_ERR_INVALID_ARG, "tuning line %d is invalid", line);
    add[k] = c;
  }
  for (const auto& kv : add) h->tuned[kv.first] = kv.second;
  return OFV_OK;
}

// ------------------------------------------------------------------ stage entry points

static ofv_status stage_prologue(ofv_ctx* h) {
  if (check_handle(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  return OFV_OK;
}

static ofv_status stage_device(ofv_ctx* h) {
  if (fault_injected("launch")) return fail(h, OFV_ERR_DEVICE, "injected launch failure");
  if (h->device < 0) return fail(h, OFV_ERR_UNSUPPORTED, "validation-only handle (created with device -1)");
  return OFV_OK;
}

ofv_status ofv_stage_normalize(ofv_handle h, const ofv_image* frame, int norm_radius, float norm_eps, int storage,
                               void* out, int64_t out_pitch) {
  if (stage_prologue(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  ofv_status r = check_image(h, frame, "frame");
  if (r != OFV_OK) return r;
  if (norm_radius < 0 || norm_radius > OFV_MAX_NORM_RADIUS)
    return fail(h, OFV_ERR_INVALID_ARG, "norm_radius %d outside 0..%d", norm_radius, OFV_MAX_NORM_RADIUS);
  if (!std::isfinite(norm_eps) || norm_eps < 0.0f) return fail(h, OFV_ERR_INVALID_ARG, "norm_eps invalid");
  if (storage < 0 || storage > 2) return fail(h, OFV_ERR_INVALID_ARG, "unknown storage %d", storage);
  if (!out) return fail(h, OFV_ERR_INVALID_ARG, "out is NULL");
  if (out_pitch < frame->width) return fail(h, OFV_ERR_INVALID_ARG, "out_pitch < width");
  if ((r = stage_device(h)) != OFV_OK) return r;
  DeviceGuard g(h->device);
  NormArgs na{};
  na.njobs = 1;
  na.nr = norm_radius;
  na.eps = norm_eps;
  na.storage = storage;
  NormJob& J = na.job[0];
  J.in = frame->data;
  J.in_pitch = frame->pitch;
  J.type = frame->type;
  J.bits = frame->bit_depth;
  J.w = frame->width;
  J.h = frame->height;
  J.out = out;
  J.out_pitch = out_pitch;
  J.tile_start = 0;
  hipError_t e = launch_normalize(na, ((J.w + kNormTW - 1) / kNormTW) * ((J.h + kNormTH - 1) / kNormTH), h->stream);
  return e == hipSuccess ? OFV_OK : device_error(h, e, "normalize");
}

static ofv_status reduce_common(ofv_ctx* h, int storage, const void* in, int w, int hgt, int64_t in_pitch, void* out,
                                int64_t out_pitch, float scale, int planes, int64_t in_plane, int64_t out_plane) {
  if (!in || !out) return fail(h, OFV_ERR_INVALID_ARG, "in or out is NULL");
  if (w < 1 || hgt < 1) return fail(h, OFV_ERR_INVALID_ARG, "size %dx%d invalid", w, hgt);
  if (in_pitch < w || out_pitch < (w + 1) / 2) return fail(h, OFV_ERR_INVALID_ARG, "pitch too small");
  ofv_status r = stage_device(h);
  if (r != OFV_OK) return r;
  DeviceGuard g(h->device);
  const size_t es = storage_bytes(storage);
  ReduceArgs ra{};
  ra.njobs = planes;
  ra.storage = storage;
  ra.scale = scale;
  int blocks = 0;
  for (int c = 0; c < planes; ++c) {
    ReduceJob& J = ra.job[c];
    J.in = static_cast<const char*>(in) + c * in_plane * es;
    J.out = static_cast<char*>(out) + c * out_plane * es;
    J.in_pitch = in_pitch;
    J.out_pitch = out_pitch;
    J.w = w;
    J.h = hgt;
    J.tile_start = blocks;
    blocks += static_cast<int>(reduce_blocks((w + 1) / 2, (hgt + 1) / 2));
  }
  hipError_t e = launch_reduce(ra, blocks, h->stream);
  return e == hipSuccess ? OFV_OK : device_error(h, e, "reduce");
}

ofv_status ofv_stage_reduce(ofv_handle h, int storage, const void* in, int width, int height, int64_t in_pitch,
                            void* out, int64_t out_pitch) {
  if (stage_prologue(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (storage < 0 || storage > 2) return fail(h, OFV_ERR_INVALID_ARG, "unknown storage %d", storage);
  return reduce_common(h, storage, in, width, height, in_pitch, out, out_pitch, 1.0f, 1, 0, 0);
}

ofv_status ofv_stage_pyramid(ofv_handle h, int storage, const void* in, int width, int height, int64_t in_pitch,
                             int levels, void* const* out, const int64_t* out_pitch) {
  if (stage_prologue(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (storage < 0 || storage > 2) return fail(h, OFV_ERR_INVALID_ARG, "unknown storage %d", storage);
  if (levels < 1 || levels > kMaxReduceLevels)
    return fail(h, OFV_ERR_INVALID_ARG, "levels %d outside 1..%d", levels, kMaxReduceLevels);
  if (!in || !out || !out_pitch) return fail(h, OFV_ERR_INVALID_ARG, "in, out or out_pitch is NULL");
  if (width < 1 || height < 1) return fail(h, OFV_ERR_INVALID_ARG, "size %dx%d invalid", width, height);
  if (in_pitch < width) return fail(h, OFV_ERR_INVALID_ARG, "in_pitch < width");
  int w = width, hh = height;
  for (int k = 0; k < levels; ++k) {
    w = (w + 1) / 2;
    hh = (hh + 1) / 2;
    if (!out[k]) return fail(h, OFV_ERR_INVALID_ARG, "out[%d] is NULL", k);
    if (out_pitch[k] < w) return fail(h, OFV_ERR_INVALID_ARG, "out_pitch[%d] < %d", k, w);
  }
  if (levels == 1) return reduce_common(h, storage, in, width, height, in_pitch, out[0], out_pitch[0], 1.0f, 1, 0, 0);
  if (static_cast<int64_t>(width) * height >= kReduceSingleLevelPixels) {
    // as the estimator builds pyramids of this size: one launch per level
    const void* src = in;
    int64_t sp = in_pitch;
    int sw = width, sh = height;
    for (int k = 0; k < levels; ++k) {
      const ofv_status rk = reduce_common(h, storage, src, sw, sh, sp, out[k], out_pitch[k], 1.0f, 1, 0, 0);
      if (rk != OFV_OK) return rk;
      src = out[k];
      sp = out_pitch[k];
      sw = (sw + 1) / 2;
      sh = (sh + 1) / 2;
    }
    return OFV_OK;
  }
  ofv_status r = stage_device(h);
  if (r != OFV_OK) return r;
  DeviceGuard g(h->device);
  ReduceMArgs ra{};
  ra.njobs = 1;
  ra.storage = storage;
  ReduceMJob& J = ra.job[0];
  J.in = in;
  J.in_pitch = in_pitch;
  for (int k = 0; k < levels; ++k) {
    J.out[k] = out[k];
    J.out_pitch[k] = out_pitch[k];
  }
  J.w = width;
  J.h = height;
  J.tile_start = 0;
  const bool small = reduce_multi_small(levels, static_cast<int64_t>(width) * height);
  int tw = 0, th = 0;
  reduce_multi_tile(levels, small, tw, th);
  const hipError_t e =
      launch_reduce_multi(ra, levels, small, ((w + tw - 1) / tw) * ((hh + th - 1) / th), h->stream);
  return e == hipSuccess ? OFV_OK : device_error(h, e, "pyramid");
}

ofv_status ofv_stage_restrict_flow(ofv_handle h, const float* in, int width, int height, int64_t in_pitch,
                                   float* out, int64_t out_pitch) {
  if (stage_prologue(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  return reduce_common(h, ST_F32, in, width, height, in_pitch, out, out_pitch, 0.5f, 2,
                       static_cast<int64_t>(height) * in_pitch, static_cast<int64_t>((height + 1) / 2) * out_pitch);
}

ofv_status ofv_stage_upsample(ofv_handle h, const float* in, int in_width, int in_height, int64_t in_pitch,
                              float* out, int width, int height, int64_t out_pitch) {
  if (stage_prologue(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (!in || !out) return fail(h, OFV_ERR_INVALID_ARG, "in or out is NULL");
  if (in_width < 1 || in_height < 1 || width < 1 || height < 1)
    return fail(h, OFV_ERR_INVALID_ARG, "sizes must be >= 1");
  if (in_pitch < in_width || out_pitch < width) return fail(h, OFV_ERR_INVALID_ARG, "pitch too small");
  ofv_status r = stage_device(h);
  if (r != OFV_OK) return r;
  DeviceGuard g(h->device);
  UpsampleArgs a{};
  a.in_u = in;
  a.in_v = in + static_cast<int64_t>(in_height) * in_pitch;
  a.out_u = out;
  a.out_v = out + static_cast<int64_t>(height) * out_pitch;
  a.in_pitch = in_pitch;
  a.out_pitch = out_pitch;
  a.cw = in_width;
  a.ch = in_height;
  a.w = width;
  a.h = height;
  hipError_t e = launch_upsample(a, h->stream);
  return e == hipSuccess ? OFV_OK : device_error(h, e, "upsample");
}

ofv_status ofv_stage_gn_iteration(ofv_handle h, int storage, const void* p0, const void* p1, int width, int height,
                                  int64_t img_pitch, int mode, const float* flow_in, int in_width, int in_height,
                                  int64_t in_pitch, float* flow_out, int64_t out_pitch, int kernel_radius,
                                  float reg_rel, float reg_abs) {
  if (stage_prologue(h) != OFV_OK) return OFV_ERR_INVALID_ARG;
  if (storage < 0 || storage > 2) return fail(h, OFV_ERR_INVALID_ARG, "unknown storage %d", storage);
  if (!p0 || !p1 || !flow_out) return fail(h, OFV_ERR_INVALID_ARG, "p0, p1 or flow_out is NULL");
  if (width < 1 || height < 1) return fail(h, OFV_ERR_INVALID_ARG, "size %dx%d invalid", width, height);
  if (img_pitch < width || out_pitch < width) return fail(h, OFV_ERR_INVALID_ARG, "pitch too small");
  if (img_pitch >= kMaxPitch || out_pitch >= kMaxPitch || img_pitch * height * 4 >= kMaxPlaneBytes ||
      out_pitch * height * 4 >= kMaxPlaneBytes)
    return fail(h, OFV_ERR_UNSUPPORTED, "image or flow plane of 2 GiB or more");
  if (kernel_radius < 1) return fail(h, OFV_ERR_INVALID_ARG, "kernel_radius < 1");
  if (kernel_radius > OFV_MAX_KERNEL_RADIUS) return fail(h, OFV_ERR_UNSUPPORTED, "kernel_radius too large");
  if (!std::isfinite(reg_rel) || reg_rel < 0 || !std::isfinite(reg_abs) || reg_abs < 0)
    return fail(h, OFV_ERR_INVALID_ARG, "reg_rel/reg_abs invalid");
  if (mode < OFV_FLOW_IN_ZERO || mode > OFV_FLOW_IN_UPSAMPLE) return fail(h, OFV_ERR_INVALID_ARG, "unknown mode");
  int iw = width, ih = height;
  if (mode != OFV_FLOW_IN_ZERO) {
    if (!flow_in) return fail(h, OFV_ERR_INVALID_ARG, "flow_in is NULL");
    if (mode == OFV_FLOW_IN_UPSAMPLE) {
      if (in_width < 1 || in_height < 1) return fail(h, OFV_ERR_INVALID_ARG, "coarse size invalid");
      iw = in_width;
      ih = in_height;
    }
    if (in_pitch < iw) return fail(h, OFV_ERR_INVALID_ARG, "in_pitch too small");
    if (in_pitch >= kMaxPitch || in_pitch * ih * 4 >= kMaxPlaneBytes)
      return fail(h, OFV_ERR_UNSUPPORTED, "flow_in plane of 2 GiB or more, or pitch of 2^24 or more");
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(flow_in);
    const uintptr_t a1 = a0 + (2ull * ih * in_pitch) * sizeof(float);
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(flow_out);
    const uintptr_t b1 = b0 + (2ull * height * out_pitch) * sizeof(float);
    if (overlap(a0, a1, b0, b1)) return fail(h, OFV_ERR_INVALID_ARG, "flow_out overlaps flow_in");
  }
  ofv_status r = stage_device(h);
  if (r != OFV_OK) return r;
  DeviceGuard g(h->device);
  GnArgs ga{};
  ga.njobs = 1;
  ga.reg_rel = reg_rel;
  ga.reg_abs = reg_abs;
  const int tx = gn_tile_w(kernel_radius);
  int variant = 0, tw = 0, th = 0;
  const int64_t strips = (width + tx - 1) / tx, rows = height;
  pick_gn(h, ofv_ctx::TuneKey{kernel_radius, storage, mode, width, height, 1}, strips, rows,
          static_cast<int64_t>(width) * height, width < 2 || height < 2, variant, ga.tile_h, &strips, &rows, 1);
  gn_tile_dims(variant, kernel_radius, ga.tile_h, tw, th);
  GnJob& J = ga.job[0];
  J.p0 = p0;
  J.p1 = p1;
  J.img_pitch = img_pitch;
  J.w = width;
  J.h = height;
  J.cw = iw;
  J.ch = ih;
  J.mode = mode;
  J.in_u = flow_in;
  J.in_v = flow_in ? flow_in + static_cast<int64_t>(ih) * in_pitch : nullptr;
  J.in_pitch = in_pitch;
  J.out_u = flow_out;
  J.out_v = flow_out + static_cast<int64_t>(height) * out_pitch;
  J.out_pitch = out_pitch;
  J.tile_start = 0;
  const int blocks = ((width + tw - 1) / tw) * ((height + th - 1) / th);
  hipError_t e = launch_gn(ga, kernel_radius, storage, mode, variant, blocks, h->stream);
  return e == hipSuccess ? OFV_OK : device_error(h, e, "gauss-newton iteration");
}

}  // extern "C"
