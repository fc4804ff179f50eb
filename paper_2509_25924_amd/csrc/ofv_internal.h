// Internal interface between the C ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ofv {

enum Storage { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };
enum FlowIn { FLOW_ZERO = 0, FLOW_DIRECT = 1, FLOW_UPSAMPLE = 2 };

// Pairs (or planes) handled by one launch; larger batches are split.
constexpr int kMaxJobs = 16;
constexpr int kGnThreads = 256;
constexpr int kMaxKR = 12;
constexpr int kMaxNR = 16;

// ---------------------------------------------------------------- normalisation
struct NormJob {
  const void* in;      // frame pixel (0,0)
  void* out;           // output plane (storage type)
  int64_t in_pitch;    // elements
  int64_t out_pitch;   // elements
  int w, h;
  int type;            // 0 u8, 1 u16, 2 f32
  int bits;            // significant bits of integer frames
  int tile_start;      // first block of this job
  int pad_;
};
// normalisation tile: kNormTW x kNormTH outputs per 256-lane workgroup, kNormPX per lane
constexpr int kNormTW = 64, kNormPX = 4, kNormTH = 4 * kNormPX;
struct NormArgs {
  int njobs;
  int nr;
  float eps;
  int storage;
  NormJob job[kMaxJobs];
};

// ---------------------------------------------------------------- REDUCE
struct ReduceJob {
  const void* in;
  void* out;
  int64_t in_pitch, out_pitch;
  int w, h;            // input size
  int tile_start;
  int pad_;
};
// Output tile of the single-level REDUCE kernel: kRedTW x kRedTH outputs per 256-lane workgroup.
constexpr int kRedTW = 64, kRedTH = 8;
inline int64_t reduce_blocks(int64_t wn, int64_t hn) { return ((wn + kRedTW - 1) / kRedTW) * ((hn + kRedTH - 1) / kRedTH); }
struct ReduceArgs {
  int njobs;
  int storage;         // element type of in/out (flows use ST_F32)
  float scale;         // 1 for images, 0.5 for the initial-flow restriction
  int pad_;
  ReduceJob job[kMaxJobs];
};

// Several pyramid levels from one input level in one launch (image pyramids).
constexpr int kMaxReduceLevels = 3;
struct ReduceMJob {
  const void* in;
  void* out[kMaxReduceLevels];     // levels 1..nlev below the input
  int64_t in_pitch;
  int64_t out_pitch[kMaxReduceLevels];
  int w, h;                        // input size
  int tile_start;
  int pad_;
};
struct ReduceMArgs {
  int njobs;
  int storage;
  int pad_[2];
  ReduceMJob job[kMaxJobs];
};
// Output tile of the deepest level and lanes per workgroup for nlev
// levels.  Three levels: launches over at least kReduceMSmallPixels input
// pixels take 8 x 8 tiles with 512 lanes (51 KB of LDS at FP32, several
// workgroups per compute unit, so that the loads of one overlap the passes
// of another), smaller launches 16 x 8 tiles with 1024 lanes (the smallest
// halo; 90 KB, one workgroup per compute unit).
constexpr int64_t kReduceMSmallPixels = int64_t{4} << 20;
// Launches over at least this many input pixels build one level per launch
// instead (the single-level kernel, wider spread over the compute units).
constexpr int64_t kReduceSingleLevelPixels = int64_t{16} << 20;
inline bool reduce_multi_small(int nlev, int64_t pixels) { return nlev == 3 && pixels >= kReduceMSmallPixels; }
constexpr int reduce_multi_tw(int nlev, bool small) { return nlev == 3 ? (small ? 8 : 16) : 32; }
constexpr int reduce_multi_th(int, bool) { return 8; }
constexpr int reduce_multi_nt(int nlev, bool small) { return nlev == 3 ? (small ? 512 : 1024) : 256; }
inline void reduce_multi_tile(int nlev, bool small, int& tw, int& th) {
  tw = reduce_multi_tw(nlev, small);
  th = reduce_multi_th(nlev, small);
}

// ---------------------------------------------------------------- live derived quantities
struct DerivedArgs {
  const float* u;
  const float* v;
  int64_t pitch;
  int w, h;
  const uint8_t* mask;              // NULL: every pixel valid
  int64_t mask_pitch;
  float cx, cy;                     // (dz / dx) / dt and (dx / dz) / dt
  int sign;                         // streamwise sign, +1 or -1
  int ntiles;                       // 64 x 16 tiles covering the field
  float* omega;                     // NULL: no vorticity
  int64_t omega_pitch;
  const float* probe_xy;
  float* probe_uv;
  int n_probes;
  float su, sv;                     // dx / dt and dz / dt
  unsigned int* partial;            // per-workgroup pixel counts (handle workspace); NULL: no area
  double* area;
  double dx, dz;
};
constexpr int kDerivedTW = 64, kDerivedRows = 8;  // a lane: one column, kDerivedRows consecutive rows
constexpr int kDerivedTH = 4 * kDerivedRows;       // 4 wavefronts per 256-lane workgroup stacked vertically
constexpr int kDerivedMaxBlocks = 2048;   // grid bound of the derived-quantities kernel (slots of partial counts)

// ---------------------------------------------------------------- up-sampling (stage entry point)
struct UpsampleArgs {
  const float* in_u; const float* in_v;
  float* out_u; float* out_v;
  int64_t in_pitch, out_pitch;
  int cw, ch, w, h;
};

// ---------------------------------------------------------------- Gauss-Newton iteration
struct GnJob {
  const void* p0; const void* p1;     // image planes of this level
  const float* in_u; const float* in_v;
  float* out_u; float* out_v;
  int64_t img_pitch, in_pitch, out_pitch;
  int w, h;            // level size
  int cw, ch;          // coarse size (FLOW_UPSAMPLE)
  int mode;            // FlowIn (equal for all jobs of a launch)
  int tile_start;
};
// GnArgs::est: estimator variants, read at run time by the generic kernels
// (forward-additive warps, increment-form update), and the switch of the
// solve's float64 fallback, read by every kernel.
enum GnEst : uint32_t { EST_FORWARD_ADDITIVE = 1u, EST_INCREMENT = 2u, EST_NO_FP64 = 4u };
struct GnArgs {
  int njobs;
  int tile_h;          // output rows per workgroup
  float reg_rel, reg_abs;
  uint32_t est;        // GnEst bits
  int pad_;
  GnJob job[kMaxJobs];
};

// Work decompositions of the fused Gauss-Newton kernel.
enum GnVariant {
  GN_MARCH = 0,
  GN_TILE_64x32 = 1,
  GN_TILE_64x16 = 2,
  GN_TILE_32x16 = 3,
  GN_TILE_16x16 = 4,
  GN_TILE_64x32W = 5,
  GN_TILE_64x16W = 6,
  GN_TILE_64x64 = 7,
  GN_TILE_16x16W = 8,
  GN_TILE_32x16W = 9,
  GN_TILE_32x32W = 10,
  GN_BAND4 = 11
};
constexpr int kGnVariants = 12;

// Columns of output produced by one 256-lane strip for window radius kr.
inline int gn_tile_w(int kr) { return kGnThreads - 2 * kr - 2; }

// Output tile of a variant: width and height (march: strip width, tile_h rows).
// 64 x 64 tiles need (64 + 2 KR + 3)^2 x 24 B of LDS: above KR 7 they would
// exceed the 160 KiB of a compute unit, and 64 x 32 tiles with 1024 lanes run
// instead.  Host block counts and device launches both go through this.
inline int gn_variant_for(int variant, int kr) {
  return variant == GN_TILE_64x64 && kr > 7 ? GN_TILE_64x32W : variant;
}

inline void gn_tile_dims(int variant, int kr, int tile_h, int& tw, int& th) {
  variant = gn_variant_for(variant, kr);
  if (variant == GN_TILE_64x32) { tw = 64; th = 32; }
  else if (variant == GN_TILE_64x16 || variant == GN_TILE_64x16W) { tw = 64; th = 16; }
  else if (variant == GN_TILE_64x32W) { tw = 64; th = 32; }
  else if (variant == GN_TILE_64x64) { tw = 64; th = 64; }
  else if (variant == GN_TILE_32x16 || variant == GN_TILE_32x16W) { tw = 32; th = 16; }
  else if (variant == GN_TILE_32x32W) { tw = 32; th = 32; }
  else if (variant == GN_TILE_16x16 || variant == GN_TILE_16x16W) { tw = 16; th = 16; }
  else { tw = gn_tile_w(kr); th = tile_h; }   // the march and the band: 256-column strips
}

// Band decomposition: workgroups of the band kernel for window radius kr,
// storage and input-flow mode that fit on one compute unit at once (0 if
// the runtime cannot tell).
int gn_band_per_cu(int kr, int storage, int mode);
// Output rows per band tile for the jobs of one launch, job j covering
// strips[j] strips of rows[j] rows.  A tile of th rows marches th + 2 kr + 2
// product rows one after another, and the launch runs ceil(tiles / slots)
// rounds of resident workgroups, tiles = sum over jobs of strips[j] x
// ceil(rows[j] / th): th is the one of rows_max / k (k = 1, 2, ...) that
// minimises rounds x (th + 2 kr + 2), no smaller than keeps the vertical
// halo below about a third of the rows computed (4 kr + 8), unless the
// tallest level is lower than that.  One round when every strip fits in the
// slots (the smallest tiles that still fit); when there are more strips than
// slots, enough tiles per strip that the last round is not mostly idle.
inline int gn_band_tile_h(const int64_t* strips, const int64_t* rows, int njobs, int64_t slots, int kr) {
  if (slots < 1) slots = 1;
  int64_t rows_max = 1;
  for (int j = 0; j < njobs; ++j) rows_max = rows[j] > rows_max ? rows[j] : rows_max;
  const int64_t lo = 4 * kr + 8 < rows_max ? 4 * kr + 8 : rows_max;
  const int64_t halo = 2 * kr + 2;
  int64_t best = rows_max, best_cost = -1;
  for (int64_t k = 1; k <= rows_max; ++k) {
    const int64_t th = (rows_max + k - 1) / k;
    if (th < lo) break;
    int64_t tiles = 0;
    for (int j = 0; j < njobs; ++j) tiles += (strips[j] > 1 ? strips[j] : 1) * ((rows[j] + th - 1) / th);
    const int64_t cost = (tiles + slots - 1) / slots * (th + halo);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = th;
    }
  }
  return static_cast<int>(best < 4 ? 4 : best);
}

hipError_t launch_normalize(const NormArgs& a, int nblocks, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& a, int nblocks, hipStream_t s);
hipError_t launch_reduce_multi(const ReduceMArgs& a, int nlev, bool small, int nblocks, hipStream_t s);
hipError_t launch_upsample(const UpsampleArgs& a, hipStream_t s);
hipError_t launch_derived(const DerivedArgs& a, int nblocks, hipStream_t s);
// All jobs of one launch share the input-flow mode (a compile-time parameter of the kernel).
// generic: the kernels that read the estimator variant from a.est (16 x 16 tiles or the march)
// instead of the symmetric estimator's consistent update compiled in.
hipError_t launch_gn(const GnArgs& a, int kr, int storage, int mode, int variant, int nblocks, hipStream_t s,
                     bool generic = false);

// ---------------------------------------------------------------- adjoint (float32 storage)
struct ImageIn {
  const void* data;
  int64_t pitch;
  int w, h, type, bits;
};

}  // namespace ofv
