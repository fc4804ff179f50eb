// Operands and launchers of the adjoint's kernels (reverse mode of the
// estimator), kept apart from the forward kernels' declarations.
#pragma once

#include "ofv_internal.h"

namespace ofv {

// ---------------------------------------------------------------- adjoint (reverse mode)
// One pair of a batched launch of the adjoint's iteration kernels, at one
// level and iteration.  Planes are float32, row-major with the pitches given
// (elements); gA holds seven planes `ps` apart (the gradients w.r.t. the
// five window sums, then the solve's direct gradient w.r.t. V(m)); st holds
// the stored record of the iteration (five window sums, then Gx, Gy, b),
// eight planes `sts` apart with pitch `stp`.
struct AdjJob {
  const float* p0; const float* p1;   // level images (pitch ip)
  const float* vu; const float* vv;   // input field of the iteration (pitch vp)
  const float* gu; const float* gv;   // gradient w.r.t. its output (pitch gp)
  float* gA;                          // 7 scratch planes (pitch sp, ps apart)
  float* st;                          // stored record (pitch stp, sts apart)
  float* ou; float* ov;               // recording forward: the output field; backward: dL/d(input field) (pitch op)
  float* gP0; float* gP1;             // image gradients of the level, accumulated (pitch ip)
  int ip, vp, gp, sp, ps, op, stp, sts;
  int w, h;
  int tile_start;
};

struct AdjArgs {
  int njobs;
  float reg_rel, reg_abs;
  int no_fp64;   // recording forward: no float64 fallback in the solve
  AdjJob job[kMaxJobs];
};
static_assert(sizeof(AdjArgs) <= 4096, "kernel arguments");

// What the window-sum kernel does after forming the sums of an output pixel.
enum AdjEpilogue : int {
  ADJ_SOLVE = 0,   // adjoint of the damped solve: gA and the direct gradient
  ADJ_RECORD = 1,  // forward iteration that also stores its sums and Gx, Gy, b
};

// Per-pair operands of the batched point-wise adjoint kernels (blockIdx.z = pair).
struct AuxJob {
  const float* in0; const float* in1;
  float* out0; float* out1;
  int ip, op;
  int w, h;     // size of the grid's plane (fine for up-sampling, fine for REDUCE^T)
  int cw, ch;   // size of the coarse plane
};

struct AuxArgs {
  int njobs;
  float scale;
  int accumulate;
  int pad_;
  AuxJob job[kMaxJobs];
};

struct NormAdjJob {
  ImageIn f;
  const float* gN; int gp;      // gradient w.r.t. the normalised plane
  float* gF; int fp;            // gradient w.r.t. the frame (written)
};

struct NormAdjArgs {
  int njobs;
  int nr;
  float eps;
  int pad_;
  NormAdjJob job[kMaxJobs];
};

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s);
// Tile height of the adjoint's iteration kernels for a launch over `pixels`
// pixels: 64 x 16 tiles, or 64 x 8 for launches too small to fill the chip.
inline int adj_tile_h(int64_t pixels) { return pixels < (int64_t{2} << 20) ? 8 : 16; }
// Window sums of one iteration over every job's level (tiles of 64 x ty outputs).
hipError_t launch_adj_sums(const AdjArgs& a, int kr, int epilogue, int ty, int nblocks, hipStream_t s);
int adj_sums_blocks(int w, int h, int ty);
// Adjoint of the solve from stored sums (point-wise, blocks of 64 x 4 pixels).
hipError_t launch_adj_solve_stored(const AdjArgs& a, int nblocks, hipStream_t s);
int adj_point_blocks(int w, int h);
// Window sums of gA, adjoints of the products, b, the central difference and
// the two warps; image gradients scattered, dL/d(input field) written.
hipError_t launch_adj_scatter(const AdjArgs& a, int kr, bool stored, int ty, int nblocks, hipStream_t s);
int adj_scatter_blocks(int w, int h, int ty);
// V = 2 bilinear(V_coarse, x / 2, y / 2) of every job (in0/in1 coarse u/v, out0/out1 fine).
hipError_t launch_upsample_batch(const AuxArgs& a, int maxw, int maxh, hipStream_t s);
// Transpose of the up-sampling, as a gather: out = coarse gradient (written).
hipError_t launch_upsample_adj(const AuxArgs& a, int maxcw, int maxch, hipStream_t s);
// out0 and out1 of every job zeroed over w x h (pitch op).
hipError_t launch_zero_fields(const AuxArgs& a, int maxw, int maxh, hipStream_t s);
// Transpose of REDUCE (times scale), as a gather; in0 coarse, out0 fine; accumulate adds to out0.
hipError_t launch_reduce_adj(const AuxArgs& a, int maxw, int maxh, hipStream_t s);
hipError_t launch_norm_adj(const NormAdjArgs& a, int maxw, int maxh, hipStream_t s);

}  // namespace ofv
