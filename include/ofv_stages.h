/*
 * ofv_stages.h - stage-level entry points of the OFV estimator.
 *
 * Each call runs exactly one step of the pipeline of section "Live-Optical
 * Flow Velocimetry" (arXiv 2509.25924) with the same kernels that
 * ofv_compute_flow() uses, on caller-provided device buffers, so that every
 * step can be checked on its own.  Conventions of ofv.h apply: status
 * return, caller-owned device memory, enqueue on the handle's stream, no
 * synchronisation, argument errors detected before any enqueue.
 *
 * A "plane" is a row-major 2-D array with a pitch in elements (>= width).
 * Image planes are stored in the given ofv_storage type (float32, IEEE
 * binary16 or bfloat16).  Flow planes are float32 and come in pairs: the v
 * plane starts `height * pitch` elements after the u plane.
 */
#ifndef OFV_STAGES_H
#define OFV_STAGES_H

#include "ofv.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Pipeline step 1, local intensity normalisation.  Scales an integer frame
 * by 1 / (2^bit_depth - 1) (float frames as given) and, if norm_radius > 0,
 * replaces each pixel by its z-score over the (2 NR + 1)^2 window truncated
 * to the image: (I - mean) / sqrt(var + norm_eps), variance by a second
 * pass about the window mean.  Output: a plane of frame->width x
 * frame->height in `storage`, pitch out_pitch. */
ofv_status ofv_stage_normalize(ofv_handle h, const ofv_image* frame, int norm_radius, float norm_eps,
                               int storage, void* out, int64_t out_pitch);

/* Pipeline step 2, one level of the Burt-Adelson Gaussian pyramid (REDUCE):
 * out(x, y) = sum_{i,j=-2..2} w_i w_j in(clamp(2x+i), clamp(2y+j)) with
 * w = [1, 4, 6, 4, 1] / 16.  Output size ceil(width/2) x ceil(height/2). */
ofv_status ofv_stage_reduce(ofv_handle h, int storage, const void* in, int width, int height,
                            int64_t in_pitch, void* out, int64_t out_pitch);

/* Pipeline step 2 as the estimator runs it: `levels` (1..3) successive
 * REDUCE levels of `in` in one launch (one launch per level from 16 Mi
 * input pixels on).  out[k] receives level k + 1
 * (ceil(width / 2^(k+1)) x ceil(height / 2^(k+1)), pitch out_pitch[k]);
 * each level is rounded to `storage` before the next is formed, so the
 * result equals `levels` chained ofv_stage_reduce calls bit for bit.  The
 * output planes must not overlap the input or each other.  `out` and
 * `out_pitch` are host arrays of `levels` entries.  OFV_ERR_INVALID_ARG for
 * levels outside 1..3, a NULL pointer, a size below 1 or a pitch below its
 * plane's width. */
ofv_status ofv_stage_pyramid(ofv_handle h, int storage, const void* in, int width, int height, int64_t in_pitch,
                             int levels, void* const* out, const int64_t* out_pitch);

/* Initial-flow restriction: out = REDUCE(in) / 2 for both flow planes
 * (float32 pairs).  Output size ceil(width/2) x ceil(height/2). */
ofv_status ofv_stage_restrict_flow(ofv_handle h, const float* in, int width, int height, int64_t in_pitch,
                                   float* out, int64_t out_pitch);

/* Pipeline step 4, up-sampling and projection to the finer level:
 * out(X, Y) = 2 * bilinear(in, X/2, Y/2), coordinates clamped to the coarse
 * image, for both flow planes.  Coarse in_width x in_height, fine width x height. */
ofv_status ofv_stage_upsample(ofv_handle h, const float* in, int in_width, int in_height, int64_t in_pitch,
                              float* out, int width, int height, int64_t out_pitch);

/* How ofv_stage_gn_iteration reads its input flow. */
typedef enum {
  OFV_FLOW_IN_ZERO = 0,     /* V = 0; flow_in is ignored (may be NULL) */
  OFV_FLOW_IN_DIRECT = 1,   /* V = flow_in, same size as the images */
  OFV_FLOW_IN_UPSAMPLE = 2  /* V = 2 * bilinear(flow_in, X/2, Y/2): flow_in is the next coarser level */
} ofv_flow_in_mode;

/* Pipeline step 3 (one Gauss-Newton iteration at one level), fused:
 * midpoint warps W0 = P0(k - V/2), W1 = P1(k + V/2) (bilinear, clamped);
 * S = (W0 + W1)/2, T = W1 - W0; G = central difference of S (clamped);
 * b = G . V(k) - T; window sums over (2 KR + 1)^2 truncated to the image of
 * Gx^2, GxGy, Gy^2, Gx b, Gy b; damped 2x2 solve
 *   (A + lam I) V'(m) = c + lam V(m),  lam = reg_rel (Sxx + Syy) + reg_abs.
 * p0, p1: image planes (storage, pitch img_pitch) of width x height.
 * flow_in: per `mode`; for UPSAMPLE its size is in_width x in_height.
 * flow_out: float32 plane pair of width x height, pitch out_pitch; it must
 * not overlap flow_in. */
ofv_status ofv_stage_gn_iteration(ofv_handle h, int storage, const void* p0, const void* p1, int width,
                                  int height, int64_t img_pitch, int mode, const float* flow_in,
                                  int in_width, int in_height, int64_t in_pitch, float* flow_out,
                                  int64_t out_pitch, int kernel_radius, float reg_rel, float reg_abs);

#ifdef __cplusplus
}
#endif

#endif /* OFV_STAGES_H */
