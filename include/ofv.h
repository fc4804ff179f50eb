/*
 * ofv.h - C ABI of the dense optical-flow velocimetry (OFV) estimator on
 * AMD Instinct MI355X (gfx950).
 *
 * The estimator is the one defined in section "Live-Optical Flow
 * Velocimetry" of Pimienta & Aider, "High Resolution and High-Speed Live
 * Optical Flow Velocimetry" (arXiv 2509.25924): for every pixel m it finds the
 * displacement V that minimises the symmetric sum of squared differences
 *     sum_{k in N(m)} [ I0(k - V/2) - I1(k + V/2) ]^2          (Eq. of_symmetric)
 * over a square window N(m) of radius KR, with Gauss-Newton iterations at
 * every level of a Gaussian pyramid, coarse to fine, after a local
 * intensity normalisation (the six-step pipeline of that section).  The
 * output is one vector per pixel, in pixels per frame pair.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - Every function returns an ofv_status; none throws, aborts or exits.
 * - Pointers named "device" are device memory owned by the caller; the
 *   library never frees or retains them beyond the call.  All work is
 *   enqueued on the handle's stream and the call returns without
 *   synchronising: results are valid once that stream has completed.
 *   Device faults surface as OFV_ERR_DEVICE from a later call, or at the
 *   caller's own synchronisation.
 * - Argument errors are detected on the host before anything is enqueued;
 *   nothing is written on error.  ofv_last_error() then holds a message.
 * - The compute entry points never allocate and never synchronise: the
 *   handle's workspace is sized once by ofv_create().
 * - Flow fields are planar float32 [2][H][W] (u plane then v plane, rows of
 *   W elements, no padding).  u is the displacement along +x (columns), v
 *   along +y (rows); V maps frame0 to frame1 and is defined at the
 *   midpoint of the two frames (Eq. of_symmetric).
 * - A handle must not be used from two threads at once.
 * - Fault injection for tests: the environment variable OFV_FAULT_INJECT,
 *   read at every call, may name "alloc" (device allocations fail:
 *   OFV_ERR_OUT_OF_MEMORY), "launch" (compute and stage calls fail with
 *   OFV_ERR_DEVICE after validation, before anything is enqueued, so
 *   nothing is written) and "sync" (every synchronisation of the library,
 *   in ofv_destroy, ofv_autotune and a reservation-replacing
 *   ofv_reserve_backward(_ex), reports OFV_ERR_DEVICE; ofv_destroy still
 *   releases everything), alone or together (e.g. "alloc,sync").
 */
#ifndef OFV_H
#define OFV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ofv_ctx* ofv_handle;

typedef enum {
  OFV_OK = 0,
  OFV_ERR_INVALID_ARG = -1,   /* null pointer, bad size, bad parameter value, aliasing */
  OFV_ERR_UNSUPPORTED = -2,   /* valid request this build does not implement (e.g. KR > OFV_MAX_KERNEL_RADIUS) */
  OFV_ERR_CAPACITY = -3,      /* image or batch larger than the handle's workspace */
  OFV_ERR_OUT_OF_MEMORY = -4, /* device allocation failed in ofv_create */
  OFV_ERR_DEVICE = -5         /* HIP runtime error (launch failure, device fault) */
} ofv_status;

typedef enum { OFV_PIX_U8 = 0, OFV_PIX_U16 = 1, OFV_PIX_F32 = 2 } ofv_pixel_type;

/* Storage of the normalised images and their pyramid levels.  Arithmetic is
 * always float32; F16/BF16 halve the bytes streamed per pixel. */
typedef enum { OFV_STORE_F32 = 0, OFV_STORE_F16 = 1, OFV_STORE_BF16 = 2 } ofv_storage;

#define OFV_MAX_LEVELS 16
#define OFV_MAX_KERNEL_RADIUS 12
#define OFV_MAX_NORM_RADIUS 16

/* One camera frame in device memory. */
typedef struct {
  const void* data;   /* device pointer to pixel (0, 0) */
  int32_t width;      /* >= 1 */
  int32_t height;     /* >= 1 */
  int64_t pitch;      /* elements per row, >= width, < 2^24; a crop is an offset pointer with the parent's
                         pitch; pitch * height * element size < 2 GiB (else OFV_ERR_UNSUPPORTED) */
  int32_t type;       /* ofv_pixel_type */
  int32_t bit_depth;  /* integer frames: significant bits, 1..8 for U8, 1..16 for U16 (right-aligned);
                         intensity = value / (2^bit_depth - 1).  Ignored for F32 (used as given). */
} ofv_image;

/* Estimator parameters (section "Live-Optical Flow Velocimetry"; ranges of
 * Table tab:OFPIV). */
typedef struct {
  int32_t num_levels;    /* pyramid levels in total = PSL + 1, 1..OFV_MAX_LEVELS (1 = no pyramid) */
  int32_t kernel_radius; /* KR, 1..OFV_MAX_KERNEL_RADIUS: window (2 KR + 1)^2, truncated at the image border */
  int32_t iterations;    /* IT >= 1 Gauss-Newton iterations at every level */
  int32_t norm_radius;   /* NR, 0..OFV_MAX_NORM_RADIUS: local z-score window (2 NR + 1)^2; 0 = off */
  float norm_eps;        /* > 0 typical 1e-4: added to the local variance (intensity units in [0,1], squared) */
  float reg_rel;         /* >= 0, typical 1e-3: damping lambda = reg_rel * trace(A) + reg_abs */
  float reg_abs;         /* >= 0, typical 1e-9; reg_rel = reg_abs = 0 gives NaN on textureless windows */
  int32_t storage;       /* ofv_storage */
  uint32_t flags;        /* 0 or an OR of OFV_FLAG_FORWARD_ADDITIVE, OFV_FLAG_INCREMENT_UPDATE,
                            OFV_FLAG_NO_FP64_FALLBACK, OFV_FLAG_STORE_ALL, OFV_FLAG_SAVE_ITERATES,
                            OFV_FLAG_SAVED_FORWARD */
} ofv_params;

/* params.flags: the forward-additive Lucas-Kanade estimator that the paper
 * contrasts its symmetric objective with (section "Live-Optical Flow
 * Velocimetry", after Eq. of_symmetric): minimise
 * sum_k [I0(k) - I1(k + V)]^2 instead, linearised the same way about V(k)
 * with the gradient of the warped second image; the field is then anchored
 * at the pixels of frame 0.  Runs on 16 x 16 tiles, or on the strip march
 * where the decomposition chosen is the march or the band (the band has no
 * build for it) and on levels one pixel thin, and has no adjoint
 * (ofv_compute_flow_backward returns OFV_ERR_UNSUPPORTED). */
#define OFV_FLAG_FORWARD_ADDITIVE 1u

/* params.flags: the increment form of the Gauss-Newton update, the
 * alternative to the consistent form of our reading of Eq. of_symmetric: the
 * residual of every pixel k of the window N(m) is linearised about the
 * window's own V(m) rather than about the V(k) its warps used, which gives
 *   (A + lam I) dV = sum_{k in N(m)} G(k) (-T(k)),   V'(m) = V(m) + dV
 * (A, lam and the warps as without the flag).  Both forms agree where the
 * field is uniform over the window and at V = 0.  Combined with
 * OFV_FLAG_FORWARD_ADDITIVE it is the textbook forward-additive
 * Lucas-Kanade step on every window.  Runs on the same kernels as
 * OFV_FLAG_FORWARD_ADDITIVE and has no adjoint. */
#define OFV_FLAG_INCREMENT_UPDATE 2u

/* params.flags: switch off the float64 fallback of the 2x2 solve (by
 * default, windows whose damped normal matrix has q = 4 det / trace^2 below
 * 1e-2 have the determinant and the solution recomputed in float64 from the
 * float32 sums).  For A/B comparisons of the fallback's effect. */
#define OFV_FLAG_NO_FP64_FALLBACK 4u

/* params.flags, read by the backward calls only (the forward ignores it):
 * store instead of recompute.  The backward's forward pass then keeps, per
 * level and iteration, the five window sums and Gx, Gy, b of every pixel (40
 * bytes per pixel with the output field, against 8 when recomputing), and
 * the adjoint reads them back instead of re-warping and re-summing.  Needs a
 * reservation made with OFV_BACKWARD_STORE_ALL. */
#define OFV_FLAG_STORE_ALL 8u

/* params.flags of the forward calls (ofv_compute_flow, _ex, _batch): also
 * keep every iteration's output field in the handle's backward workspace
 * (the last one of level 0 is flow_out itself), as the backward's own
 * forward pass does, so that a backward call with OFV_FLAG_SAVED_FORWARD on
 * the same inputs can skip that pass (the usual forward-then-backward of
 * training).  Costs what a plain forward costs.  With OFV_FLAG_STORE_ALL
 * the store-all record is kept too.  Needs a reservation covering the
 * levels, iterations, pairs and mode, F32 storage and the symmetric
 * estimator's consistent update (OFV_ERR_CAPACITY / OFV_ERR_UNSUPPORTED
 * otherwise); ofv_compute_flow_static, ofv_stream_push and the autotuner
 * reject it. */
#define OFV_FLAG_SAVE_ITERATES 16u

/* params.flags of the backward calls: skip the forward pass where the handle
 * holds the iterates of a forward with OFV_FLAG_SAVE_ITERATES (or of a
 * backward call) on the same inputs: the same frame and initial-field
 * pointers, sizes, pitches and types, and the same parameters (these two
 * flags aside).  Any other forward call on the handle, and a new
 * reservation, discard them; the backward then runs the forward itself.  The
 * frames and initial fields must not have been modified since. */
#define OFV_FLAG_SAVED_FORWARD 32u

/* Fill *p with the defaults: 3 levels, KR 4, IT 3, NR 1, eps 1e-4,
 * reg_rel 1e-3, reg_abs 1e-9, F32 storage.  p == NULL is ignored. */
void ofv_default_params(ofv_params* p);

/* Create a handle on HIP device `device` whose workspace holds up to
 * `max_batch` pairs of up to max_width x max_height pixels.  `stream` is a
 * hipStream_t (NULL = the default stream) on which all work is enqueued.
 * Allocates the workspace (pyramids and flow ping-pong buffers, about
 * 8/3 * 4 + 16 bytes per pixel per pair).  A float plane of the maximum
 * size must stay below 2 GiB and its row pitch (max_width rounded up to 64)
 * below 2^24 elements, else OFV_ERR_UNSUPPORTED.  On error *out is set to
 * NULL. */
ofv_status ofv_create(ofv_handle* out, int device, int max_width, int max_height, int max_batch,
                      void* stream);

/* Change the stream later calls enqueue on (a hipStream_t, NULL = default). */
ofv_status ofv_set_stream(ofv_handle h, void* stream);

/* Bytes of device workspace the handle owns (writes *bytes). */
ofv_status ofv_workspace_bytes(ofv_handle h, size_t* bytes);

/* Dense flow of one pair, starting from zero flow at the coarsest level.
 * frame0 and frame1 must have equal width and height; flow_out is a device
 * float32 [2][H][W] buffer that must not overlap either frame. */
ofv_status ofv_compute_flow(ofv_handle h, const ofv_image* frame0, const ofv_image* frame1,
                            const ofv_params* params, float* flow_out);

/* As ofv_compute_flow, with an optional initial field flow_init (device
 * float32 [2][H][W], NULL = zero).  The initial field is restricted to the
 * coarsest level by REDUCE / 2 per level before any output is written, so
 * flow_init may alias flow_out (time-resolved warm start). */
ofv_status ofv_compute_flow_ex(ofv_handle h, const ofv_image* frame0, const ofv_image* frame1,
                               const ofv_params* params, const float* flow_init, float* flow_out);

/* n pairs, possibly of different sizes, processed together: every stage
 * runs as one launch over all pairs (per pyramid level and iteration).
 * frame0, frame1 and flow_out are arrays of n entries; flow_init is NULL or
 * an array of n pointers (entries may be NULL).  1 <= n <= max_batch.
 * Results equal n separate ofv_compute_flow_ex calls bit for bit when every
 * level runs the same work decomposition in both (see ofv_set_gn_variant;
 * the default choice depends on the pixels of the whole launch); other
 * decompositions differ from them by float32 rounding only. */
ofv_status ofv_compute_flow_batch(ofv_handle h, int n, const ofv_image* frame0, const ofv_image* frame1,
                                  const ofv_params* params, const float* const* flow_init,
                                  float* const* flow_out);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * estimator of ofv_compute_flow without a handle.  Its workspace (both
 * frames' pyramids and the flow ping-pong buffers, 8/3 * 4 * 2 + 16 bytes
 * per pixel with rows padded to 64 elements) lives in a static 48 MiB device
 * array of the library, one per device, held until the process ends; pairs
 * needing more (above about 1.5 Mi pixels, e.g. 1280 x 1024 fits, 1536 x
 * 1024 does not) give OFV_ERR_CAPACITY before anything is enqueued.  Work
 * runs on the current device, enqueued on `stream` (a hipStream_t, NULL =
 * the default stream); the call allocates nothing and does not synchronise.
 * The array is shared by every call on the device and keeps the last
 * call's contents (nothing in it needs to start at zero): calls that
 * overlap on one device, e.g. on two streams, race and give undefined
 * results.  The work decomposition is the default one (tuned tables live in
 * handles).  Arguments, errors and results as ofv_compute_flow;
 * ofv_last_error(NULL) holds the message of a failing call on this thread. */
ofv_status ofv_compute_flow_static(const ofv_image* frame0, const ofv_image* frame1, const ofv_params* params,
                                   float* flow_out, void* stream);

/* ofv_reserve_backward_ex mode: also reserve the store-all record (OFV_FLAG_STORE_ALL). */
#define OFV_BACKWARD_STORE_ALL 1u

/* Device bytes that ofv_reserve_backward_ex(h, max_levels, max_iterations,
 * max_pairs, mode) allocates, for pairs up to the handle's max size: per
 * pair the output field of every iteration of every level (8 bytes per
 * pixel of the level per iteration), with OFV_BACKWARD_STORE_ALL also the
 * record (32 bytes per pixel per iteration, and the first iteration's input
 * field per level), 15 level-0 scratch planes, and two image-gradient
 * pyramids.  No allocation. */
ofv_status ofv_backward_workspace_bytes(ofv_handle h, int max_levels, int max_iterations, int max_pairs,
                                        uint32_t mode, size_t* bytes);

/* Reserve device memory for the backward calls on batches of up to
 * max_pairs pairs (at most the handle's max_batch) with up to max_levels
 * levels and max_iterations iterations per level; mode 0 or
 * OFV_BACKWARD_STORE_ALL.  A set-up call: it allocates, and to replace a
 * smaller reservation it synchronises the handle's stream and frees it (the
 * new one covers both).  Reserving no more than is held does nothing. */
ofv_status ofv_reserve_backward_ex(ofv_handle h, int max_levels, int max_iterations, int max_pairs, uint32_t mode);

/* ofv_reserve_backward_ex(h, max_levels, max_iterations, 1, 0). */
ofv_status ofv_reserve_backward(ofv_handle h, int max_levels, int max_iterations);

/* Reverse-mode derivative of the whole estimator (normalisation, pyramid,
 * every Gauss-Newton iteration, up-sampling, initial-field restriction):
 * given grad_flow = dL/dflow_out (device float32 [2][H][W]) it writes
 *   grad_frame0, grad_frame1: dL/dframe, device float32 [H][W] (row pitch W),
 *     in the frames' own units (integer frames: per digital number);
 *   grad_flow_init: dL/dflow_init, device float32 [2][H][W] (needs flow_init).
 * Each output may be NULL.  The forward is re-run first (unless
 * OFV_FLAG_SAVED_FORWARD finds it saved), keeping only each iteration's
 * output field; the adjoint of each iteration recomputes the
 * warps, gradients, products and window sums of its tiles in on-chip memory
 * (or, with OFV_FLAG_STORE_ALL, reads the stored record).  The image
 * gradients are accumulated with float atomics, so results are
 * reproducible only up to summation order.  Needs the symmetric
 * estimator's consistent update and F32 storage (OFV_ERR_UNSUPPORTED
 * otherwise) and a reservation covering the levels, iterations, one pair and
 * the mode (OFV_ERR_CAPACITY otherwise).  Enqueues only: no allocation, no
 * sync.  Outputs must not overlap the inputs or each other. */
ofv_status ofv_compute_flow_backward(ofv_handle h, const ofv_image* frame0, const ofv_image* frame1,
                                     const ofv_params* params, const float* flow_init, const float* grad_flow,
                                     float* grad_frame0, float* grad_frame1, float* grad_flow_init);

/* ofv_compute_flow_backward over n pairs (sizes may differ), each stage one
 * launch for up to 16 pairs: frames0[i], frames1[i], grad_flow[i]; the
 * pointer arrays flow_init, grad_frame0, grad_frame1 and grad_flow_init may
 * each be NULL (no pair has one) or hold NULL entries.  The reservation must
 * cover n pairs.  No output may overlap any input or output of the batch. */
ofv_status ofv_compute_flow_backward_batch(ofv_handle h, int n, const ofv_image* frames0, const ofv_image* frames1,
                                           const ofv_params* params, const float* const* flow_init,
                                           const float* const* grad_flow, float* const* grad_frame0,
                                           float* const* grad_frame1, float* const* grad_flow_init);

/* Work decompositions of the fused Gauss-Newton kernel, chosen per pyramid
 * level and input-flow mode.  All give the same results up to float32
 * rounding order (parity with the FP64 reference holds for each). */
#define OFV_GN_AUTO (-1)      /* tuned table entry if any, else for launches of >= 3 Mi pixels the band
                                 (kernel_radius >= 8) or the march, OFV_GN_TILE_64x16 below */
#define OFV_GN_MARCH 0        /* 256-column strips marching down tile_h rows */
#define OFV_GN_TILE_64x32 1   /* 64 x 32 output tiles, 512 lanes per workgroup */
#define OFV_GN_TILE_64x16 2   /* 64 x 16 output tiles, 256 lanes per workgroup */
#define OFV_GN_TILE_32x16 3   /* 32 x 16 output tiles, 256 lanes (coarse levels) */
#define OFV_GN_TILE_16x16 4   /* 16 x 16 output tiles, 256 lanes (coarse levels) */
#define OFV_GN_TILE_64x32W 5  /* 64 x 32 output tiles, 1024 lanes per workgroup */
#define OFV_GN_TILE_64x16W 6  /* 64 x 16 output tiles, 512 lanes per workgroup */
#define OFV_GN_TILE_64x64 7   /* 64 x 64 output tiles, 1024 lanes per workgroup */
#define OFV_GN_TILE_16x16W 8  /* 16 x 16 output tiles, 1024 lanes per workgroup (coarse levels) */
#define OFV_GN_TILE_32x16W 9  /* 32 x 16 output tiles, 512 lanes per workgroup (coarse levels) */
#define OFV_GN_TILE_32x32W 10 /* 32 x 32 output tiles, 1024 lanes per workgroup */
#define OFV_GN_BAND 11        /* 256-column strips marching down in blocks of 4 rows, vertical window sums
                                 in registers; tile_h 0 = as many rows per tile as give every resident
                                 workgroup slot one tile */

/* Force a decomposition for later calls on h (OFV_GN_AUTO restores the
 * default); tile_h (rows per strip for OFV_GN_MARCH and OFV_GN_BAND) is 0 for automatic or
 * 4..1024.  The environment variable OFV_GN_VARIANT (march, tile64x32,
 * tile64x16, tile32x16, tile16x16, tile64x32w, tile64x16w, tile64x64,
 * tile16x16w, tile32x16w, tile32x32w or band; tile32 and tile16 are accepted for
 * tile64x32 and tile64x16), read at every launch, overrides both this
 * choice and the tuned table; levels one pixel wide or high always take the
 * march. */
ofv_status ofv_set_gn_variant(ofv_handle h, int variant, int tile_h);

/* Autotuner: runs the estimator on this pair with every candidate
 * decomposition (16x16, 32x16, 32x32, 64x16, 64x32 and 64x64 tiles with
 * 256 to 1024 lanes, strips of 16/32/64 rows): one untimed run each, then
 * `repeats` rounds in which the candidates take turns, every Gauss-Newton
 * launch timed with HIP events; per (window radius, storage, flow mode,
 * level size, batch size) it records the candidate with the lowest median
 * launch time in the handle, and later calls with matching geometry use it.
 * flow_out receives the flow (as ofv_compute_flow).  Unlike the compute
 * calls this synchronises the stream and may create HIP events; call it at
 * set-up, not inside graph capture.  1 <= repeats <= 1000. */
ofv_status ofv_autotune(ofv_handle h, const ofv_image* frame0, const ofv_image* frame1, const ofv_params* params,
                        float* flow_out, int repeats);

/* The autotuner on a batch: as ofv_autotune, with n pairs (possibly of
 * different sizes) computed together as ofv_compute_flow_batch computes
 * them, so the recorded choices are keyed by the batch's launch groups
 * (largest level size in the group, batch size n) and later batch calls of
 * the same geometry use them.  Arrays as ofv_compute_flow_batch (no initial
 * fields); 1 <= n <= max_batch. */
ofv_status ofv_autotune_batch(ofv_handle h, int n, const ofv_image* frame0, const ofv_image* frame1,
                              const ofv_params* params, float* const* flow_out, int repeats);

/* The tuned table as text, one entry per line:
 * "kr storage mode width height batch variant tile_h" (tile_h 4..1024; for
 * OFV_GN_BAND also 0: sized at every launch from the occupancy query, as
 * the autotuner's fixed heights 64, 128 and 256 are not).  Writes at most cap
 * bytes (NUL-terminated) to buf when buf is not NULL; *needed (if not NULL)
 * receives the size including the NUL.  OFV_ERR_CAPACITY if cap is short. */
ofv_status ofv_tuning_export(ofv_handle h, char* buf, size_t cap, size_t* needed);

/* Merge entries in the export format into h's table, one per line (blank
 * lines skipped); nothing is merged if any line is malformed (not exactly
 * eight integers) or invalid (OFV_ERR_INVALID_ARG). */
ofv_status ofv_tuning_import(ofv_handle h, const char* text);

/* ---- Time-resolved streaming (the paper's live regime: consecutive frames
 * of one camera, pairs (t, t+1)).  Each pushed frame is normalised and its
 * pyramid built once, into slot 0 of the handle's workspace; the next push
 * pairs it with the new frame.  ofv_stream_push(h, frame, ...) returns with
 * *produced = 0 on the first push after ofv_create, ofv_stream_reset or any
 * other compute call on h (those reuse the same workspace), and otherwise
 * writes to flow_out exactly what ofv_compute_flow_ex(previous frame, frame,
 * params, flow_init, flow_out) writes, bit for bit, with *produced = 1.
 * flow_init (nullable, e.g. the previous field as a warm start) and
 * flow_out follow ofv_compute_flow_ex; flow_out must be valid on every push.
 * num_levels, norm_radius, norm_eps and storage and the frame size must stay
 * those of the retained frame (OFV_ERR_INVALID_ARG otherwise); the window
 * radius, iterations and damping may change.  Host-side state: a push
 * captured in a hipGraph replays with the slab roles it had when captured,
 * so a graph loop alternates two captured pushes. */
ofv_status ofv_stream_push(ofv_handle h, const ofv_image* frame, const ofv_params* params, const float* flow_init,
                           float* flow_out, int* produced);

/* Forget the retained frame (the next push produces no flow). */
ofv_status ofv_stream_reset(ofv_handle h);

/* ---- Live derived quantities (cylinder-wake experiment of the paper's
 * section on live measurements; Eq. RA): observables computed from each
 * measured field as it streams, so that no field needs to be stored. */
typedef struct {
  float dx, dz;             /* pixel size along x (columns) and along y (rows), any length unit; > 0 */
  float dt;                 /* time between the two frames of a pair; > 0 */
  int32_t streamwise_sign;  /* +1: the free stream runs along +x, -1: along -x */
} ofv_derived_params;

/* dx = dz = dt = 1 (results in pixels and frame pairs), streamwise_sign = +1. */
void ofv_default_derived_params(ofv_derived_params* p);

/* One pass over a flow field (device, [2][height][pitch] float32, u plane
 * then v plane, displacement in pixels per pair, as ofv_compute_flow writes
 * it) that produces any of:
 *  - vorticity (device float32 plane, pitch vort_pitch): in image
 *    coordinates (x along columns, y along rows, y down) of the physical
 *    velocity (U, V) = (u dx / dt, v dz / dt):
 *      omega = ((dz / dx) dv/di - (dx / dz) du/dj) / dt,
 *    d/di the per-pixel central difference (f[i+1] - f[i-1]) / 2, one-sided
 *    f[1] - f[0] and f[n-1] - f[n-2] at the edges, 0 along a dimension of one
 *    pixel; 0 at masked pixels.
 *  - area (device, one double): the recirculation area of Eq. (RA),
 *    dx dz times the number of unmasked pixels with streamwise_sign * u < 0
 *    (strictly); the pixel count is exact.
 *  - probe_uv (device float32 [n_probes][2]): (u dx / dt, v dz / dt) by
 *    bilinear interpolation with clamped coordinates at the points
 *    probe_xy (device float32 [n_probes][2], (x, y) in pixels).
 * mask (device uint8 plane, pitch mask_pitch; NULL = every pixel valid):
 * 0 marks a masked pixel.  Each output is skipped when its pointer is NULL
 * (probes when n_probes == 0).  One kernel launch, plus a one-workgroup
 * launch that sums the per-workgroup pixel counts (kept in the handle's
 * workspace, so calls on one handle must not overlap: one handle per
 * stream) when the area is requested.
 * OFV_ERR_INVALID_ARG for NULL flow, sizes below 1, pitches below width,
 * non-positive or non-finite dx, dz, dt, a sign other than +-1,
 * n_probes outside 0..2^20, NULL probe arrays with n_probes > 0, or an
 * output overlapping the flow; OFV_ERR_UNSUPPORTED for planes of 2 GiB or
 * more. */
ofv_status ofv_derived(ofv_handle h, const float* flow, int width, int height, int64_t pitch, const uint8_t* mask,
                       int64_t mask_pitch, const ofv_derived_params* params, float* vorticity, int64_t vort_pitch,
                       const float* probe_xy, int n_probes, float* probe_uv, double* area);

/* Release the handle and its workspace.  NULL is accepted.  Synchronises the
 * handle's stream first. */
ofv_status ofv_destroy(ofv_handle h);

/* Static description of a status code. */
const char* ofv_status_string(ofv_status s);

/* Message of the last failing call on h (empty if none); valid until the
 * next call on h.  h == NULL gives the message of the last failing
 * ofv_create on this thread. */
const char* ofv_last_error(ofv_handle h);

#ifdef __cplusplus
}
#endif

#endif /* OFV_H */
