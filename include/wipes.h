/*
 * wipes.h -- C ABI of the MI355X (gfx950) wavelet rasterizer.
 *
 * The library renders, and differentiates, images made of wavelet
 * primitives as defined in "WIPES: Wavelet-based Visual Primitives"
 * (arXiv 2508.12615):
 *   - primitive:   W(x) = 1/2 [cos(f.(x - mu)) + 1] G(x; mu, Sigma)      Sec. 4.1, Eq. 6
 *   - projection:  Sigma' = 2x2 block of J W Sigma W^T J^T; f goes through
 *                  the same ray-space map                                 Sec. 3.1 Eq. 2; Sec. 4.1 Eq. 7
 *   - blending:    additive weighted sum (2D images)                      Sec. 3.2, Eq. 4
 *                  front-to-back alpha compositing (3D scenes)           Sec. 3.1, Eq. 3
 *   - rasterizer:  tile binning + depth-keyed sort + per-tile blending,
 *                  as in 3D Gaussian splatting                             Sec. 4.1
 *   - backward:    explicit gradients for every parameter                 Sec. 1 (contributions)
 *
 * Conventions for every call:
 *   - All pointers named "device" are HIP device pointers owned by the
 *     caller; the library never allocates on the render path.  Host
 *     structs (params, camera, batch) are read during the call only.
 *   - Every call returns a wipes_status and never throws.  Host-side
 *     validation (NULL pointers, sizes, mode mismatches) returns
 *     WIPES_ERR_INVALID before any work is queued.  A HIP failure returns
 *     WIPES_ERR_DEVICE; wipes_last_error() then holds the HIP message.
 *   - Calls are asynchronous on the given hipStream_t (passed as void*;
 *     NULL = the default stream) unless stated otherwise.
 *   - A wipes_ctx is used by one host thread at a time.  A wipes_server is
 *     internally synchronised.
 *   - Arrays are row-major; "[n, k]" means n rows of k float32 values.
 *
 * The per-pixel rule, identical for every tile shape and launch form:
 *   pixel (x, y) has centre p = (x + 1/2, y + 1/2); d = p - mu'; q = d^T A d
 *   with A = Sigma'^-1; phi = f'.d + phi0 (phi0 = 0 unless a phase is given);
 *   W' = 1/2 (1 + cos phi) exp(-q/2).
 *   Additive:  C = sum_i c_i o_i W'_i over primitives with q_i <= q_add, in
 *              primitive order.
 *   Alpha:     primitives in ascending depth key (ties by index); a = o W';
 *              skip if a < alpha_min; alpha = min(a, alpha_max);
 *              C += T alpha c; T *= 1 - alpha; stop after the pair that
 *              leaves T < T_min; finally C += T bg.
 */
#ifndef WIPES_H
#define WIPES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */

typedef enum {
    WIPES_OK = 0,
    WIPES_ERR_INVALID = 1,   /* bad argument; nothing was queued */
    WIPES_ERR_NOMEM = 2,     /* a buffer is too small, or a server arena is full */
    WIPES_ERR_CAPACITY = 3,  /* more tile instances than the bins buffer holds */
    WIPES_ERR_DEVICE = 4,    /* HIP runtime error (see wipes_last_error) */
    WIPES_ERR_BUSY = 5,      /* server queue full, or scene still in use */
    WIPES_ERR_NOTFOUND = 6   /* unknown scene or request id */
} wipes_status;

typedef enum {
    WIPES_2D_ADDITIVE = 0,   /* 2D primitives on the image plane, Eq. 4 with W' (Sec. 4.3) */
    WIPES_3D_ALPHA = 1       /* 3D primitives, EWA projection, Eq. 3 with W' (Sec. 4.1) */
} wipes_mode;

typedef enum {
    WIPES_COV_CHOLESKY = 0,  /* 2D: cov = (l11, l21, l22), Sigma = L L^T (Sec. 5.1) */
    WIPES_COV_RS = 1,        /* 2D: cov = (s1, s2, theta), Sigma = R diag(s1^2, s2^2) R^T (Sec. 5.1) */
    WIPES_COV_QUAT_SCALE = 2 /* 3D: Sigma = R(q) S S^T R(q)^T, q = (w,x,y,z) normalised inside (Sec. 3.1) */
} wipes_cov;

typedef enum {
    WIPES_FREQ_VECTOR = 0,   /* f' = J W f, the ray-space map applied to f as to Sigma (Sec. 4.1) */
    WIPES_FREQ_COVECTOR = 1  /* f' = first two components of (J3 W)^-T f, J3 = J with the third row
                                t/|t|: the carrier's phase f.(x - mu) is carried to first order
                                (3D only; 2D has f' = f either way) */
} wipes_freq_xform;

/* ---------------------------------------------------------------- inputs */

/* Rasterizer constants.  wipes_params_default() fills the documented defaults. */
typedef struct {
    int32_t mode;         /* wipes_mode */
    int32_t cov;          /* wipes_cov; must be QUAT_SCALE for 3D, CHOLESKY or RS for 2D */
    int32_t freq_xform;   /* wipes_freq_xform */
    int32_t tile_w;       /* tile width in pixels: 8, 16 or 32 */
    int32_t tile_h;       /* tile height in pixels: 8 or 16; tile_w * tile_h in {64, 128, 256, 512} */
    int32_t persistent;   /* blend launch form: 0: grid launch, a workgroup per tile, in tile
                             order; 1: persistent tile queue in tile order; 2: persistent queue,
                             longest tile list first; 3: grid launch, longest tile list first
                             (default).  Other values: WIPES_ERR_INVALID */
    float alpha_min;      /* 1/255: pairs with o W' below it are skipped (alpha) */
    float alpha_max;      /* 0.99: clamp of o W' (alpha) */
    float T_min;          /* 1e-4: termination threshold on transmittance (alpha) */
    float q_add;          /* 9: additive support q <= q_add (3-sigma ellipse) */
    float blur_eps;       /* Sigma' += eps I: 0.3 px^2 (3D), 0 (2D) */
    float near_plane;     /* 0.01: cull primitives with camera z <= near */
    float fov_guard;      /* 1.3: x/z, y/z clamped to +-guard*half-fov inside J */
    float bg[3];          /* background colour added with the final T (alpha) */
    int32_t sh_degree;    /* -1 (default): colour is the direct RGB input; 0..3 (3D only): colour is the
                             real spherical-harmonic expansion of degree sh_degree (Sec. 3.1) at the
                             unit direction from the camera centre to the mean, no offset, no clamp */
    int32_t lds_batch;    /* list positions a wave stages into LDS per batch: 64 (0 = 64); fixed at
                           * one 64-bit contribution-mask word, one position per lane */
} wipes_params;

/* Pinhole camera.  viewmat is world->camera, row-major 4x4, OpenCV axes
 * (x right, y down, z forward).  2D mode uses width/height only. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float viewmat[16];
    float time;           /* tau: means move as mu0 + v tau when velocity != NULL */
} wipes_camera;

/* Device arrays of one image's primitives (structure of arrays, float32).
 * D = 2 (2D) or 3 (3D).  Unused members may be NULL.
 *   mean [n, D], cov [n, 3] (2D), quat [n, 4] (3D), scale [n, 3] (3D),
 *   freq [n, D] (rad per pixel in 2D, rad per world unit in 3D),
 *   color [n, 3] (unused with sh_degree >= 0), opacity [n], velocity [n, 3] (3D, optional),
 *   phase [n] (optional carrier phase phi0 in radians: the carrier becomes
 *   cos(f'.(x - mu') + phi0); NULL = 0, the primitive of Eq. 6),
 *   sh [n, (sh_degree + 1)^2, 3] (spherical-harmonic colour coefficients, 3D). */
typedef struct {
    int64_t n;
    const float* mean;
    const float* cov;
    const float* quat;
    const float* scale;
    const float* freq;
    const float* color;
    const float* opacity;
    const float* velocity;
    const float* phase;
    const float* sh;
} wipes_prims;

/* Device gradient outputs, same shapes as wipes_prims; NULL members are skipped.
 * render_bwd overwrites (does not accumulate into) every non-NULL array. */
typedef struct {
    float* mean;
    float* cov;
    float* quat;
    float* scale;
    float* freq;
    float* color;
    float* opacity;
    float* velocity;
    float* phase;
    float* sh;
} wipes_prims_grad;

typedef struct {
    wipes_camera cam;
    wipes_prims prims;
    wipes_prims_grad grads;   /* read by wipes_render_bwd only */
    float* out_image;         /* optional device [W H, 3]: wipes_render_fwd writes this image's colours
                                 here instead of into the batch image array (NULL: batch array) */
} wipes_image;

/* A batch of images rendered together (B = 1 is the plain rasterizer).
 * Pixels of image b occupy [pix_b, pix_b + W_b H_b) of every per-pixel
 * array, pix_b = sum of W H over earlier images; tiles are numbered the same
 * way (global tile = tiles of earlier images + ty * tiles_x + tx). */
typedef struct {
    int32_t n_images;
    const wipes_image* images;   /* host array of n_images */
} wipes_batch;

/* Caller-allocated device workspace.  For the bins buffer, capacity and
 * with_backward must be the values passed to wipes_workspace_size (the
 * buffer layout depends on them); the screen buffer ignores both. */
typedef struct {
    void* base;
    size_t bytes;
    int64_t capacity;        /* bins: instance capacity */
    int32_t with_backward;   /* bins: sized for the backward pass */
    int32_t reserved;
} wipes_buffer;

/* Screen-space record written by wipes_project, one per primitive, 64 bytes,
 * at the start of the screen buffer in batch order (image 0's primitives
 * first).  The mean is mx + mx_lo (an FP32 pair carrying an FP64 value, so
 * the carrier phase stays exact at 1080p).  r, g, b are the colour the blend
 * uses (evaluated from the spherical harmonics when sh_degree >= 0).
 * box0/box1 pack the pixel box (x0 | y0 << 16, x1 | y1 << 16) and are written
 * by wipes_bin_sort. */
typedef struct {
    float mx, my;          /* mu' (pixels), FP32 rounding */
    float ca, cb, cc;      /* conic A = Sigma'^-1 = [[ca, cb], [cb, cc]] */
    float fx, fy;          /* f' (rad per pixel) */
    float opacity;
    float r, g, b;
    float mx_lo, my_lo;    /* mu' - (mx, my) */
    float phase_rev;       /* carrier phase phi0 / (2 pi), in revolutions */
    uint32_t box0, box1;
} wipes_screen_record;

/* Binning inputs written by wipes_project right after the records
 * (screen buffer offset sum_n * 64), one per primitive, 16 bytes. */
typedef struct {
    float rx, ry;          /* half-extents of the support box (pixels); rx < 0: culled */
    float depth;           /* FP32 depth key (3D), 0 (2D) */
    float reserved;
} wipes_bin_input;

/* ------------------------------------------------------------- context */

typedef struct wipes_ctx wipes_ctx;

/* Fill p with the defaults listed in wipes_params for the given mode. */
void wipes_params_default(int32_t mode, wipes_params* p);

/* Create a context on HIP device `device` (made current for the call). */
wipes_status wipes_ctx_create(int32_t device, wipes_ctx** out);
void wipes_ctx_destroy(wipes_ctx* ctx);
/* Message of the last failing call on this context ("" if none).  Owned by ctx. */
const char* wipes_last_error(const wipes_ctx* ctx);

/* Bytes of the screen and bins buffers for a batch and an instance capacity
 * (number of (primitive, tile) pairs).  with_backward != 0 adds room for the
 * backward pass.  Host only; no device work. */
wipes_status wipes_workspace_size(const wipes_params* p, const wipes_batch* batch, int64_t capacity_instances,
                                  int32_t with_backward, size_t* screen_bytes, size_t* bins_bytes);

/* ---------------------------------------------------------- render path */

/* Project every primitive of the batch to its screen record (Eq. 2, Eq. 7 and
 * the frequency transform of Sec. 4.1 for 3D; identity placement for 2D). */
wipes_status wipes_project(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* batch, wipes_buffer* screen,
                           void* stream);

/* Tile binning and sort (Sec. 4.1: the tile pipeline of 3D Gaussian
 * splatting with W' in place of the projected Gaussian; Sec. 1: primitives
 * sorted with a GPU sort, depth-ordered per tile for Eq. 3): pixel boxes,
 * per-primitive tile counts, instance emission, stable sort by (tile, depth
 * key, index), per-tile ranges.
 * n_instances_out != NULL: the call synchronises the stream once to read the
 * instance count K into *n_instances_out, and returns WIPES_ERR_CAPACITY
 * (with *n_instances_out = K) if K exceeds the bins buffer's capacity.
 * n_instances_out == NULL: no host synchronisation (graph capture); an
 * overflow sets a device flag that turns the later stages into no-ops and is
 * reported by wipes_check_overflow.
 * It also clears the persistent-queue counters, contribution mask and slot
 * marks of the renders that follow, so the first wipes_render_fwd and the
 * first wipes_render_bwd on the same context and buffers skip their own
 * clearing; later renders of the same bins clear again.  Rendering these
 * buffers through another context in between is not supported.
 * wipes_project stores the batch's descriptor table in the screen buffer;
 * the later stages of the frame reuse it when the batch is unchanged, so the
 * screen buffer must still hold what wipes_project wrote (as it must anyway). */
wipes_status wipes_bin_sort(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* batch, wipes_buffer* screen,
                            wipes_buffer* bins, int64_t* n_instances_out, void* stream);

/* Forward blend (Eq. 3 or Eq. 4 with W').  image: device [sum W H, 3];
 * T_final, last: device [sum W H] (alpha mode; may be NULL in additive mode).
 * last holds the sorted-list position of the last contributing pair (-1: none).
 * With a bins buffer sized with_backward, the forward also records, per 8 x 8
 * pixel block of each tile, which list positions contributed to a pixel of the
 * block; wipes_render_bwd replays exactly those. */
wipes_status wipes_render_fwd(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* batch,
                              const wipes_buffer* screen, const wipes_buffer* bins, float* image, float* T_final,
                              int32_t* last, void* stream);

/* Backward pass (Sec. 1: explicit gradients of Eq. 3 / Eq. 4 with W' of
 * Eq. 6-7 for every primitive parameter, in place of automatic
 * differentiation): dL/dimage (device [sum W H, 3]) -> parameter gradients
 * written to each image's grads.  Alpha mode walks each pixel's list back
 * to front from `last`, recovering transmittance by dividing by (1 - alpha)
 * (nothing per pair is stored by the forward).  dscreen (optional, device
 * [sum n, 12]) receives the screen-space gradients d/d(mu'x, mu'y, ca, cb, cc,
 * f'x, f'y, opacity, r, g, b, phi0).  Needs the bins buffer sized with_backward, on
 * which wipes_render_fwd has run after the last wipes_bin_sort (the backward
 * reads the forward's per-block contribution record from it). */
wipes_status wipes_render_bwd(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* batch,
                              const wipes_buffer* screen, const wipes_buffer* bins, const float* T_final,
                              const int32_t* last, const float* dL_dimage, float* dscreen, void* stream);

/* Read back the instance count K and the overflow flag of the last bin_sort
 * on this screen buffer (synchronises the stream).  Returns WIPES_ERR_CAPACITY
 * if K exceeded the bins capacity, WIPES_OK otherwise. */
wipes_status wipes_check_overflow(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* batch,
                                  const wipes_buffer* screen, int64_t* required_instances, void* stream);

/* Device views into the bins buffer after bin_sort (for inspection and tests):
 * sorted tile keys and primitive indices [K] and tile ranges [n_tiles, 2]. */
wipes_status wipes_bins_view(const wipes_params* p, const wipes_batch* batch, const wipes_buffer* screen,
                             const wipes_buffer* bins, const uint32_t** keys, const uint32_t** vals,
                             const uint32_t** ranges, int64_t* n_tiles);

/* ------------------------------------------------ allocation-free form */

/* Size of the static device workspace of wipes_render_fwd_noalloc. */
#define WIPES_NOALLOC_WORKSPACE_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: one forward
 * frame, i.e. wipes_project + wipes_bin_sort + wipes_render_fwd with the same
 * kernels and the same outputs, whose screen and bins workspaces are carved
 * from a static device array of WIPES_NOALLOC_WORKSPACE_BYTES (the screen
 * part first, then bins of the largest instance capacity that fits).  Each
 * device the library runs on holds its own array until the process ends.
 * The call allocates nothing: no hipMalloc, hipFree, event creation or other
 * allocating routine, on any path.
 *   image, T_final, last: the caller's device arrays, as wipes_render_fwd.
 *   n_instances_out != NULL: the stream is synchronised once to read the
 *     instance count K (as wipes_bin_sort does); if K exceeds the capacity
 *     that fits, nothing is rendered and WIPES_ERR_CAPACITY is returned with
 *     *n_instances_out = K.  NULL: no host synchronisation; a frame that
 *     overflows leaves image, T_final and last unwritten.
 * Errors: WIPES_ERR_INVALID as wipes_render_fwd; WIPES_ERR_CAPACITY, before
 * any work is queued, when the batch's projection workspace (about 200 bytes
 * per primitive) leaves no room for bins; wipes_last_error names the sizes.
 * Every call on a device uses that device's one array and leaves its
 * contents behind (nothing needs to start zeroed: the stages clear what they
 * use): calls that overlap on one device -- from two host threads, or on two
 * streams not ordered with each other -- race and give wrong images.
 * Asynchronous on the stream unless n_instances_out is set. */
wipes_status wipes_render_fwd_noalloc(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* batch, float* image,
                                      float* T_final, int32_t* last, int64_t* n_instances_out, void* stream);

/* ---------------------------------------------------- deformation network */

/* The network F of Sec. 4.3, Eq. 8, that maps the positional encodings of a
 * primitive's position and of the time to offsets of its position, frequency
 * and covariance, in the D-3DGS configuration the paper keeps for its other
 * settings (Sec. 3.2, Sec. 5.3):
 *   e = (gamma(x), gamma(t)), gamma(p) = (p, sin(2^k pi p), cos(2^k pi p) for
 *   k < L), the components of p kept together inside each block; L = 10 for
 *   the position, 6 for the time: 63 + 13 = 76 inputs;
 *   8 ReLU layers of 256 units; e joins the fifth layer's output (the sixth
 *   layer reads 256 + 76 inputs); a linear output layer of 13 values
 *   (dx[3], df[3], dq[4], ds[3]): the offsets added to mean, freq, quat (before
 *   normalisation) and the linear scales of a 3D primitive.
 * Parameters: one flat FP32 device array, per layer W [out][in] row-major
 * then b [out]: W0 [256][76], b0, W1..W4 [256][256], b1..b4, W5 [256][332],
 * b5, W6, W7 [256][256], b6, b7, Wo [13][256], bo -- wipes_deform_param_count()
 * values (503053).
 *
 * The products run on the matrix cores.  WIPES_DEFORM_BF16X3 splits every
 * operand into two bf16 parts and keeps three of the four partial products
 * (FP32 accumulation; about 2^-16 relative per product, FP32-class);
 * WIPES_DEFORM_BF16 keeps the leading one (about 2^-8 relative). */
enum { WIPES_DEFORM_BF16X3 = 0, WIPES_DEFORM_BF16 = 1 };

/* Number of FP32 values in the flat parameter array. */
int64_t wipes_deform_param_count(void);

/* Device workspace bytes for n primitives; with_backward != 0 adds the stored
 * layer inputs and the backward's scratch (about 17 KB per primitive). */
wipes_status wipes_deform_workspace_size(int64_t n, int32_t with_backward, size_t* bytes);

/* offsets[n][13] = F(e(mean[i], time)) for mean[n][3] (device, FP32).  The
 * workspace (device, caller-owned, >= wipes_deform_workspace_size(n,
 * keep_for_backward)) receives the split weights and, when keep_for_backward
 * != 0, the layer inputs wipes_deform_bwd reads; it must then be left as is
 * until that call.  Asynchronous on `stream`.  INVALID for a bad precision,
 * n < 0 or missing pointers; NOMEM when workspace_bytes is too small. */
wipes_status wipes_deform_fwd(wipes_ctx* ctx, int32_t precision, const float* params, int64_t n, const float* mean,
                              float time, float* offsets, void* workspace, size_t workspace_bytes,
                              int32_t keep_for_backward, void* stream);

/* Gradients for the upstream d_offsets[n][13]: d_params (overwritten, laid
 * out like params) and d_mean[n][3] (overwritten; the encoding's derivative).
 * Needs the workspace of a wipes_deform_fwd call with keep_for_backward != 0
 * on the same params, mean, time and precision.  Deterministic: the row sums
 * are taken in a fixed order.  Asynchronous on `stream`; errors as above. */
wipes_status wipes_deform_bwd(wipes_ctx* ctx, int32_t precision, const float* params, int64_t n, const float* mean,
                              float time, const float* d_offsets, void* workspace, size_t workspace_bytes,
                              float* d_params, float* d_mean, void* stream);

/* The deformed primitive set of Sec. 4.3 (the offsets of Eq. 8 added to a 3D
 * primitive's parameters): out_mean = mean + dx, out_freq = freq + df,
 * out_quat = quat + dq, out_scale = scale + ds, for offsets[n][13] from
 * wipes_deform_fwd and device arrays mean/freq/scale [n][3], quat [n][4];
 * the outputs may alias the inputs.  Its backward is the identity: the
 * rasterizer's gradients for the deformed mean, freq, quat and scale are the
 * columns 0-2, 3-5, 6-9 and 10-12 of d_offsets.  Asynchronous on `stream`;
 * INVALID for n < 0 or a missing array. */
wipes_status wipes_deform_apply(wipes_ctx* ctx, int64_t n, const float* offsets, const float* mean,
                                const float* freq, const float* quat, const float* scale, float* out_mean,
                                float* out_freq, float* out_quat, float* out_scale, void* stream);

/* ------------------------------------------------------- fitting, graphs */

/* Gradient of the L2 fitting loss L = sum over images of the mean over that
 * image's 3 W H values of (C - target)^2 (the 2D image-fitting objective,
 * Sec. 5.1): dL_dimage = 2 (image - target) / (3 W H).  All three arrays are
 * device [sum W H, 3]. */
wipes_status wipes_l2_grad(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* batch,
                           const wipes_buffer* screen, const float* image, const float* target, float* dL_dimage,
                           void* stream);

typedef struct wipes_graph wipes_graph;

/* Capture one whole render step of a fixed batch into a hipGraph: project,
 * bin/sort (no host synchronisation; grids sized by bins->capacity), forward
 * blend, then, if target != NULL, the L2 gradient into dL_dimage, and, if
 * backward != 0, the backward pass into each image's grads.  Every pointer
 * (batch arrays, buffers, outputs) must stay valid and the batch unchanged for
 * the graph's lifetime; parameter values may change between launches.  If
 * the instance count outgrows the capacity the replay leaves its outputs
 * untouched and wipes_check_overflow reports WIPES_ERR_CAPACITY; capture again
 * with a larger bins buffer.  The capture itself runs on a private stream and
 * synchronises it once (descriptor upload). */
wipes_status wipes_graph_capture(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* batch,
                                 wipes_buffer* screen, wipes_buffer* bins, float* image, float* T_final,
                                 int32_t* last, const float* target, float* dL_dimage, int32_t backward,
                                 wipes_graph** out);

/* Replay a captured step on a stream (asynchronous). */
wipes_status wipes_graph_launch(wipes_graph* g, void* stream);
void wipes_graph_destroy(wipes_graph* g);

/* One Adam step (the optimiser of the 2D fitting experiments, Sec. 5.1) over
 * up to WIPES_ADAM_MAX_GROUPS parameter groups, in one launch.  Per element,
 * with t = *step + 1:
 *   m = m + (1 - beta1)(g - m),  v = beta2 v + (1 - beta2) g^2,
 *   param = param - (lr / (1 - beta1^t)) m / (sqrt(v) / sqrt(1 - beta2^t) + eps),
 * then *step = t.  Each group: device float32 param, grad, m and v of n
 * elements (m and v start at zero and belong to the caller) and its learning
 * rate.  step: device uint32 count of applied steps (the bias corrections are
 * formed on the device from it, so a captured sequence can replay this call).
 * When screen is given (p and batch describing it), the step is skipped on the
 * device -- nothing written, *step unchanged -- if the last bin_sort on that
 * screen buffer overflowed its capacity, so a replayed render + Adam sequence
 * never applies the gradients of a truncated render; the caller learns of a
 * skipped step from *step.  Asynchronous.  WIPES_ERR_INVALID for n_groups
 * outside [1, WIPES_ADAM_MAX_GROUPS], a NULL array with n > 0, or more than
 * 2^31 elements in all. */
#define WIPES_ADAM_MAX_GROUPS 8
typedef struct {
    float* param;
    const float* grad;
    float* m;
    float* v;
    int64_t n;
    double lr;
} wipes_adam_group;

wipes_status wipes_adam(wipes_ctx* ctx, int32_t n_groups, const wipes_adam_group* groups, double beta1, double beta2,
                        double eps, uint32_t* step, const wipes_params* p, const wipes_batch* batch,
                        const wipes_buffer* screen, void* stream);

/* ------------------------------------------------------------ autotuning */

/* Candidates the autotuner tries, in the order of its times_ms output:
 * tile shapes 8x8, 16x8, 8x16, 16x16, 32x8, 32x16, each as a grid launch
 * (persistent 0), a persistent queue in tile order (1), a persistent queue
 * longest list first (2) and a grid launch longest list first (3).  Fills up
 * to max entries; returns the count. */
int32_t wipes_autotune_candidates(int32_t* tile_w, int32_t* tile_h, int32_t* persistent, int32_t max);

/* Time the render path of this batch (project, bin/sort, forward, and the
 * backward if with_backward) for every candidate, reps timed runs each after
 * one warm-up, and copy p with the fastest tile shape and launch form into
 * *best.  times_ms (optional) receives each candidate's mean.  Offline call:
 * allocates and frees its own scratch and synchronises the stream.  The
 * per-pixel rule is tile-independent, so every candidate renders the same
 * image. */
wipes_status wipes_autotune(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* batch, int32_t with_backward,
                            int32_t reps, wipes_params* best, double* times_ms, void* stream);

/* --------------------------------------------------------------- serving */

/* Rendering of resident 3D scenes on request: each request is one novel view
 * of a scene (Sec. 3.1 projection and Eq. 3 compositing with W', Sec. 4.1),
 * optionally at a time t for the scenes with a linear-in-time mean (the
 * dynamic setting of Sec. 4.3 with its deformation reduced to a velocity). */

typedef struct wipes_server wipes_server;

typedef struct {
    int32_t max_slots;         /* requests in flight at once */
    int32_t max_pending;       /* waiting requests before submit returns WIPES_ERR_BUSY */
    int32_t max_batch;         /* requests per launch */
    int32_t persistent;        /* blend launch form across the batch, as wipes_params.persistent */
    int64_t hbm_budget_bytes;  /* arena for per-request workspaces, allocated at create */
} wipes_serve_config;

typedef struct {
    double p50_ms, p99_ms, mean_ms;   /* submit -> completion latency of completed requests */
    double frames_per_s;              /* completed / (last completion - first submit) */
    int64_t completed, admitted, deferred, batches;
    double mean_batch;                /* requests per launch */
    int64_t arena_peak_bytes;
} wipes_serve_report;

/* Create a server on `device` for 3D alpha rendering with constants p.  It
 * owns a context, two streams, its scene copies and one arena of
 * hbm_budget_bytes; a worker thread admits requests in FIFO order when request
 * slots and one arena block for the batch's workspace (projection records,
 * bins, per-pixel state) are free, renders each admitted batch -- requests of
 * any resolution together -- with projection and sort on one stream and the
 * blend on another, so the next batch is prepared while the current one
 * blends.  Internally synchronised: every serve call may come from any thread. */
wipes_status wipes_serve_create(const wipes_serve_config* cfg, const wipes_params* p, int32_t device,
                                wipes_server** out);
/* Copy a scene (device arrays, 3D layout of wipes_prims) into server memory. */
wipes_status wipes_serve_load_scene(wipes_server* s, const wipes_prims* prims, int32_t* scene_id);
/* WIPES_ERR_BUSY while requests for the scene are pending or in flight. */
wipes_status wipes_serve_unload_scene(wipes_server* s, int32_t scene_id);
/* Queue a render of scene scene_id seen from cam (Eq. 3 with W', as
 * wipes_render_fwd; non-blocking).  out_image: device array of out_floats
 * floats, at least W H 3 ([H, W, 3] row-major), that must stay valid until
 * poll reports the request done.  stream: the caller's stream (NULL = the
 * default stream); the server writes out_image only after the work queued on
 * that stream before this call, so the caller may still be filling or reading
 * the buffer there.  WIPES_ERR_NOMEM if out_floats < W H 3, WIPES_ERR_BUSY if
 * the queue is full, WIPES_ERR_NOTFOUND for an unknown scene. */
wipes_status wipes_serve_submit(wipes_server* s, int32_t scene_id, const wipes_camera* cam, float* out_image,
                                size_t out_floats, void* stream, uint64_t* req_id);
/* *done = 1 once the image is in out_image; then *latency_ms is the submit ->
 * completion time and the id is forgotten. */
wipes_status wipes_serve_poll(wipes_server* s, uint64_t req_id, int32_t* done, double* latency_ms);
/* Block until every submitted request has completed. */
wipes_status wipes_serve_drain(wipes_server* s);
wipes_status wipes_serve_stats(wipes_server* s, wipes_serve_report* out);
wipes_status wipes_serve_reset_stats(wipes_server* s);
void wipes_serve_destroy(wipes_server* s);

/* Host-only model of the server's scheduler with a fake executor (no device
 * work): request i arrives at t_arrive[i] (sorted), holds footprint[i] arena
 * bytes while admitted; a batch's preparation takes the sum of its prep_s on
 * the prep stream, its blend the sum of blend_s on the blend stream (blends run
 * one after another, overlapping the next preparation).  Writes admission and
 * completion times, the batch index of each request and the arena peak. */
wipes_status wipes_serve_simulate(const wipes_serve_config* cfg, int64_t n, const double* t_arrive,
                                  const int64_t* footprint, const double* prep_s, const double* blend_s,
                                  double* t_admit, double* t_done, int64_t* batch_of, int64_t* arena_peak);

/* ------------------------------------------------------------ profiling */

/* Stages of the render path, in pipeline order. */
enum {
    WIPES_STAGE_PROJECT = 0, WIPES_STAGE_BIN_COUNT, WIPES_STAGE_SCAN, WIPES_STAGE_DEPTH_SORT,
    WIPES_STAGE_RANK_SCAN, WIPES_STAGE_EMIT, WIPES_STAGE_TILE_SORT, WIPES_STAGE_RANGES,
    WIPES_STAGE_BLEND_FWD, WIPES_STAGE_BLEND_BWD, WIPES_STAGE_PROJECT_BWD, WIPES_N_STAGES
};

/* Name of a stage ("" if out of range). */
const char* wipes_stage_name(int32_t stage);

/* When enabled, every stage of the render path on this context is bracketed
 * by a pair of HIP events recorded on the stream it is launched on (for
 * benchmarks; adds two event records per stage). */
wipes_status wipes_profile_enable(wipes_ctx* ctx, int32_t enable);

/* Waits for the recorded events and returns, per stage, the summed duration
 * in ms (ms[WIPES_N_STAGES]) and the number of launches since the last read;
 * then forgets them. n must be >= WIPES_N_STAGES. */
wipes_status wipes_profile_read(wipes_ctx* ctx, double* ms, int64_t* launches, int32_t n);

/* Issue-rate probe for the blend's roofline (synchronises; allocates two
 * events): the sustained lane operations per second of one instruction on
 * this device -- op 0: FP32 fused multiply-add, 1: exp2, 2: cos, 3: sin,
 * 4: reciprocal, the transcendentals of the per-pixel rule (Eq. 6-7 and its
 * derivatives) -- from a kernel of independent chains of that instruction
 * over every SIMD.  The FMA rate divided by a transcendental's rate is the
 * number of issue slots that transcendental takes. */
wipes_status wipes_probe_issue_rate(wipes_ctx* ctx, int32_t op, double* lane_ops_per_s, void* stream);

/* Work counts of a rendered frame, for roofline accounting (synchronises):
 *   out[0]  support pairs the forward evaluates: (pixel, primitive) pairs with
 *           the pixel inside the primitive's support (q <= q_add, or in alpha
 *           mode q <= 2 ln(o / alpha_min)), up to the pixel's stopping pair;
 *   out[1]  support pairs the backward revisits (alpha: up to `last`);
 *   out[2]  tile pairs: instances x valid pixels of their tile;
 *   out[3]  pairs visited after 8x8 sub-block culling.
 * T_final and last are the forward's outputs (alpha mode). */
wipes_status wipes_render_stats(wipes_ctx* ctx, const wipes_params* p, const wipes_batch* batch,
                                const wipes_buffer* screen, const wipes_buffer* bins, const float* T_final,
                                const int32_t* last, uint64_t* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WIPES_H */
