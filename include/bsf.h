/*
 * bsf.h -- C ABI of libbsf, a space-variant box-spline filter for AMD Instinct
 * MI355X (gfx950).
 *
 * The filter is the O(1) space-variant elliptical filter of K. N. Chaudhury and
 * S. Sanyal, "Improvements on 'Fast space-variant elliptical filtering using box
 * splines'" (arXiv:1109.5114): one global pre-integration of the image by
 * running sums along N integer lattice directions (Section 1.1, first step of
 * BoxFilter; Alg. 3 step 2), followed at every pixel by a signed finite
 * difference of the running sum whose steps are that pixel's own box lengths
 * (Section 1.1, second step of BoxFilter; Table 1; Alg. 3 step 3), divided by
 * the product of the steps (the weight w of Table 1).  "Order r" convolves the
 * box spline with itself r times (Section 1.2 and Section 2.1: higher-order box
 * splines), so there are M = N*r box factors per pixel.
 *
 * What each pixel computes (x = column, y = row, f = 0 outside the image):
 *
 *   integer steps:     out(x) = sum_{i in prod_j I_j} f(x + sum_j i_j u_j) / prod_j s_j
 *                      with I_j = {c_j - s_j + 1, ..., c_j}, c_j = floor((s_j - 1)/2),
 *                      the half-open box Box_s of Section 1.1 used as a
 *                      convolution kernel;
 *   continuous steps:  out(x) = sum_{i in Z^M} prod_j w_{s_j}(i_j) f(x + sum_j i_j u_j) / prod_j s_j
 *                      with w_s(i) = |[i - 1/2, i + 1/2] ^ [-s/2, s/2]|, the box of
 *                      length s integrated over the unit cells of its lattice
 *                      line.  This equals reading the running sum linearly
 *                      between lattice points along u_j, the one-direction
 *                      restriction of the box-spline interpolation of
 *                      eq. interpolation.  bsf_filter_alg3 computes the
 *                      paper's own two-dimensional form of Alg. 3 in FP64.
 *
 * Arithmetic.  The running sums and the signed tap combination are exact
 * two's-complement integers modulo 2^64 (BSF_ARITH_EXACT): a float image is
 * first scaled to fixed point, f_q = nearest-even(f * 2^F); the tap combination
 * is an integer that is bounded even though the running sums wrap, so it comes
 * out exact.  Phase weights of continuous steps and the final division are FP64,
 * rounded once to FP32.  BSF_ARITH_FP64 runs the same method with plain FP64
 * running sums and FP64 taps; it is provided as the plain baseline and loses
 * accuracy through cancellation on large images and at order 2.
 *
 * Conventions for every entry point:
 *   - Device pointers unless noted "host".  The caller owns every buffer; the
 *     library never allocates device memory and never synchronises, except
 *     bsf_read_device_status which synchronises the given stream.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *   - Images are row-major with a row pitch counted in elements (>= W).
 *   - Step fields are FP32 [planes][H][W], dense.  planes = N when tied (one
 *     step per direction, used by its r box factors), N*r when untied (factor
 *     j = k*r + q lies along direction k and reads plane j).
 *   - Host-side validation returns BSF_E_* before anything is enqueued.  Values
 *     found bad on the device (a NaN step, a step below 1 or above max_step, a
 *     non-integer step in integer mode, a fixed-point overflow bound) raise
 *     sticky bits in the status word at the start of the workspace, read with
 *     bsf_read_device_status; the outputs of such pixels are unspecified.
 *   - Calls that share a workspace must not overlap in time.
 */
#ifndef BSF_H
#define BSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BSF_OK = 0,
    BSF_E_INVALID = 1,     /* bad argument: null pointer, bad direction, pitch < W, ... */
    BSF_E_RANGE = 2,       /* device status: a step out of range, NaN or non-integer */
    BSF_E_OVERFLOW = 3,    /* fixed-point headroom cannot hold the tap combination */
    BSF_E_WORKSPACE = 4,   /* workspace too small */
    BSF_E_DEVICE = 5,      /* a HIP call failed */
    BSF_E_UNSUPPORTED = 6  /* valid request outside what this build implements */
} bsf_status;

typedef enum { BSF_U8 = 1, BSF_U16 = 2, BSF_F32 = 3 } bsf_dtype;
typedef enum { BSF_STEPS_INT = 0, BSF_STEPS_REAL = 1 } bsf_step_mode;
typedef enum { BSF_ARITH_EXACT = 0, BSF_ARITH_FP64 = 1 } bsf_arith;

#define BSF_MAX_DIRS 8
#define BSF_MAX_FACTORS 16

/* Device status bits (bsf_read_device_status). */
#define BSF_FLAG_RANGE 1u      /* a step NaN, below 1, above max_step, or non-integer in integer mode */
#define BSF_FLAG_OVERFLOW 2u   /* a requested F leaves the tap combination without int64 headroom */
#define BSF_FLAG_NONFINITE 4u  /* a NaN or infinite image sample or upstream gradient */

/*
 * Filter configuration.
 *   dirs:      n_dirs distinct primitive integer vectors (dx, dy), x = column,
 *              y = row, in canonical sign (dx > 0, or dx == 0 and dy > 0), e.g.
 *              (1,0), (0,1), (1,1), (1,-1) for the box spline of Section 1.1 or
 *              (2,1), (1,2), (1,-2), (2,-1) for the one of Alg. 3 and Table 1.
 *              The running sums are taken in the order given, each line started
 *              at zero where it enters the finite window; what that leaves out is
 *              cancelled exactly by the taps' differences along every direction.
 *   order:     r >= 1 (box spline convolved r times); n_dirs * order <= 16.
 *   tied:      1: one step plane per direction, 0: one plane per box factor.
 *   mode:      BSF_STEPS_INT (integer steps, exact integer output) or
 *              BSF_STEPS_REAL (continuous steps).
 *   max_step:  upper bound on every step (>= 1); it sizes the padding of the
 *              running-sum window.  Steps above it raise BSF_FLAG_RANGE.
 *   frac_bits: F for float images: 0..62 fixes it, -1 chooses on the device the
 *              largest F for which the tap combination cannot overflow,
 *              F = 62 - ceil(log2 max|f|) - max_x ceil(log2 prod_j L_j(x)) with
 *              L_j = 2 floor((s_j - 1)/2) + 3 (continuous) or s_j (integer steps):
 *              it is not clamped, so images of tiny magnitude get F > 62 and
 *              huge ones F < 0 (f_q = nearest-even(f 2^F) in both cases).
 *              Ignored for integer images (F = 0) and for BSF_ARITH_FP64.
 *   arith:     BSF_ARITH_EXACT or BSF_ARITH_FP64.
 */
typedef struct {
    int32_t n_dirs;
    int32_t dirs[2 * BSF_MAX_DIRS];
    int32_t order;
    int32_t tied;
    int32_t mode;
    float max_step;
    int32_t frac_bits;
    int32_t arith;
} bsf_config;

/*
 * Geometry of the running-sum window for a (config, H, W): the window covers
 * rows [-pad_top, H + pad_bottom) and columns [-pad_left, W + pad_right) so
 * that every tap of every pixel lands inside it.  G is stored row-major
 * [win_h][win_w] with 8-byte elements (int64, or double for BSF_ARITH_FP64);
 * the value at (x, y) sits at G[(y + pad_top) * win_w + (x + pad_left)].
 * win_w is padded to a multiple of 16 elements.
 */
typedef struct {
    int64_t pad_top, pad_bottom, pad_left, pad_right;
    int64_t win_h, win_w;
    size_t g_bytes;          /* win_h * win_w * 8 */
    size_t workspace_bytes;  /* bytes bsf_filter_varying needs when G is not saved */
    size_t workspace_bytes_g_external; /* bytes it needs when the caller passes G_save */
} bsf_geometry;

/*
 * Enqueues the clearing of the status word at the start of a workspace.  Call
 * once on every new workspace before its first use (the flags are sticky).
 */
bsf_status bsf_workspace_init(void *ws, size_t ws_bytes, void *stream);

/* Host only.  Fills *geo; BSF_E_INVALID for a bad configuration or size. */
bsf_status bsf_plan(const bsf_config *cfg, int64_t H, int64_t W, bsf_geometry *geo);

/*
 * Pre-integration alone (Section 1.1, first step; Alg. 3 step 2).
 *   img:   [H][pitch] of dtype.
 *   F:     fixed-point bits for float images (0..62); ignored for integer images
 *          and for BSF_ARITH_FP64.
 *   G:     output window, bsf_geometry layout (int64 or double by cfg->arith).
 *   ws:    scratch of at least bsf_geometry.workspace_bytes_g_external bytes.
 * G = (S_{u_N})^r ... (S_{u_1})^r f_q on the window, each running sum
 * S_u g(p) = g(p) + S_u g(p - u) started at zero where its line enters the
 * window, wrapping modulo 2^64.
 */
bsf_status bsf_preintegrate(const bsf_config *cfg, bsf_dtype dtype, const void *img,
                            int64_t H, int64_t W, int64_t pitch, int32_t F,
                            void *G, void *ws, size_t ws_bytes, void *stream);

/*
 * Forward filter, the whole hot path: the running sums of the image along every
 * direction (Section 1.1, first step of BoxFilter; Alg. 3 step 2), then at each
 * pixel the signed taps of the running sums at the pixel's own steps, combined
 * and divided by the product of the steps (Section 1.1, second step of
 * BoxFilter; Alg. 3 step 3; the signs and the weight w of Table 1; the shift
 * of eq. shifts), with the fixed-point load and the exact combination
 * described above.
 *   steps:       FP32 [planes][H][W].
 *   out:         FP32 [H][W] (nullable).
 *   out_num:     int64 [H][W] numerators, integer-step mode only (nullable):
 *                the exact sample sum for integer images, the fixed-point sum
 *                (value * 2^F) for float images.
 *   out_den:     int64 [H][W], prod_j s_j, integer-step mode only (nullable).
 *   dout_dsteps: FP32 [planes][H][W] (nullable, continuous steps): the
 *                derivative of out(x) with respect to each of the pixel's own
 *                step planes (right derivative where a step's phase is at a kink).
 *                The filter is local in its steps, so this is all the backward
 *                pass needs for the step gradient.
 *   G_save:      nullable; when given, the running sums are built there (layout
 *                of bsf_geometry) and ws needs only workspace_bytes_g_external.
 */
bsf_status bsf_filter_varying(const bsf_config *cfg, bsf_dtype dtype, const void *img,
                              int64_t H, int64_t W, int64_t pitch, const float *steps,
                              float *out, int64_t *out_num, int64_t *out_den, float *dout_dsteps,
                              void *G_save, void *ws, size_t ws_bytes, void *stream);

/*
 * The forward filter in its two stages; bsf_filter_varying is exactly
 * bsf_forward_prepare followed by bsf_forward_apply.
 *
 * bsf_forward_prepare: range check of the steps, choice of F (frac_bits), and
 *   the running sums of img into G (bsf_geometry layout; G == NULL puts them in
 *   the workspace).  ws: workspace_bytes (G == NULL) or
 *   workspace_bytes_g_external bytes.
 * bsf_forward_apply: the per-pixel taps of G with the pixel's steps,
 *   normalised (Section 1.1, second step of BoxFilter; Alg. 3 step 3).  G and
 *   ws must come from a bsf_forward_prepare on the same configuration, image
 *   size and workspace (ws holds F).  The steps may differ from the ones given
 *   to bsf_forward_prepare (one pre-integration serves several step fields, as
 *   the two banks of Alg. 2 do); the taps check their range and their
 *   fixed-point headroom at the stored F (BSF_FLAG_RANGE, BSF_FLAG_OVERFLOW;
 *   log2_bound keeps the preparing pass's value).  G == NULL reads the
 *   running sums from the workspace.
 */
bsf_status bsf_forward_prepare(const bsf_config *cfg, bsf_dtype dtype, const void *img, int64_t H,
                               int64_t W, int64_t pitch, const float *steps, void *G, void *ws,
                               size_t ws_bytes, void *stream);
bsf_status bsf_forward_apply(const bsf_config *cfg, bsf_dtype dtype, int64_t H, int64_t W,
                             const float *steps, const void *G, float *out, int64_t *out_num,
                             int64_t *out_den, float *dout_dsteps, void *ws, size_t ws_bytes,
                             void *stream);

/*
 * Adjoint of the forward filter with continuous steps (differentiation of a
 * loss through the filter; the paper does not differentiate its filter: this
 * is the transpose of the linear map of Section 1.1 in the image, and the
 * derivative of its continuous-step form in the steps).  Given the upstream
 * gradient gout [H][W] of a scalar loss L:
 *   grad_img   [H][W]          dL/df = K^T gout (nullable), computed as the scatter
 *                              of the pixel's tap patterns weighted in fixed point
 *                              by gout / prod s times the phase products, followed
 *                              by the transposed running sums (exact int64; the
 *                              rounding of those weights is the only error);
 *   grad_steps [planes][H][W]  dL/ds = gout * dout_dsteps (nullable; needs the
 *                              dout_dsteps saved by the forward call).
 * The image itself is not needed: the filter is linear in it.  ws: at least
 * bsf_backward_workspace_bytes bytes (status block, a window-sized int64
 * accumulator and the scan carries).
 */
size_t bsf_backward_workspace_bytes(const bsf_config *cfg, int64_t H, int64_t W);
bsf_status bsf_filter_backward(const bsf_config *cfg, int64_t H, int64_t W, const float *steps,
                               const float *gout, const float *dout_dsteps, float *grad_img,
                               float *grad_steps, void *ws, size_t ws_bytes, void *stream);

/*
 * Batched forward over B images of uneven sizes (FP32 images, one shared
 * configuration; the forward of bsf_filter_varying, i.e. the two steps of
 * BoxFilter in Section 1.1, applied to each image, with results identical to B
 * separate calls; the paper filters one image at a time).  descs is a host array of B entries:
 * img FP32 [H][pitch], steps FP32 [planes][H][W], out FP32 [H][W], all device
 * pointers owned by the caller; H = 0 or W = 0 skips an entry.  Each stage of
 * the path is one launch over the whole batch (a work list of (image, tile)
 * items), so small images do not leave the device idle.
 *
 * ws (device, >= bsf_batched_workspace_bytes for the same cfg and descs, and
 * the same tuning) holds a batch status block at its start (read with
 * bsf_read_device_status: flags OR-ed over the images, F_used the smallest F,
 * log2_bound the largest), the launch tables, and one single-image workspace
 * per image.  use_graph = 1 on a non-NULL stream that is not already capturing
 * records the launches into a HIP graph on the first call for a (device, cfg,
 * descs, ws, tuning) key and replays it on later calls with the same key
 * (a process-wide cache of up to 16 graphs, least recently used evicted);
 * otherwise the launches are enqueued directly.  Errors: BSF_E_INVALID for a
 * bad cfg, B < 0 or > 65536, a NULL pointer or pitch < W; BSF_E_WORKSPACE
 * when ws is too small; BSF_E_DEVICE when a launch or the capture fails.
 * bsf_batched_workspace_bytes returns 0 for invalid arguments.
 */
typedef struct {
    const float *img;
    const float *steps;
    float *out;
    int64_t H, W, pitch;
} bsf_image_desc;

size_t bsf_batched_workspace_bytes(const bsf_config *cfg, int32_t B, const bsf_image_desc *descs);
bsf_status bsf_filter_batched(const bsf_config *cfg, int32_t B, const bsf_image_desc *descs,
                              void *ws, size_t ws_bytes, void *stream, int32_t use_graph);

/*
 * Steps from a covariance field (Section 1.1, eq. cov and eq. geometry; the
 * minimum-kurtosis scales of Section 1.1 and Section 2.4), for a configuration of four
 * directions (any four that span the 2x2 covariances: those of Section 1.1,
 * those of Alg. 3).  cov: FP32 [3][H][W], the planes C11, C12, C22 of each
 * pixel's target covariance in pixel units (x = column, y = row).  sub is
 * subtracted from C11 and C22 first (Alg. 1 step 4 subtracts sigma^2 I).  Each
 * of the r copies of an order-r filter carries C / r.  The scales a_k of the box
 * spline with covariance sum_k (a_k^2 / 12) uhat_k uhat_k^T are, in lattice steps
 * s_k = a_k / |u_k|, the non-negative solution with the smallest Frobenius norm
 * of the kurtosis matrix sum_k a_k^4 uhat_k uhat_k^T; steps are floored at 1 and
 * written to steps [planes][H][W] (tied: one plane per direction; untied: the
 * same step on the r planes of a direction).  A covariance that is not
 * positive definite, not finite, or too elongated for the directions at its
 * orientation (beyond eq. boundE for those of Section 1.1) gets the scales
 * that keep the smallest A_k = s_k^2 / 12 largest, and BSF_FLAG_RANGE, as do
 * steps above max_step (clamped).  ws: at least 256 bytes (the status block).
 * BSF_E_UNSUPPORTED unless n_dirs == 4.
 */
bsf_status bsf_cov_to_steps(const bsf_config *cfg, const float *cov, int64_t H, int64_t W, float sub, float *steps,
                            void *ws, size_t ws_bytes, void *stream);

/*
 * Alg. 1 (Section 2.1, better accuracy): C = sigma^2 I + Delta C (eq. SigmaIso)
 * with sigma^2 half the bound of condition2 (with e(phi) of eq. boundE at each
 * pixel's orientation), taken as the smallest over the image because the
 * first pass is one global convolution (Alg. 1 steps 1-3: the box spline of
 * Section 1.1 with all four scales sqrt(6) sigma); then every pixel's
 * minimum-kurtosis scales for C - sigma^2 I (step 4, as bsf_cov_to_steps) filter
 * the first pass's output (step 5).  By Prop. 1 and Prop. 2 the result is one
 * space-variant filter whose kernel at each pixel has covariance C.
 *   cfg:  the four directions of Section 1.1 in any order, continuous steps;
 *         order r (the paper's BoxFilter is r = 1; each pass uses r copies);
 *         max_step bounds the steps of both passes.
 *   img:  FP32 [H][pitch];  cov: FP32 [3][H][W] (C11, C12, C22);  out: FP32 [H][W].
 *   ws:   at least bsf_alg1_workspace_bytes (status block first; it receives
 *         the flags of both passes, F_used of the second, and sigma^2 in an
 *         internal word).  The first pass's output is kept in FP32 in ws.
 * BSF_E_UNSUPPORTED for other directions or integer steps.
 */
size_t bsf_alg1_workspace_bytes(const bsf_config *cfg, int64_t H, int64_t W);
bsf_status bsf_filter_alg1(const bsf_config *cfg, const float *img, int64_t H, int64_t W, int64_t pitch,
                           const float *cov, float *out, void *ws, size_t ws_bytes, void *stream);

/*
 * Alg. 2 (Section 2.2, improved elongation): running sums of the image along
 * both four-direction sets, (1,0), (0,1), (1,1), (1,-1) of Section 1.1 and
 * (2,1), (1,2), (-1,2), (-2,1) of Alg. 3 (canonical sign (1,-2), (2,-1));
 * each pixel's orientation (the top eigenvector of its C) picks the set whose
 * axes lie nearer (the sectors S and S'; ties go to the first set), whose
 * minimum-kurtosis scales for C (bsf_cov_to_steps) give its finite difference on
 * that set's running sums.
 *   cfg:      order, tied, continuous steps, max_step, frac_bits, arith; its
 *             directions are not used.
 *   img:      [H][pitch] of dtype;  cov: FP32 [3][H][W];  out: FP32 [H][W].
 *   bank_out: nullable uint8 [H][W]: 0 or 1, the set each pixel used.
 *   ws:       at least bsf_alg2_workspace_bytes (status block first: flags of
 *             both sets, the smaller F).
 *   stream:   the second set's pass runs on a library-owned stream of the
 *             current device (created on the first call, default priority),
 *             forked from and joined back into this stream by events, so the
 *             call is ordered on `stream` as a whole and can be captured into a
 *             graph on it.
 */
size_t bsf_alg2_workspace_bytes(const bsf_config *cfg, int64_t H, int64_t W);
bsf_status bsf_filter_alg2(const bsf_config *cfg, bsf_dtype dtype, const void *img, int64_t H, int64_t W,
                           int64_t pitch, const float *cov, float *out, uint8_t *bank_out, void *ws, size_t ws_bytes,
                           void *stream);

/*
 * Alg. 3 (Section 2.3, the filter with the box spline of Table 1) as the paper
 * computes it, in FP64: running sums of the image along the four directions
 * (step 2), then at every pixel the 16 taps of Table 1 at the shifts of
 * eq. shifts, each one a value of the running sum between lattice points read
 * through eq. interpolation with the box spline of one lattice step along each
 * direction (the paper's beta'_b), weighted +-1 / prod a (step 3).  Generalised
 * to any four directions: tap t sits at x + sum_k ((s_k - 1)/2 - t_k s_k) u_k
 * (t_k bit k of t), with sign (-1)^(t_0 + .. + t_3) and weight 1 / prod s_k.  The
 * result equals the image convolved with the centred box spline of the pixel's
 * own continuous scales, sampled on the lattice (up to FP64 rounding).
 *   cfg:   four directions, any distinct canonical ones (the paper's are
 *          (2,1), (1,2), (1,-2), (2,-1) here: the signs do not change the
 *          result), order 1, tied, BSF_STEPS_REAL; max_step bounds the steps
 *          and sizes the LDS rectangle of running sums a tile works in
 *          (BSF_E_UNSUPPORTED when one pixel's rectangle, (floor(S sum|dx|) +
 *          sum|dx| + 1) (floor(S sum|dy|) + sum|dy| + 1) FP64 values at
 *          S = max_step, exceeds 148 KiB: S <= 21 for the paper's directions).
 *          frac_bits and arith are ignored.
 *   img:   [H][pitch] of dtype;  steps: FP32 [4][H][W], s_k in lattice steps
 *          along u_k (the paper's a_k / |u_k|), each in [1, max_step].
 *   out:   FP32 [H][W] and/or out_f64: FP64 [H][W] (at least one non-NULL).
 *   ws:    at least bsf_alg3_workspace_bytes (the status block).
 * A step that is NaN or outside [1, max_step] raises BSF_FLAG_RANGE and gives
 * that pixel NaN; a non-finite image sample raises BSF_FLAG_NONFINITE and
 * poisons the outputs of the tiles whose rectangles hold it.
 */
size_t bsf_alg3_workspace_bytes(const bsf_config *cfg, int64_t H, int64_t W);
bsf_status bsf_filter_alg3(const bsf_config *cfg, bsf_dtype dtype, const void *img, int64_t H, int64_t W,
                           int64_t pitch, const float *steps, float *out, double *out_f64, void *ws, size_t ws_bytes,
                           void *stream);

/*
 * Launch shapes (process-wide; set them before sizing workspaces and
 * launching work, not concurrently with other calls):
 *   gather_wx  width in pixels of one wavefront's block in the tied order-2
 *              four-direction gather: 8, 16, 32 or 64 (default 16);
 *   line_tl    steps per tile of the sheared running sums: a power of two in
 *              [16, 4096] (default 64).  Workspace sizes depend on it.
 * The result of every call is the same for every setting; only its speed
 * differs.  bsf_set_tuning returns BSF_E_INVALID for other values and keeps
 * the current ones; bsf_get_tuning writes the current values (NULL skips).
 */
bsf_status bsf_set_tuning(int32_t gather_wx, int32_t line_tl);
void bsf_get_tuning(int32_t *gather_wx, int32_t *line_tl);

/*
 * Tile of the tied order-2 gather along (1,0), (0,1), (1,1), (1,-1) (the
 * kernel that stages the running sums in LDS boxes): 8 (16 x 8 pixels, boxes
 * of up to 38 rows; the default) or 4 (16 x 4 pixels, boxes of up to 18 rows).
 * Tiles whose step range needs taller boxes read their taps from the window
 * directly, so the faster choice depends on how fast the steps vary; results
 * are the same.  Same rules as bsf_set_tuning; BSF_E_INVALID for other values.
 */
bsf_status bsf_set_box_tile(int32_t tile_h);
int32_t bsf_get_box_tile(void);

/*
 * Synchronises `stream`, then copies the status word from the workspace
 * (host outputs): *flags gets BSF_FLAG_* bits, *F_used the fixed-point bits of
 * the last forward call, *log2_bound the bound ceil(log2 max|f| + log2 max prod)
 * it was chosen from.  Any pointer may be NULL.  Clears the flags when clear != 0.
 */
bsf_status bsf_read_device_status(void *ws, void *stream, uint32_t *flags, int32_t *F_used,
                                  int32_t *log2_bound, int32_t clear);

const char *bsf_status_string(bsf_status s);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the forward
 * filter of bsf_filter_varying with the same arguments and results, but with
 * no workspace argument and no saved running sums.  The library keeps one
 * scratch array of BSF_NOALLOC_SCRATCH_BYTES in device memory per GPU (a
 * static device symbol, resident from the library's load until the process
 * ends; its address is looked up once per device, with that device current),
 * which holds the status words, the running-sum window and the scan carries.
 *   status_out: nullable device int32[4]; receives this call's flags
 *               (BSF_FLAG_*), F_used, log2_bound and 0.  The flags are cleared
 *               at the start of every call.
 * Returns BSF_E_WORKSPACE, before anything is enqueued, when the call needs more
 * than BSF_NOALLOC_SCRATCH_BYTES (bsf_geometry.workspace_bytes of the same
 * configuration and size), and BSF_E_DEVICE when the scratch address cannot be
 * looked up.  Calls nothing that allocates.  Every call on a GPU shares that
 * GPU's scratch array, which keeps the last call's contents: calls that overlap
 * in time on one GPU (other streams, other host threads) race and must not be
 * issued; calls in order on one stream are safe.  The stream's device must be
 * the current device.
 */
#define BSF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
bsf_status bsf_filter_varying_noalloc(const bsf_config *cfg, bsf_dtype dtype, const void *img, int64_t H,
                                      int64_t W, int64_t pitch, const float *steps, float *out, int64_t *out_num,
                                      int64_t *out_den, float *dout_dsteps, int32_t *status_out, void *stream);

/* Library version string, e.g. "bsf 0.1 gfx950". */
const char *bsf_version(void);

#ifdef __cplusplus
}
#endif
#endif
