/*
 * bsf_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU implementation of the space-variant box-spline filter of
 * K. N. Chaudhury and S. Sanyal, "Improvements on 'Fast space-variant elliptical
 * filtering using box splines'" (arXiv:1109.5114).  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or helper with the GPU library; the two meet only
 * through the seeded inputs and the documented array layouts.
 *
 * Everything here is written from the definitions, in the order the paper states
 * them, without blocking, fusion or reordering:
 *
 *   - the box distribution Box_a (Section 1.1): 1/a on the half-open interval
 *     (-a/2, a/2], zero elsewhere;
 *   - the box spline as the convolution of boxes laid along lattice directions
 *     (eq. boxSpline), here with one box per factor j along the integer
 *     direction u_j and a per-pixel length s_j(x) counted in lattice steps;
 *   - the pre-integration by running sums along each direction (Section 1.1,
 *     first step of BoxFilter; Alg. 3 step 2 gives the recursion form
 *     g(p) = f(p) + g(p - u));
 *   - the filter output as the image convolved with the pixel's own box spline,
 *     i.e. the space-variant filtering integral of Section 2.1.
 *
 * Readings of points the paper leaves open (each is listed in the design notes):
 *   - Continuous (non-integer) steps: each box of length s is integrated over the
 *     unit cells of the lattice line, w_s(i) = |[i-1/2, i+1/2] ^ [-s/2, s/2]|.
 *     This is the exact result of reading the running sum linearly between
 *     lattice points along u_j, the one-direction restriction of the box-spline
 *     interpolation of eq. interpolation.
 *   - Integer steps: the half-open Box_s used as a convolution kernel, so an
 *     even length puts its extra sample on the -u side.
 *   - Steps are in lattice steps along u_j, the running sums carry no sqrt(5)
 *     (or sqrt(2)) weight, and the output divides by the product of the steps.
 *   - The image is zero outside [0,W) x [0,H).
 *
 * Pins: every function below is checked by the "not gpu" tests against closed
 * forms (mass, mean, covariance, discrete-time Fourier transform), brute-force
 * enumeration on tiny inputs and textbook special cases.
 *
 * Layouts (shared with the GPU library only as documented interfaces):
 *   image  [H][pitch] row-major; x = column (0..W-1), y = row (0..H-1)
 *   dirs   n_dirs pairs (dx, dy), u = (dx, dy) in (column, row) units
 *   steps  [planes][H][W] float32; factor j (0 <= j < n_dirs*order) lies along
 *          direction j / order and reads plane (tied ? j / order : j)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { BSFO_U8 = 1, BSFO_U16 = 2, BSFO_F32 = 3, BSFO_F64 = 4 };
enum { BSFO_INT = 0, BSFO_REAL = 1 };

#define BSFO_MAX_FACTORS 16

/* Read one image sample as a double; zero outside the image (zero extension). */
static double img_at(const void *img, int dtype, long H, long W, long pitch, long x, long y)
{
    if (x < 0 || y < 0 || x >= W || y >= H) return 0.0;
    switch (dtype) {
    case BSFO_U8: return (double)((const uint8_t *)img)[y * pitch + x];
    case BSFO_U16: return (double)((const uint16_t *)img)[y * pitch + x];
    case BSFO_F64: return ((const double *)img)[y * pitch + x];
    default: return (double)((const float *)img)[y * pitch + x];
    }
}

static __int128 img_at_int(const void *img, int dtype, long H, long W, long pitch, long x, long y)
{
    if (x < 0 || y < 0 || x >= W || y >= H) return 0;
    if (dtype == BSFO_U8) return ((const uint8_t *)img)[y * pitch + x];
    return ((const uint16_t *)img)[y * pitch + x];
}

/* ------------------------------------------------------------------------- */
/* One box factor, as 1-D weights over lattice offsets i in [-h, h].          */
/* ------------------------------------------------------------------------- */

/* Continuous step s > 0: the length-s box integrated over the unit cell around
 * each lattice point, w_s(i) = |[i-1/2, i+1/2] ^ [-s/2, s/2]|.  Returns h. */
int bsfo_weights_real(double s, double *w, int cap)
{
    int h = (int)floor(s / 2.0 + 0.5) + 1;
    if (2 * h + 1 > cap) return -1;
    for (int i = -h; i <= h; i++) {
        double lo = fmax(i - 0.5, -s / 2.0);
        double hi = fmin(i + 0.5, s / 2.0);
        w[i + h] = hi > lo ? hi - lo : 0.0;
    }
    return h;
}

/* Derivative of w_s(i) with respect to s (right derivative at cell edges): the
 * two end cells, the ones holding +s/2 and -s/2, each gain 1/2. */
int bsfo_dweights_real(double s, double *dw, int cap)
{
    int h = (int)floor(s / 2.0 + 0.5) + 1;
    if (2 * h + 1 > cap) return -1;
    for (int i = -h; i <= h; i++) {
        double d = 0.0;
        if (i - 0.5 <= s / 2.0 && s / 2.0 < i + 0.5) d += 0.5;     /* cell holding +s/2 */
        if (i - 0.5 < -s / 2.0 && -s / 2.0 <= i + 0.5) d += 0.5;   /* cell holding -s/2 */
        dw[i + h] = d;
    }
    return h;
}

/* Integer step s >= 1: the unnormalised half-open box (-s/2, s/2] as a
 * convolution kernel.  Convolution places the sample at offset -t for each
 * t in the box, so the weight at offset i is 1 when -s/2 < -i <= s/2. */
int bsfo_weights_int(long s, int64_t *w, int cap)
{
    int h = (int)(s / 2) + 1;
    if (2 * h + 1 > cap) return -1;
    for (int i = -h; i <= h; i++) {
        long t = -i;
        /* -s/2 < t <= s/2, tested in integers as -s < 2t <= s */
        w[i + h] = (-s < 2 * t && 2 * t <= s) ? 1 : 0;
    }
    return h;
}

/* ------------------------------------------------------------------------- */
/* The 2-D kernel of one pixel: convolution of its line boxes (eq. boxSpline). */
/* ------------------------------------------------------------------------- */

typedef struct {
    long x0, y0, w, h;   /* kernel value for offset (x0 + a, y0 + b) at k[b*w + a] */
    double *k;
} kern_f64;

typedef struct {
    long x0, y0, w, h;
    int64_t *k;
} kern_i64;

/* Convolve a 2-D kernel with 1-D weights wt[-hw..hw] laid along (dx, dy). */
static void conv_line_f64(kern_f64 *K, int dx, int dy, const double *wt, int hw)
{
    long ex = (long)hw * labs(dx), ey = (long)hw * labs(dy);
    kern_f64 N;
    N.x0 = K->x0 - ex; N.y0 = K->y0 - ey;
    N.w = K->w + 2 * ex; N.h = K->h + 2 * ey;
    N.k = (double *)calloc((size_t)(N.w * N.h), sizeof(double));
    for (long b = 0; b < K->h; b++)
        for (long a = 0; a < K->w; a++) {
            double v = K->k[b * K->w + a];
            if (v == 0.0) continue;
            long px = K->x0 + a, py = K->y0 + b;
            for (int i = -hw; i <= hw; i++) {
                double wi = wt[i + hw];
                if (wi == 0.0) continue;
                long qx = px + (long)i * dx, qy = py + (long)i * dy;
                N.k[(qy - N.y0) * N.w + (qx - N.x0)] += wi * v;
            }
        }
    free(K->k);
    *K = N;
}

static void conv_line_i64(kern_i64 *K, int dx, int dy, const int64_t *wt, int hw)
{
    long ex = (long)hw * labs(dx), ey = (long)hw * labs(dy);
    kern_i64 N;
    N.x0 = K->x0 - ex; N.y0 = K->y0 - ey;
    N.w = K->w + 2 * ex; N.h = K->h + 2 * ey;
    N.k = (int64_t *)calloc((size_t)(N.w * N.h), sizeof(int64_t));
    for (long b = 0; b < K->h; b++)
        for (long a = 0; a < K->w; a++) {
            int64_t v = K->k[b * K->w + a];
            if (v == 0) continue;
            long px = K->x0 + a, py = K->y0 + b;
            for (int i = -hw; i <= hw; i++) {
                int64_t wi = wt[i + hw];
                if (wi == 0) continue;
                long qx = px + (long)i * dx, qy = py + (long)i * dy;
                N.k[(qy - N.y0) * N.w + (qx - N.x0)] += wi * v;
            }
        }
    free(K->k);
    *K = N;
}

/* Factor j's step at pixel index pidx. */
static double step_of(const float *steps, long HW, int order, int tied, int j, long pidx)
{
    int plane = tied ? j / order : j;
    return (double)steps[(long)plane * HW + pidx];
}

/* Unnormalised continuous-step kernel of one pixel: the convolution over all
 * factors of w_{s_j}.  If dplane >= 0, the factors reading that step plane are
 * differentiated one at a time and the results summed (product rule). */
static kern_f64 pixel_kernel_real(int M, const int *fdx, const int *fdy, const double *s,
                                  const int *fplane, int dplane)
{
    double *wt = (double *)malloc(sizeof(double) * 4096);
    kern_f64 acc = {0, 0, 1, 1, NULL};
    acc.k = (double *)calloc(1, sizeof(double));
    if (dplane < 0) {
        acc.k[0] = 1.0;
        for (int j = 0; j < M; j++) {
            int h = bsfo_weights_real(s[j], wt, 4096);
            conv_line_f64(&acc, fdx[j], fdy[j], wt, h);
        }
        free(wt);
        return acc;
    }
    /* sum over the differentiated factor d of (dw_d * prod_{j != d} w_j) */
    for (int d = 0; d < M; d++) {
        if (fplane[d] != dplane) continue;
        kern_f64 t = {0, 0, 1, 1, NULL};
        t.k = (double *)calloc(1, sizeof(double));
        t.k[0] = 1.0;
        for (int j = 0; j < M; j++) {
            int h = (j == d) ? bsfo_dweights_real(s[j], wt, 4096) : bsfo_weights_real(s[j], wt, 4096);
            conv_line_f64(&t, fdx[j], fdy[j], wt, h);
        }
        /* acc += t, on the union bounding box */
        long x0 = acc.x0 < t.x0 ? acc.x0 : t.x0, y0 = acc.y0 < t.y0 ? acc.y0 : t.y0;
        long x1 = (acc.x0 + acc.w > t.x0 + t.w) ? acc.x0 + acc.w : t.x0 + t.w;
        long y1 = (acc.y0 + acc.h > t.y0 + t.h) ? acc.y0 + acc.h : t.y0 + t.h;
        kern_f64 u = {x0, y0, x1 - x0, y1 - y0, NULL};
        u.k = (double *)calloc((size_t)(u.w * u.h), sizeof(double));
        for (long b = 0; b < acc.h; b++)
            for (long a = 0; a < acc.w; a++)
                u.k[(acc.y0 + b - y0) * u.w + (acc.x0 + a - x0)] += acc.k[b * acc.w + a];
        for (long b = 0; b < t.h; b++)
            for (long a = 0; a < t.w; a++)
                u.k[(t.y0 + b - y0) * u.w + (t.x0 + a - x0)] += t.k[b * t.w + a];
        free(acc.k); free(t.k);
        acc = u;
    }
    free(wt);
    return acc;
}

static kern_i64 pixel_kernel_int(int M, const int *fdx, const int *fdy, const long *s)
{
    int64_t *wt = (int64_t *)malloc(sizeof(int64_t) * 4096);
    kern_i64 acc = {0, 0, 1, 1, NULL};
    acc.k = (int64_t *)calloc(1, sizeof(int64_t));
    acc.k[0] = 1;
    for (int j = 0; j < M; j++) {
        int h = bsfo_weights_int(s[j], wt, 4096);
        conv_line_i64(&acc, fdx[j], fdy[j], wt, h);
    }
    free(wt);
    return acc;
}

/* Exported for the closed-form tests: the normalised continuous-step kernel
 * (divided by the product of the steps), written into k[h][w] with its origin
 * offset.  Call with k == NULL to get the extents only. */
int bsfo_kernel_real(int M, const int *fdx, const int *fdy, const double *s,
                     long *x0, long *y0, long *w, long *h, double *k, long cap)
{
    int fplane[BSFO_MAX_FACTORS];
    if (M < 1 || M > BSFO_MAX_FACTORS) return -1;
    for (int j = 0; j < M; j++) fplane[j] = j;
    kern_f64 K = pixel_kernel_real(M, fdx, fdy, s, fplane, -1);
    double den = 1.0;
    for (int j = 0; j < M; j++) den *= s[j];
    *x0 = K.x0; *y0 = K.y0; *w = K.w; *h = K.h;
    if (k) {
        if (K.w * K.h > cap) { free(K.k); return -2; }
        for (long i = 0; i < K.w * K.h; i++) k[i] = K.k[i] / den;
    }
    free(K.k);
    return 0;
}

/* Exported: the unnormalised integer-step kernel (sample counts). */
int bsfo_kernel_int(int M, const int *fdx, const int *fdy, const long *s,
                    long *x0, long *y0, long *w, long *h, int64_t *k, long cap)
{
    if (M < 1 || M > BSFO_MAX_FACTORS) return -1;
    kern_i64 K = pixel_kernel_int(M, fdx, fdy, s);
    *x0 = K.x0; *y0 = K.y0; *w = K.w; *h = K.h;
    if (k) {
        if (K.w * K.h > cap) { free(K.k); return -2; }
        memcpy(k, K.k, sizeof(int64_t) * (size_t)(K.w * K.h));
    }
    free(K.k);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The filter: each output pixel is the image convolved with its own kernel.  */
/* ------------------------------------------------------------------------- */

static int factor_layout(int n_dirs, const int *dirs, int order, int tied, int *fdx, int *fdy, int *fplane)
{
    int M = n_dirs * order;
    if (n_dirs < 1 || order < 1 || M > BSFO_MAX_FACTORS) return -1;
    for (int j = 0; j < M; j++) {
        fdx[j] = dirs[2 * (j / order)];
        fdy[j] = dirs[2 * (j / order) + 1];
        fplane[j] = tied ? j / order : j;
    }
    return M;
}

/*
 * out[n]  = filtered value at pixel pix[n] (or at every pixel when pix == NULL),
 *           in FP64: sum_p k(p) f(x + p) / prod_j s_j.
 * num/den = for integer images in integer-step mode, the exact numerator
 *           sum_p k(p) f(x + p) and denominator prod_j s_j (nullable).
 * Returns 0, or a negative code for bad arguments (non-integer step in integer
 * mode, step below 1).
 */
int bsfo_filter(const void *img, int dtype, long H, long W, long pitch,
                int n_dirs, const int *dirs, int order, int tied, int mode,
                const float *steps, long n_pix, const long *pix,
                double *out, int64_t *num, int64_t *den, int n_threads)
{
    int fdx[BSFO_MAX_FACTORS], fdy[BSFO_MAX_FACTORS], fplane[BSFO_MAX_FACTORS];
    int M = factor_layout(n_dirs, dirs, order, tied, fdx, fdy, fplane);
    if (M < 0) return -1;
    long HW = H * W;
    long count = pix ? n_pix : HW;
    int bad = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (long n = 0; n < count; n++) {
        long pidx = pix ? pix[n] : n;
        long x = pidx % W, y = pidx / W;
        double s[BSFO_MAX_FACTORS];
        for (int j = 0; j < M; j++) s[j] = step_of(steps, HW, order, tied, j, pidx);
        if (mode == BSFO_INT) {
            long si[BSFO_MAX_FACTORS];
            __int128 d = 1;
            for (int j = 0; j < M; j++) {
                if (s[j] < 1.0 || s[j] != floor(s[j])) { bad = 1; si[j] = 1; }
                else si[j] = (long)s[j];
                d *= si[j];
            }
            kern_i64 K = pixel_kernel_int(M, fdx, fdy, si);
            if (dtype == BSFO_F32 || dtype == BSFO_F64) {
                double acc = 0.0;
                for (long b = 0; b < K.h; b++)
                    for (long a = 0; a < K.w; a++) {
                        int64_t kv = K.k[b * K.w + a];
                        if (kv) acc += (double)kv * img_at(img, dtype, H, W, pitch, x + K.x0 + a, y + K.y0 + b);
                    }
                if (out) out[n] = acc / (double)d;
                if (num) num[n] = 0;
            } else {
                __int128 acc = 0;
                for (long b = 0; b < K.h; b++)
                    for (long a = 0; a < K.w; a++) {
                        int64_t kv = K.k[b * K.w + a];
                        if (kv) acc += (__int128)kv * img_at_int(img, dtype, H, W, pitch, x + K.x0 + a, y + K.y0 + b);
                    }
                if (out) out[n] = (double)acc / (double)d;
                if (num) num[n] = (int64_t)acc;
            }
            if (den) den[n] = (int64_t)d;
            free(K.k);
        } else {
            double d = 1.0;
            for (int j = 0; j < M; j++) {
                if (!(s[j] >= 1.0)) bad = 1;
                d *= s[j];
            }
            kern_f64 K = pixel_kernel_real(M, fdx, fdy, s, fplane, -1);
            double acc = 0.0;
            for (long b = 0; b < K.h; b++)
                for (long a = 0; a < K.w; a++) {
                    double kv = K.k[b * K.w + a];
                    if (kv != 0.0) acc += kv * img_at(img, dtype, H, W, pitch, x + K.x0 + a, y + K.y0 + b);
                }
            if (out) out[n] = acc / d;
            if (num) num[n] = 0;
            if (den) den[n] = 0;
            free(K.k);
        }
    }
    return bad ? -2 : 0;
}

/*
 * Gradients of L = sum_x gout(x) * out(x) for continuous steps, in FP64.
 *   grad_img[H][W]          = sum_x gout(x) k_x(p - x) / prod s(x)   (adjoint
 *                             of the space-variant filter; nullable)
 *   grad_steps[n*planes+q]  = gout(x) * d out(x) / d s_q(x) at pixel pix[n]
 *                             (or every pixel), plane-major per pixel
 *                             (nullable).  d out / d s = (sum_p dk(p) f(x+p) -
 *                             out * d prod s / d s) / prod s.
 * grad_img is produced by scattering every pixel's kernel, so it is meant for
 * small images or a window: only pixels x in [gx0,gx1) x [gy0,gy1) contribute.
 */
int bsfo_grad_real(const float *img, long H, long W, long pitch,
                   int n_dirs, const int *dirs, int order, int tied,
                   const float *steps, const float *gout,
                   double *grad_img, long gx0, long gx1, long gy0, long gy1,
                   long n_pix, const long *pix, double *grad_steps, int n_threads)
{
    int fdx[BSFO_MAX_FACTORS], fdy[BSFO_MAX_FACTORS], fplane[BSFO_MAX_FACTORS];
    int M = factor_layout(n_dirs, dirs, order, tied, fdx, fdy, fplane);
    if (M < 0) return -1;
    int planes = tied ? n_dirs : M;
    long HW = H * W;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    if (grad_img) {
        memset(grad_img, 0, sizeof(double) * (size_t)HW);
#pragma omp parallel
        {
            double *priv = (double *)calloc((size_t)HW, sizeof(double));
#pragma omp for schedule(dynamic, 4)
            for (long y = gy0; y < gy1; y++)
                for (long x = gx0; x < gx1; x++) {
                    long pidx = y * W + x;
                    double g = gout[pidx];
                    if (g == 0.0) continue;
                    double s[BSFO_MAX_FACTORS], d = 1.0;
                    for (int j = 0; j < M; j++) { s[j] = step_of(steps, HW, order, tied, j, pidx); d *= s[j]; }
                    kern_f64 K = pixel_kernel_real(M, fdx, fdy, s, fplane, -1);
                    for (long b = 0; b < K.h; b++)
                        for (long a = 0; a < K.w; a++) {
                            long px = x + K.x0 + a, py = y + K.y0 + b;
                            if (px < 0 || py < 0 || px >= W || py >= H) continue;
                            priv[py * W + px] += g * K.k[b * K.w + a] / d;
                        }
                    free(K.k);
                }
#pragma omp critical
            for (long i = 0; i < HW; i++) grad_img[i] += priv[i];
            free(priv);
        }
    }
    if (grad_steps) {
        long count = pix ? n_pix : HW;
#pragma omp parallel for schedule(dynamic, 8)
        for (long n = 0; n < count; n++) {
            long pidx = pix ? pix[n] : n;
            long x = pidx % W, y = pidx / W;
            double s[BSFO_MAX_FACTORS], d = 1.0;
            for (int j = 0; j < M; j++) { s[j] = step_of(steps, HW, order, tied, j, pidx); d *= s[j]; }
            kern_f64 K = pixel_kernel_real(M, fdx, fdy, s, fplane, -1);
            double acc = 0.0;
            for (long b = 0; b < K.h; b++)
                for (long a = 0; a < K.w; a++)
                    acc += K.k[b * K.w + a] * img_at(img, BSFO_F32, H, W, pitch, x + K.x0 + a, y + K.y0 + b);
            free(K.k);
            double outv = acc / d;
            for (int q = 0; q < planes; q++) {
                kern_f64 D = pixel_kernel_real(M, fdx, fdy, s, fplane, q);
                double dacc = 0.0;
                for (long b = 0; b < D.h; b++)
                    for (long a = 0; a < D.w; a++)
                        dacc += D.k[b * D.w + a] * img_at(img, BSFO_F32, H, W, pitch, x + D.x0 + a, y + D.y0 + b);
                free(D.k);
                /* d(prod s)/d s_q / prod s = (number of factors on plane q) / s_q */
                int mult = 0;
                double sq = 0.0;
                for (int j = 0; j < M; j++) if (fplane[j] == q) { mult++; sq = s[j]; }
                grad_steps[n * planes + q] = (double)gout[pidx] * (dacc / d - outv * (double)mult / sq);
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Pre-integration (running sums), in exact integers modulo 2^64.             */
/* ------------------------------------------------------------------------- */

/*
 * G = (S_{u_N})^order ... (S_{u_1})^order f_q on the window
 * rows [-pad_top, H + pad_bottom) x cols [-pad_left, W + pad_right), with
 * f_q = f (integer images) or f_q = nearest-even integer of f * 2^F (float
 * images), zero outside the image.  Each running sum follows the recursion of
 * Alg. 3 step 2, g(p) = f(p) + g(p - u), started at zero where a line enters the
 * window; the passes run in the order the directions are given, and the
 * arithmetic wraps modulo 2^64.  G is stored [Hp][Wp], with G[(y + pad_top) *
 * Wp + (x + pad_left)] holding the value at (x, y).
 */
int bsfo_preintegrate(const void *img, int dtype, long H, long W, long pitch,
                      int n_dirs, const int *dirs, int order, int F,
                      long pad_top, long pad_bottom, long pad_left, long pad_right,
                      uint64_t *G)
{
    long Hp = H + pad_top + pad_bottom, Wp = W + pad_left + pad_right;
    for (long yy = 0; yy < Hp; yy++)
        for (long xx = 0; xx < Wp; xx++) {
            long x = xx - pad_left, y = yy - pad_top;
            uint64_t q = 0;
            if (x >= 0 && y >= 0 && x < W && y < H) {
                if (dtype == BSFO_F32) {
                    double v = ldexp((double)((const float *)img)[y * pitch + x], F);
                    q = (uint64_t)(int64_t)nearbyint(v);
                } else {
                    q = (uint64_t)(int64_t)img_at_int(img, dtype, H, W, pitch, x, y);
                }
            }
            G[yy * Wp + xx] = q;
        }
    for (int k = 0; k < n_dirs; k++) {
        int dx = dirs[2 * k], dy = dirs[2 * k + 1];
        for (int rep = 0; rep < order; rep++) {
            /* Visit points so that p - u is always finished before p: order the
             * rows along dy and, within a row (dy == 0), the columns along dx. */
            for (long t = 0; t < Hp; t++) {
                long yy = dy >= 0 ? t : Hp - 1 - t;
                for (long c = 0; c < Wp; c++) {
                    long xx = dx >= 0 ? c : Wp - 1 - c;
                    long px = xx - dx, py = yy - dy;
                    if (px < 0 || py < 0 || px >= Wp || py >= Hp) continue;
                    G[yy * Wp + xx] += G[py * Wp + px];
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Scales from a covariance: eq. cov gives the covariance of a box spline as   */
/* sum_k (a_k^2 / 12) u_k u_k^T over its unit directions, i.e. sum_k          */
/* (s_k^2 / 12) u_k u_k^T with s_k counted in lattice steps along the integer  */
/* vector u_k; four directions leave one free parameter, fixed by the minimum  */
/* kurtosis: the Frobenius norm of sum_k a_k^4 uhat_k uhat_k^T (the matrix of  */
/* Section 2.4 for the directions of Alg. 3, the same construction for the     */
/* directions of Section 1.1), which is sum_k A_k^2 |u_k|^2 u_k u_k^T up to a  */
/* constant, A_k = s_k^2 / 12.                                                 */
/* ------------------------------------------------------------------------- */

static double frob2_kurtosis(const int *dirs, const double A[4])
{
    double k11 = 0, k12 = 0, k22 = 0;
    for (int k = 0; k < 4; k++) {
        double ux = dirs[2 * k], uy = dirs[2 * k + 1], n2 = ux * ux + uy * uy;
        k11 += A[k] * A[k] * n2 * ux * ux;
        k12 += A[k] * A[k] * n2 * ux * uy;
        k22 += A[k] * A[k] * n2 * uy * uy;
    }
    return k11 * k11 + 2 * k12 * k12 + k22 * k22;
}

static double det3(double a[3][3])
{
    return a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1])
         - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0])
         + a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
}

/* Steps s[4] (lattice steps, one per direction, the same for the `order`
 * copies of a direction, each copy carrying C / order) of the minimum-kurtosis
 * box spline along the four integer directions dirs with covariance C.
 * Returns 0, or 1 when no non-negative scales reproduce C (the elongation
 * exceeds what the directions allow): then the choice maximising the smallest
 * A_k is taken, negative parts dropped.  Steps are floored at 1 (a box of one
 * lattice step is the identity).  -1 for degenerate directions. */
int bsfo_cov_to_steps(const int *dirs, int order, double c11, double c12, double c22, double *steps)
{
    double c[3] = {c11 / order, c12 / order, c22 / order};
    double m[3][4];
    for (int k = 0; k < 4; k++) {
        double ux = dirs[2 * k], uy = dirs[2 * k + 1];
        m[0][k] = ux * ux;
        m[1][k] = ux * uy;
        m[2][k] = uy * uy;
    }
    /* null vector by cofactors, and a particular solution from the best-
     * conditioned three columns */
    double n[4], A0[4] = {0, 0, 0, 0}, best = 0;
    int skip_best = -1;
    for (int k = 0; k < 4; k++) {
        double sub[3][3];
        for (int r = 0; r < 3; r++)
            for (int q = 0, cc = 0; q < 4; q++)
                if (q != k) sub[r][cc++] = m[r][q];
        double d = det3(sub);
        n[k] = (k % 2 ? -1.0 : 1.0) * d;
        if (fabs(d) > best) {
            best = fabs(d);
            skip_best = k;
        }
    }
    if (skip_best < 0) return -1;
    {
        /* Cramer's rule on the columns other than skip_best */
        int cols[3], cc = 0;
        double sub[3][3];
        for (int q = 0; q < 4; q++)
            if (q != skip_best) cols[cc++] = q;
        for (int r = 0; r < 3; r++)
            for (int q = 0; q < 3; q++) sub[r][q] = m[r][cols[q]];
        double d = det3(sub);
        for (int q = 0; q < 3; q++) {
            double t[3][3];
            memcpy(t, sub, sizeof(t));
            for (int r = 0; r < 3; r++) t[r][q] = c[r];
            A0[cols[q]] = det3(t) / d;
        }
    }
    /* feasible t: A0 + t n >= 0 */
    double lo = -INFINITY, hi = INFINITY;
    int infeasible = 0;
    for (int k = 0; k < 4; k++) {
        if (n[k] > 0) lo = fmax(lo, -A0[k] / n[k]);
        else if (n[k] < 0) hi = fmin(hi, -A0[k] / n[k]);
        else if (A0[k] < 0) infeasible = 1;
    }
    double A[4], tbest;
    if (!infeasible && lo <= hi) {
        /* dense scan of the quartic, then golden-section refinement */
        const int N = 4096;
        double fbest = INFINITY;
        int ibest = 0;
        for (int i = 0; i <= N; i++) {
            double t = lo + (hi - lo) * i / N;
            for (int k = 0; k < 4; k++) A[k] = A0[k] + t * n[k];
            double f = frob2_kurtosis(dirs, A);
            if (f < fbest) {
                fbest = f;
                ibest = i;
            }
        }
        double a = lo + (hi - lo) * (ibest > 0 ? ibest - 1 : 0) / N;
        double b = lo + (hi - lo) * (ibest < N ? ibest + 1 : N) / N;
        const double g = (sqrt(5.0) - 1.0) / 2.0;
        for (int it = 0; it < 200; it++) {
            double t1 = b - g * (b - a), t2 = a + g * (b - a), f1, f2;
            for (int k = 0; k < 4; k++) A[k] = A0[k] + t1 * n[k];
            f1 = frob2_kurtosis(dirs, A);
            for (int k = 0; k < 4; k++) A[k] = A0[k] + t2 * n[k];
            f2 = frob2_kurtosis(dirs, A);
            if (f1 <= f2) b = t2;
            else a = t1;
        }
        tbest = 0.5 * (a + b);
        for (int k = 0; k < 4; k++) A[k] = A0[k] + tbest * n[k];
        if (frob2_kurtosis(dirs, A) > fbest) tbest = lo + (hi - lo) * ibest / N;
        tbest = fmin(fmax(tbest, lo), hi);
    } else {
        /* maximise min_k A_k(t): the best of the crossings of two lines */
        infeasible = 1;
        double vbest = -INFINITY;
        tbest = 0;
        for (int i = 0; i < 4; i++)
            for (int j = i + 1; j < 4; j++) {
                if (n[i] == n[j]) continue;
                double t = (A0[j] - A0[i]) / (n[i] - n[j]), v = INFINITY;
                for (int k = 0; k < 4; k++) v = fmin(v, A0[k] + t * n[k]);
                if (v > vbest) {
                    vbest = v;
                    tbest = t;
                }
            }
    }
    for (int k = 0; k < 4; k++) {
        double Ak = fmax(A0[k] + tbest * n[k], 0.0);
        steps[k] = fmax(sqrt(12.0 * Ak), 1.0);
    }
    return infeasible;
}

/* Orientation of C: the angle in [0, pi) of its top eigenvector (Section 1.1). */
double bsfo_orientation(double c11, double c12, double c22)
{
    double phi = 0.5 * atan2(2.0 * c12, c11 - c22);
    if (phi < 0) phi += M_PI;
    if (phi >= M_PI) phi -= M_PI;
    return phi;
}

/* eq. boundE: the largest elongation of the box spline of Section 1.1 at
 * orientation phi; infinite along its axes. */
double bsfo_elongation_bound(double phi)
{
    double sn = sin(phi), cs = cos(phi);
    if (sn == 0.0 || cs == 0.0) return INFINITY;
    double t = fabs(sn / cs - cs / sn) / 2.0;
    double q = sqrt(1.0 + t * t);
    if (1.0 + t - q <= 0.0) return INFINITY;
    return (1.0 + t + q) / (1.0 + t - q);
}

/* condition2: sigma^2 below this keeps C - sigma^2 I a covariance the
 * box spline of Section 1.1 can reach at C's orientation. */
double bsfo_condition2_bound(double c11, double c12, double c22)
{
    double e = bsfo_elongation_bound(bsfo_orientation(c11, c12, c22));
    double f = isinf(e) ? 1.0 : (e + 1.0) / (e - 1.0);
    return 0.5 * (c11 + c22 - f * sqrt((c11 - c22) * (c11 - c22) + 4.0 * c12 * c12));
}

/* Sector of Alg. 2: 0 when phi is closer (modulo pi) to an axis of the first
 * bank, 0, 45, 90, 135 degrees, than to one of the second, atan(1/2),
 * atan(2), pi - atan(2), pi - atan(1/2); ties go to the first. */
int bsfo_bank_of(double phi)
{
    const double a1[4] = {0.0, M_PI / 4, M_PI / 2, 3 * M_PI / 4};
    const double a2[4] = {atan(0.5), atan(2.0), M_PI - atan(2.0), M_PI - atan(0.5)};
    double d1 = INFINITY, d2 = INFINITY;
    for (int k = 0; k < 4; k++) {
        double d = fabs(phi - a1[k]);
        d1 = fmin(d1, fmin(d, M_PI - d));
        d = fabs(phi - a2[k]);
        d2 = fmin(d2, fmin(d, M_PI - d));
    }
    return d2 < d1 ? 1 : 0;
}

/* The same over a field of n pixels: cov = [3][n] (C11, C12, C22), sub is
 * subtracted from the diagonal first (Alg. 1 step 4); steps = [4][n]; flags[n]
 * gets the return value of bsfo_cov_to_steps. */
int bsfo_cov_to_steps_field(const int *dirs, int order, long n, const float *cov, double sub, double *steps,
                            int *flags)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long i = 0; i < n; i++) {
        double s[4];
        int r = bsfo_cov_to_steps(dirs, order, (double)cov[i] - sub, (double)cov[n + i], (double)cov[2 * n + i] - sub, s);
        if (r < 0) bad = 1;
        flags[i] = r;
        for (int k = 0; k < 4; k++) steps[k * n + i] = s[k];
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Alg. 3 as printed, with eq. interpolation: the running sum g of the image  */
/* along four directions is read between lattice points as                    */
/*     F(p) = sum_m g(m) beta_b(p - m),                                        */
/* beta_b the box spline of one lattice step along each of the directions (the */
/* paper's beta'_b with scales sqrt(5), the length of those lattice vectors),  */
/* and the 2^4 signed taps of Table 1 sit at the real positions                */
/*     p = x + sum_k ((s_k - 1)/2 - eps_k s_k) u_k                             */
/* (the first is x + tau of eq. shifts), with w = 1 / prod s_k.               */
/* ------------------------------------------------------------------------- */

/* Area of the intersection of two convex quadrilaterals, each given by its
 * corners in counter-clockwise order: the corners of each inside the other
 * and the crossings of their edges, ordered by angle about their mean, then
 * the shoelace formula. */
static int inside_convex(const double Q[4][2], double x, double y)
{
    for (int i = 0; i < 4; i++) {
        const double *a = Q[i], *b = Q[(i + 1) % 4];
        double cr = (b[0] - a[0]) * (y - a[1]) - (b[1] - a[1]) * (x - a[0]);
        if (cr < -1e-12) return 0;
    }
    return 1;
}

static double area_of_intersection(const double P[4][2], const double Q[4][2])
{
    double pts[32][2];
    int n = 0;
    for (int i = 0; i < 4; i++) {
        if (inside_convex(Q, P[i][0], P[i][1])) { pts[n][0] = P[i][0]; pts[n][1] = P[i][1]; n++; }
        if (inside_convex(P, Q[i][0], Q[i][1])) { pts[n][0] = Q[i][0]; pts[n][1] = Q[i][1]; n++; }
    }
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            const double *a = P[i], *b = P[(i + 1) % 4], *c = Q[j], *d = Q[(j + 1) % 4];
            double rx = b[0] - a[0], ry = b[1] - a[1], sx = d[0] - c[0], sy = d[1] - c[1];
            double den = rx * sy - ry * sx;
            if (fabs(den) < 1e-15) continue;
            double t = ((c[0] - a[0]) * sy - (c[1] - a[1]) * sx) / den;
            double u = ((c[0] - a[0]) * ry - (c[1] - a[1]) * rx) / den;
            if (t < 0 || t > 1 || u < 0 || u > 1) continue;
            pts[n][0] = a[0] + t * rx;
            pts[n][1] = a[1] + t * ry;
            n++;
        }
    if (n < 3) return 0.0;
    double cx = 0, cy = 0;
    for (int i = 0; i < n; i++) { cx += pts[i][0]; cy += pts[i][1]; }
    cx /= n;
    cy /= n;
    double ang[32];
    for (int i = 0; i < n; i++) ang[i] = atan2(pts[i][1] - cy, pts[i][0] - cx);
    for (int i = 1; i < n; i++)  /* insertion sort by angle */
        for (int j = i; j > 0 && ang[j] < ang[j - 1]; j--) {
            double ta = ang[j]; ang[j] = ang[j - 1]; ang[j - 1] = ta;
            double tx = pts[j][0], ty = pts[j][1];
            pts[j][0] = pts[j - 1][0]; pts[j][1] = pts[j - 1][1];
            pts[j - 1][0] = tx; pts[j - 1][1] = ty;
        }
    double a2 = 0.0;
    for (int i = 0; i < n; i++) {
        int k = (i + 1) % n;
        a2 += pts[i][0] * pts[k][1] - pts[k][0] * pts[i][1];
    }
    return 0.5 * fabs(a2);
}

/* The parallelogram {a u + b v : |a|, |b| <= 1/2} centred at (cx, cy), corners
 * counter-clockwise. */
static void parallelogram(const int *u, const int *v, double cx, double cy, double Q[4][2])
{
    const double s[4][2] = {{-0.5, -0.5}, {0.5, -0.5}, {0.5, 0.5}, {-0.5, 0.5}};
    for (int i = 0; i < 4; i++) {
        Q[i][0] = cx + s[i][0] * u[0] + s[i][1] * v[0];
        Q[i][1] = cy + s[i][0] * u[1] + s[i][1] * v[1];
    }
    if ((double)u[0] * v[1] - (double)u[1] * v[0] < 0) {  /* make it counter-clockwise */
        for (int i = 0; i < 2; i++) {
            double tx = Q[i][0], ty = Q[i][1];
            Q[i][0] = Q[3 - i][0]; Q[i][1] = Q[3 - i][1];
            Q[3 - i][0] = tx; Q[3 - i][1] = ty;
        }
    }
}

/* beta_b at (x, y) for the four integer directions dirs: the box splines of
 * the pairs (u0, u1) and (u2, u3) are their parallelograms with unit mass, so
 * beta_b(p) = |P01 ^ (p - P23)| / (|det(u0, u1)| |det(u2, u3)|) (P23 is
 * symmetric about 0, so p - P23 = p + P23). */
double bsfo_unit_box_spline(const int *dirs, double x, double y)
{
    double P[4][2], Q[4][2];
    parallelogram(dirs + 0, dirs + 2, 0.0, 0.0, P);
    parallelogram(dirs + 4, dirs + 6, x, y, Q);
    double d01 = fabs((double)dirs[0] * dirs[3] - (double)dirs[1] * dirs[2]);
    double d23 = fabs((double)dirs[4] * dirs[7] - (double)dirs[5] * dirs[6]);
    return area_of_intersection(P, Q) / (d01 * d23);
}

/* Alg. 3 at pixels pix (or at every pixel) of a float image [H][W] (FP64 out).
 *
 * dirs: four canonical integer directions (dy > 0, or dy == 0 and dx > 0);
 * steps [4][H][W]: the length s_k >= 1 of direction k's box at each pixel, in
 * lattice steps along u_k (the paper's a_k / sqrt(5) for its directions).
 *
 * Step 2, the recursions g <- g + g(. - u_k) one direction after another, runs
 * over a rectangle of lattice points holding every point the interpolation
 * reads together with every point those depend on: all directions point into
 * y >= 0, so a point (x, y) depends only on points (x', y') with y' <= y and
 * x' <= x + c (y - y'), c = max ceil(-dx/dy) over directions with dx < 0, and
 * the sums vanish left of x = -c y.  No pass is cut short, so g is the running
 * sum of the zero-extended image, accumulated in long double.  Those sums grow
 * like the fourth power of the region's side (about 1e12 max|f| for a 2048^2
 * frame), and their rounding with them: large frames are compared block by
 * block, on crops that hold each block's footprints (the result at a pixel
 * depends on nothing else).
 *
 * Step 3 takes the 16 taps of Table 1 in the order of dirs (bit k of the tap
 * index moves the tap by -s_k u_k, the sign is (-1)^(number of set bits)), the
 * shift of eq. shifts, generalised to tau = (1/2) sum_k (s_k - 1) u_k (the
 * paper's -3 in tau_2 is -(1/2) sum_k u_k for its directions: each running sum
 * read through a unit box is displaced by half a step), and w = 1 / prod s_k
 * (the sqrt(5) weights of the recursions and of a_k cancel).  Returns 0, -1
 * for directions outside the accepted half-plane, -2 for a step below 1. */
int bsfo_alg3(const float *img, long H, long W, const int *dirs, const float *steps, long n_pix, const long *pix,
              double *out)
{
    const long HW = H * W, count = pix ? n_pix : HW;
    long c = 0;
    double ex = 0, ey = 0;
    for (int k = 0; k < 4; k++) {
        int dx = dirs[2 * k], dy = dirs[2 * k + 1];
        if (dy < 0 || (dy == 0 && dx <= 0)) return -1;
        if (dx < 0) {
            long slope = (-dx + dy - 1) / dy; /* ceil(-dx / dy) */
            if (slope > c) c = slope;
        }
        ex += 0.5 * abs(dx);
        ey += 0.5 * dy;
    }
    /* the lattice points the interpolation reads: a bounding box over all taps */
    long qx_lo = 0, qx_hi = W - 1, qy_hi = H - 1;
    for (long n = 0; n < count; n++) {
        long pidx = pix ? pix[n] : n, x = pidx % W, y = pidx / W;
        for (int k = 0; k < 4; k++)
            if (!(steps[k * HW + pidx] >= 1.0f)) return -2;
        for (int e = 0; e < 16; e++) {
            double qx = x, qy = y;
            for (int k = 0; k < 4; k++) {
                double s = steps[k * HW + pidx], t = (s - 1.0) / 2.0 - ((e >> k) & 1) * s;
                qx += t * dirs[2 * k];
                qy += t * dirs[2 * k + 1];
            }
            long xl = (long)floor(qx - ex) - 1, xh = (long)ceil(qx + ex) + 1, yh = (long)ceil(qy + ey) + 1;
            if (xl < qx_lo) qx_lo = xl;
            if (xh > qx_hi) qx_hi = xh;
            if (yh > qy_hi) qy_hi = yh;
        }
    }
    const long y1 = qy_hi, x0 = (qx_lo < -c * y1 - 1 ? qx_lo : -c * y1 - 1), x1 = qx_hi + c * y1;
    const long RW = x1 - x0 + 1, RH = y1 + 1;
    long double *g = calloc((size_t)RW * RH, sizeof(long double));
    if (!g) return -3;
    for (long y = 0; y < H; y++)
        for (long x = 0; x < W; x++) g[y * RW + (x - x0)] = img[y * W + x];
    /* step 2: g_k(m) = g_{k-1}(m) + g_k(m - u_k), rows ascending, columns ascending */
    for (int k = 0; k < 4; k++) {
        const long dx = dirs[2 * k], dy = dirs[2 * k + 1];
        for (long y = 0; y < RH; y++)
            for (long x = x0; x <= x1; x++) {
                long px = x - dx, py = y - dy;
                if (px < x0 || px > x1 || py < 0) continue; /* zero there */
                g[y * RW + (x - x0)] += g[py * RW + (px - x0)];
            }
    }
    /* step 3 */
#pragma omp parallel for schedule(dynamic, 16)
    for (long n = 0; n < count; n++) {
        long pidx = pix ? pix[n] : n, x = pidx % W, y = pidx / W;
        double s[4], den = 1.0;
        for (int k = 0; k < 4; k++) {
            s[k] = steps[k * HW + pidx];
            den *= s[k];
        }
        long double acc = 0.0L;
        for (int e = 0; e < 16; e++) {
            double qx = x, qy = y;
            for (int k = 0; k < 4; k++) {
                double t = (s[k] - 1.0) / 2.0 - ((e >> k) & 1) * s[k];
                qx += t * dirs[2 * k];
                qy += t * dirs[2 * k + 1];
            }
            /* eq. interpolation: F(q) = sum over |m - q| <= reach of g(m) beta_b(q - m) */
            long double F = 0.0L;
            for (long my = (long)ceil(qy - ey); my <= (long)floor(qy + ey); my++)
                for (long mx = (long)ceil(qx - ex); mx <= (long)floor(qx + ex); mx++) {
                    if (my < 0 || mx < x0) continue; /* g vanishes there */
                    double wgt = bsfo_unit_box_spline(dirs, qx - mx, qy - my);
                    if (wgt != 0.0) F += g[my * RW + (mx - x0)] * (long double)wgt;
                }
            acc += (__builtin_popcount(e) & 1) ? -F : F;
        }
        out[n] = (double)(acc / den);
    }
    free(g);
    return 0;
}

int bsfo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
