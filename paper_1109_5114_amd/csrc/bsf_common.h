// Internal definitions shared by the libbsf translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bsf.h"

namespace bsf {

// Status block at the start of every workspace (32-bit words).
enum StatusWord : int {
    ST_FLAGS = 0,      // sticky BSF_FLAG_* bits
    ST_F_USED = 1,     // fixed-point bits used by the last forward pass
    ST_LOG2_BOUND = 2, // ceil(log2 max|f_q| bound exponent) the choice came from
    ST_EP_MAX = 3,     // scratch: max over pixels of ceil(log2 prod of box lengths)
    ST_FABS_BITS = 4,  // scratch: float bits of max |f|
    ST_F_REQUEST = 5,  // requested F (-1 = auto)
    ST_EF = 6,         // ceil(log2 max|f|) of the image the window was built from
    ST_ARITH = 7,      // arithmetic of the window (bsf_arith)
    ST_WORDS = 64
};
constexpr size_t kStatusBytes = 256;
constexpr size_t kAlign = 256;

inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// Input kinds for the first running-sum pass.
enum SrcKind : int { SRC_WINDOW = 0, SRC_F32 = 1, SRC_U8 = 2, SRC_U16 = 3 };

// Host-side plan of one (config, H, W).
struct Plan {
    int n_dirs, order, M, tied, mode, arith, planes;
    int dx[BSF_MAX_DIRS], dy[BSF_MAX_DIRS];
    float max_step;
    int R_max;                  // floor((max_step - 1) / 2)
    int64_t H, W;
    int64_t pad_top, pad_bottom, pad_left, pad_right, Hp, Wp;
    size_t g_bytes;
    size_t scan_aux_bytes;      // carries of the line scans
};

// Source image description for the first pass.
struct Src {
    const void *img;
    int kind;          // SrcKind
    int64_t H, W, pitch;
    int64_t pad_top, pad_left;
};

bsf_status make_plan(const bsf_config *cfg, int64_t H, int64_t W, Plan *p);

// Launch-shape choices (set by the tuner through bsf_set_tuning).
struct Tuning {
    int gather_wx;   // width in pixels of the wavefront block of the tied order-2 gather (8, 16, 32, 64)
    int line_tl;     // steps per line tile of the sheared scans (power of two, 16 .. 4096)
    int box_h;       // tile height of the cluster-box tied order-2 gather (4 or 8)
};
const Tuning &tuning();

// Sheared line tiles of a running sum along (dx, dy), dy != 0.
struct LineGeom {
    int dx, dy, ay, tl;
    int64_t Hp, Wp;
    int64_t T;         // steps per residue class (rows / |dy|, rounded up)
    int64_t c_lo;      // start column of the first line
    int64_t n_groups;  // groups of 64 lines
    int64_t n_chunks;  // chunks of tl steps
};
LineGeom line_geom(int dx, int dy, int64_t Hp, int64_t Wp, int tl);

// One image's share of a running-sum pass, for batched launches.
struct ScanJob {
    void *G;
    void *aux;
    const int32_t *status;
    Src src;
    LineGeom g;
    int64_t Hp, Wp;
    int dir;  // row passes: +1 forward, -1 reversed
};

// Workgroups are handed to the 8 XCDs of the device in turn, each XCD with its
// own L2.  Block b of a grid padded to a multiple of 8 takes item
// (b % 8) * per + b / 8 (per = ceil(n / 8)): every XCD works through one
// contiguous range of items, so neighbouring tiles, whose boxes of the window
// overlap, meet in the same L2.  Items >= n are idle.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_item(int64_t b, int64_t n) {
    const int64_t per = (n + kXcds - 1) / kXcds;
    return (b % kXcds) * per + b / kXcds;
}
inline int64_t xcd_grid(int64_t n) { return (n + kXcds - 1) / kXcds * kXcds; }

// Job b of a batched launch owns the work items [prefix[b], prefix[b+1]).
__device__ __forceinline__ int find_job(const int64_t *__restrict__ prefix, int B, int64_t item) {
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Running sums on the window (scan.hip).  G is int64 (exact) or double (fp64).
size_t scan_aux_bytes(const Plan &p);
// One pass over a batch: jobs and the three work prefixes (rows / tiles /
// line groups) are device tables; totals are the last prefix entries.
bsf_status run_pass_batch(int arith, int order, int src_kind, int dx, int dy, const ScanJob *jobs,
                          const int64_t *prefix_items, int64_t total_items, const int64_t *prefix_groups,
                          int64_t total_groups, int B, hipStream_t st);
bsf_status run_preintegrate(const Plan &p, const Src &src, void *G, void *aux, const int32_t *status,
                            hipStream_t st);
// Reverse (transposed) running sums on the window, last direction first.
bsf_status run_preintegrate_transpose(const Plan &p, void *G, void *aux, const int32_t *status, hipStream_t st);
// Inclusive 2-D prefix sum, in place, of a dense int64 [rows][cols] array
// (rows <= Hp and cols <= Wp of a plan whose scan_aux_bytes sized aux).
bsf_status run_prefix2d(int64_t *D, int64_t rows, int64_t cols, void *aux, const int32_t *status, hipStream_t st);

// Per-pixel taps (gather.hip).
struct GatherArgs {
    const void *G;
    int64_t Wp, pad_top, pad_left;
    int64_t H, W;
    const float *steps;     // [planes][H][W]
    float *out;             // nullable
    float *dsteps;          // nullable: d out / d step, [planes][H][W] (continuous steps)
    int64_t *out_num;       // nullable
    int64_t *out_den;       // nullable
    const int32_t *status;  // F at status[ST_F_USED]
    float max_step;
    int M, order, tied, n_dirs, mode;
    int32_t off[BSF_MAX_FACTORS];    // window offset (elements) of one lattice step along factor j
    int32_t plane[BSF_MAX_FACTORS];  // step plane of factor j
    // Four directions that are exactly (1,0), (0,1), (1,1), (1,-1) in some
    // order: canon = 1; exactly (2,1), (1,2), (1,-2), (2,-1): canon = 2; then
    // canon_plane[k] is the step plane of the k-th of those (the cluster-box
    // kernels address taps in that fixed frame).  Otherwise canon = 0.
    int32_t canon;
    int32_t canon_plane[4];
    // nullable: only pixels whose sel entry equals sel_id are written (the
    // sectors of Alg. 2 filter their pixels from their own running sums)
    const uint8_t *sel;
    int32_t sel_id;
};
bsf_status run_gather(const Plan &p, const GatherArgs &a, hipStream_t st);
// The tied order-2 cluster-box gather of one image in the frame of Table 1's
// directions (canon = 2), launched on the given grid (gather_f1.hip).
bsf_status launch_gather_f1(const GatherArgs &a, dim3 grid, dim3 block, hipStream_t st);
// Arguments of the gather for one image (bsf_api.hip).
GatherArgs gather_args(const Plan &p, const void *G, const float *steps, float *out, int64_t *num, int64_t *den,
                       float *dsteps, const int32_t *status);
// Single-image workspace: [status][G when internal][scan carries].
size_t ws_bytes_for(const Plan &p, bool g_internal);
// Batched gather: table / prefix are device arrays over B images; prefix has
// the cumulative pixel-tile counts gather_tiles() gives per image.
int64_t gather_tiles(const Plan &p, const GatherArgs &a);
// Images with equal variants run the same gather kernel and tile shape.
int gather_variant(const Plan &p, const GatherArgs &a);
bsf_status run_gather_batch(const Plan &p0, const GatherArgs &a0, const GatherArgs *table, const int64_t *prefix,
                            int B, int64_t total_tiles, hipStream_t st);
// Batched range check / fixed-point choice: jobs are BoundJob records
// (make_bound_job), prefix the cumulative row counts.
size_t bound_job_bytes();
void make_bound_job(const float *steps, const float *img, int64_t H, int64_t W, int64_t pitch, int32_t *status,
                    void *out);
bsf_status run_bound_batch(const Plan &p0, int img_kind, int32_t F_request, const void *jobs, const int64_t *prefix,
                           int B, int64_t total_rows, hipStream_t st);

// Bound / range check and fixed-point choice (gather.hip): the range check of
// the steps, the bound max|f| prod(box lengths) and the choice of F.  The taps
// repeat the range and headroom checks for the steps they are given.
bsf_status run_bound(const Plan &p, const Src &src, const float *steps, int32_t F_request, int32_t *status,
                     hipStream_t st);

// Adjoint (adjoint.hip).  Status words of the backward pass live in the
// workspace's status block after the forward ones.
enum AdjStatusWord : int {
    ST_G_ABSMAX_BITS = 16,  // scratch: float bits of max |gout| over the finite values
    ST_FG = 17,             // fixed-point bits of the scattered adjoint weights
    ST_G_NONFINITE = 18,    // this backward call saw a NaN or infinite upstream gradient
    ST_COLSUM_MAX = 20,     // scratch, 64 bits (words 20-21): max over p of 2^24 * the bound on sum_x k_x(p - x)
};

struct AdjointArgs {
    int64_t *Ghat;           // int64 window accumulating the scattered stencils
    int64_t Wp, pad_top, pad_left;
    int64_t H, W;
    const float *steps;
    const float *gout;
    const int32_t *status;   // Fg at status[ST_FG]
    float max_step;
    int M, order, tied, n_dirs;
    int32_t off[BSF_MAX_FACTORS];
    int32_t plane[BSF_MAX_FACTORS];
    int32_t canon;            // as in GatherArgs
    int32_t canon_plane[4];
    int32_t adx[BSF_MAX_DIRS], ady[BSF_MAX_DIRS];  // |dx|, |dy| of each direction (config order)
};
// aux: scan carries (at least scan_aux_bytes of the plan).
bsf_status run_adjoint_scatter(const Plan &p, const AdjointArgs &a, int32_t *status, void *aux, hipStream_t st);
bsf_status run_adjoint_finish(const Plan &p, const int64_t *Ghat, const int32_t *status, float *grad_img,
                              const float *gout, const float *dsteps, float *grad_steps, hipStream_t st);

// Covariance -> steps (cov.hip).  For a plan of four directions: n spans the
// null space of A -> sum_k A_k u_k u_k^T, P maps (C11, C12, C22) to a
// particular solution, w[e][k] = |u_k|^2 (u_k u_k^T)_e weighs K.
struct CovBank {
    double n[4];
    double P[4][3];
    double w[3][4];
};
bsf_status make_cov_bank(const Plan &p, CovBank *b);
// steps1 (and steps2, sel with a second bank): planes of the plans' layout;
// sub_dev (nullable, device float) or sub is subtracted from the diagonal.
bsf_status run_cov_to_steps(const Plan &p, const CovBank &b1, const CovBank *b2, const float *cov,
                            const float *sub_dev, float sub, float *steps1, float *steps2, uint8_t *sel,
                            int32_t *status, hipStream_t st);

}  // namespace bsf

#define BSF_HIP_CHECK(expr)                                   \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return BSF_E_DEVICE;            \
    } while (0)
