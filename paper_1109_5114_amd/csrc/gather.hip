// Per-pixel signed taps of the running sum (Section 1.1, second step of
// BoxFilter; Table 1; Alg. 3 step 3), plus the range check and the choice of
// the fixed-point bits.
//
// Each box factor j of step s contributes, for integer steps, the difference
// T_{c} - T_{c-s} of the running sum along u_j (c = floor((s-1)/2)), and for
// continuous steps the running sum read linearly between lattice points:
//     D_j = (1 - phi) (T_R - T_{-R-1}) + phi (T_{R+1} - T_{-R-2}),
//     R = floor((s-1)/2), phi = (s-1)/2 - R,
// a mix of two odd integer boxes.  The product of the D_j over the M factors is
// expanded into integer tap combinations J (one per choice of box per factor),
// each exact modulo 2^64 and small in magnitude, and only then weighted by the
// FP64 phase products.
//
// Every kernel runs on one image (arguments by value, 2-D grid of pixel
// tiles) or on a batch (BATCH: a 1-D work list of (image, tile) items, each
// block looking up its image's arguments).
#include <string.h>

#include <type_traits>
#include <utility>

#include "bsf_common.h"
#include "cluster_box.h"

namespace bsf {
namespace {

constexpr int kTile = 16;

// This block's image arguments and pixel-tile coordinates.
template <bool BATCH>
__device__ __forceinline__ bool tile_of_block(const GatherArgs &one, const GatherArgs *__restrict__ table,
                                              const int64_t *__restrict__ prefix, int B, int tile_w, int tile_h,
                                              GatherArgs &a, int64_t &bx, int64_t &by) {
    if constexpr (BATCH) {
        const int64_t gi = blockIdx.x;
        const int b = find_job(prefix, B, gi);
        a = table[b];
        const int64_t item = gi - prefix[b];
        if (item >= prefix[b + 1] - prefix[b]) return false;
        const int64_t tiles_x = (a.W + tile_w - 1) / tile_w;
        bx = item % tiles_x;
        by = item / tiles_x;
    } else {
        a = one;
        bx = blockIdx.x;
        by = blockIdx.y;
    }
    (void)tile_h;
    return true;
}

// Tile of work item `item` in an image of tiles_x x tiles_y tiles: bands of
// `band` tile rows, each band taken column by column.  The items one XCD runs
// at the same time then cover a block about as tall as it is wide (a few tens
// of tiles each way) instead of a strip one tile row high, and the boxes of
// the window its tiles read, which are offset from the tile by up to the
// steps' reach in every direction, stay in its L2 for all the combinations.
__device__ __forceinline__ void banded_tile(int64_t item, int64_t tiles_x, int64_t tiles_y, int band, int64_t &bx,
                                            int64_t &by) {
    const int64_t per_band = (int64_t)band * tiles_x;
    const int64_t b = item / per_band, in = item - b * per_band;
    const int64_t h = min((int64_t)band, tiles_y - b * band);  // rows of this band (the last may be short)
    bx = in / h;
    by = b * band + in % h;
}

// As tile_of_block, for a 1-D grid of xcd_grid(tiles) blocks in XCD order.
template <bool BATCH>
__device__ __forceinline__ bool tile_of_block_xcd(const GatherArgs &one, const GatherArgs *__restrict__ table,
                                                  const int64_t *__restrict__ prefix, int B, int tile_w, int tile_h,
                                                  GatherArgs &a, int64_t &bx, int64_t &by) {
    if constexpr (BATCH) {
        const int64_t total = prefix[B];
        const int64_t gi = xcd_item(blockIdx.x, total);
        if (gi >= total) return false;
        const int b = find_job(prefix, B, gi);
        a = table[b];
        const int64_t item = gi - prefix[b];
        const int64_t tiles_x = (a.W + tile_w - 1) / tile_w, tiles_y = (a.H + tile_h - 1) / tile_h;
        banded_tile(item, tiles_x, tiles_y, 64 / tile_h, bx, by);
    } else {
        a = one;
        const int64_t tiles_x = (a.W + tile_w - 1) / tile_w, tiles_y = (a.H + tile_h - 1) / tile_h;
        const int64_t item = xcd_item(blockIdx.x, tiles_x * tiles_y);
        if (item >= tiles_x * tiles_y) return false;
        banded_tile(item, tiles_x, tiles_y, 64 / tile_h, bx, by);
    }
    return true;
}

// 16 x 16 tile, each wavefront an 8 x 8 block.
__device__ __forceinline__ bool pixel_16x16(const GatherArgs &a, int64_t bx, int64_t by, int64_t &x, int64_t &y) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    x = bx * kTile + (w & 1) * 8 + (lane & 7);
    y = by * kTile + (w >> 1) * 8 + (lane >> 3);
    return x < a.W && y < a.H;
}

// Wavefront of WX x (64/WX) pixels; the four wavefronts of a workgroup stack
// vertically, so the workgroup covers WX x (256/WX).
template <int WX>
__device__ __forceinline__ bool pixel_wx(const GatherArgs &a, int64_t bx, int64_t by, int64_t &x, int64_t &y) {
    constexpr int WY = 64 / WX;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    x = bx * WX + (lane % WX);
    y = by * (4 * WY) + w * WY + (lane / WX);
    return x < a.W && y < a.H;
}

// Pixels of another bank (a.sel non-null and not a.sel_id) are left alone.
__device__ __forceinline__ bool selected(const GatherArgs &a, int64_t idx) {
    return !a.sel || a.sel[idx] == a.sel_id;
}

__device__ __forceinline__ float clamp_step(float s, float max_step) {
    // NaN -> 1 (fmaxf returns the non-NaN operand); keeps every tap in the window
    return fminf(fmaxf(s, 1.0f), max_step);
}

// ceil(log2(v)) for v >= 1, from the binary exponent (frexp: v = m 2^e, m in [0.5, 1)).
__device__ __forceinline__ int ceil_log2(double v) {
    int e;
    const double m = __builtin_frexp(v, &e);
    return m == 0.5 ? e - 1 : e;
}

// The checks of the preparing pass, repeated by the taps for the steps they
// are given (they may differ from the ones the window was prepared with):
// one factor's step s adds to `bad` (NaN, below 1, above max_step, or not an
// integer in integer mode) and multiplies its box length into `prod`.
__device__ __forceinline__ void step_check(float s, float max_step, int mode, int reps, bool &bad, double &prod) {
    if (!(s >= 1.0f) || s > max_step) bad = true;
    const float sc = clamp_step(s, max_step);
    double len;
    if (mode == BSF_STEPS_INT) {
        if (sc != floorf(sc)) bad = true;
        len = (double)rintf(sc);
    } else {
        len = (double)(2.0f * floorf((sc - 1.0f) * 0.5f) + 3.0f);
    }
    for (int r = 0; r < reps; ++r) prod *= len;
}

// Raises BSF_FLAG_RANGE for a bad step and BSF_FLAG_OVERFLOW when the product
// of box lengths leaves the tap combination without int64 headroom at the
// window's F (ef + F + ceil log2 prod > 62).
__device__ __forceinline__ void report_steps(const GatherArgs &a, bool bad, double prod) {
    int32_t *status = const_cast<int32_t *>(a.status);
    if (bad) atomicOr((unsigned *)&status[ST_FLAGS], BSF_FLAG_RANGE);
    const int ef = a.status[ST_EF];
    if (a.status[ST_ARITH] == BSF_ARITH_EXACT && ef > -1000 &&
        ef + a.status[ST_F_USED] + ceil_log2(prod * (1.0 + 0x1p-40)) > 62)
        atomicOr((unsigned *)&status[ST_FLAGS], BSF_FLAG_OVERFLOW);
}

// Every plane of a pixel through step_check, then report_steps.
__device__ __forceinline__ void check_pixel_steps(const GatherArgs &a, int64_t idx) {
    const int64_t HW = a.H * a.W;
    const int planes = a.tied ? a.n_dirs : a.M, reps = a.tied ? a.order : 1;
    bool bad = false;
    double prod = 1.0;
    for (int q = 0; q < planes; ++q) step_check(a.steps[q * HW + idx], a.max_step, a.mode, reps, bad, prod);
    report_steps(a, bad, prod);
}

__device__ __forceinline__ double ldexp_neg(double v, int F) { return __builtin_ldexp(v, -F); }

// ----------------------------------------------------------------------------
// Range check and fixed-point bound.
// ----------------------------------------------------------------------------
struct BoundJob {
    const float *steps;
    const float *img;  // nullable: float image whose max |f| bounds F
    int64_t H, W, pitch;
    int32_t *status;
};

template <bool BATCH>
__global__ void k_status_begin(BoundJob one, const BoundJob *__restrict__ jobs, int32_t F_request) {
    if (threadIdx.x != 0) return;
    int32_t *status = BATCH ? jobs[blockIdx.x].status : one.status;
    status[ST_EP_MAX] = 0;
    status[ST_FABS_BITS] = 0;
    status[ST_F_REQUEST] = F_request;
}

// Rows y = first, first + stride, ...; threads stride over columns; a
// wavefront and LDS reduction, and one atomic per workgroup.  Single image:
// one workgroup per group of rows; batch: one workgroup per (image, row).
template <bool BATCH>
__global__ __launch_bounds__(256) void k_bound(BoundJob one, const BoundJob *__restrict__ jobs,
                                               const int64_t *__restrict__ prefix, int B, int planes, int per_plane,
                                               int mode, float max_step) {
    __shared__ int s_ep[4], s_bad[4], s_nf[4];
    __shared__ unsigned s_fb[4];
    BoundJob job;
    int64_t first, stride;
    if constexpr (BATCH) {
        const int64_t gi = blockIdx.x;
        const int b = find_job(prefix, B, gi);
        job = jobs[b];
        first = gi - prefix[b];
        stride = job.H;
    } else {
        job = one;
        first = blockIdx.x;
        stride = gridDim.x;
    }
    int ep_max = 0;
    unsigned fbits = 0;
    int bad = 0, nonfinite = 0;
    const int64_t H = job.H, W = job.W, HW = H * W;
    // one factor step: range check, its box length into prod
    auto factor = [&](float s, double &prod) {
        if (!(s >= 1.0f) || s > max_step) bad = 1;  // catches NaN
        const float sc = clamp_step(s, max_step);
        double len;
        if (mode == BSF_STEPS_INT) {
            if (sc != floorf(sc)) bad = 1;
            len = (double)rintf(sc);
        } else {
            len = (double)(2.0f * floorf((sc - 1.0f) * 0.5f) + 3.0f);
        }
        for (int r = 0; r < per_plane; ++r) prod *= len;
    };
    // products of small integers are exact in FP64 up to 2^53; above that
    // round the bound up a little so it stays an upper bound
    auto finish = [&](double prod) { ep_max = max(ep_max, ceil_log2(prod * (1.0 + 0x1p-40))); };
    auto image = [&](float f_abs) {
        if (f_abs <= 3.402823466e38f) fbits = max(fbits, __float_as_uint(f_abs));
        else nonfinite = 1;  // NaN or infinity
    };
    // four consecutive pixels per thread and 16-byte loads where rows and
    // pitches allow them, one pixel at a time otherwise
    const bool vec = (W % 4 == 0) && (!job.img || job.pitch % 4 == 0);
    for (int64_t y = first; y < H; y += stride) {
        if (vec) {
            for (int64_t x = 4 * (int64_t)threadIdx.x; x < W; x += 4 * (int64_t)blockDim.x) {
                double p0 = 1.0, p1 = 1.0, p2 = 1.0, p3 = 1.0;
                for (int q = 0; q < planes; ++q) {
                    const float4 v = *reinterpret_cast<const float4 *>(job.steps + q * HW + y * W + x);
                    factor(v.x, p0);
                    factor(v.y, p1);
                    factor(v.z, p2);
                    factor(v.w, p3);
                }
                finish(p0);
                finish(p1);
                finish(p2);
                finish(p3);
                if (job.img) {
                    const float4 fv = *reinterpret_cast<const float4 *>(job.img + y * job.pitch + x);
                    image(fabsf(fv.x));
                    image(fabsf(fv.y));
                    image(fabsf(fv.z));
                    image(fabsf(fv.w));
                }
            }
        } else {
            for (int64_t x = threadIdx.x; x < W; x += blockDim.x) {
                const int64_t i = y * W + x;
                double prod = 1.0;
                for (int q = 0; q < planes; ++q) factor(job.steps[q * HW + i], prod);
                finish(prod);
                if (job.img) image(fabsf(job.img[y * job.pitch + x]));
            }
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        ep_max = max(ep_max, __shfl_xor(ep_max, d, 64));
        fbits = max(fbits, (unsigned)__shfl_xor((int)fbits, d, 64));
        bad |= __shfl_xor(bad, d, 64);
        nonfinite |= __shfl_xor(nonfinite, d, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_ep[w] = ep_max;
        s_fb[w] = fbits;
        s_bad[w] = bad;
        s_nf[w] = nonfinite;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            ep_max = max(ep_max, s_ep[k]);
            fbits = max(fbits, s_fb[k]);
            bad |= s_bad[k];
            nonfinite |= s_nf[k];
        }
        atomicMax(&job.status[ST_EP_MAX], ep_max);
        if (job.img) atomicMax((unsigned *)&job.status[ST_FABS_BITS], fbits);
        if (bad) atomicOr((unsigned *)&job.status[ST_FLAGS], BSF_FLAG_RANGE);
        if (nonfinite) atomicOr((unsigned *)&job.status[ST_FLAGS], BSF_FLAG_NONFINITE);
    }
}

// img_kind: SRC_F32, SRC_U8 or SRC_U16; arith: exact or fp64.
template <bool BATCH>
__global__ void k_choose_F(BoundJob one, const BoundJob *__restrict__ jobs, int img_kind, int arith) {
    if (threadIdx.x != 0) return;
    int32_t *status = BATCH ? jobs[blockIdx.x].status : one.status;
    const int eP = status[ST_EP_MAX];
    int ef;
    bool zero = false;
    if (img_kind == SRC_U8) {
        ef = 8;
    } else if (img_kind == SRC_U16) {
        ef = 16;
    } else {
        const float fmax = __uint_as_float((unsigned)status[ST_FABS_BITS]);
        if (fmax == 0.0f) {
            zero = true;
            ef = 0;
        } else {
            ef = ceil_log2((double)fmax);  // |f| <= 2^ef
        }
    }
    int F;
    if (img_kind != SRC_F32) {
        F = 0;
    } else if (status[ST_F_REQUEST] >= 0) {
        F = status[ST_F_REQUEST];
    } else {
        // not clamped: a tiny image keeps its significant bits (F > 62), a
        // huge one is quantised more coarsely (F < 0) instead of overflowing
        F = 62 - (zero ? 0 : ef) - eP;
    }
    // |f_q| <= 2^(ef + F) (+1/2 from rounding) and |J| <= |f_q| * prod <= 2^(ef + F + eP)
    if (arith == BSF_ARITH_EXACT && !zero && ef + F + eP > 62)
        atomicOr((unsigned *)&status[ST_FLAGS], BSF_FLAG_OVERFLOW);
    status[ST_F_USED] = F;
    status[ST_LOG2_BOUND] = ef + eP;
    status[ST_EF] = zero ? -1000 : ef;
    status[ST_ARITH] = arith;
}

// ----------------------------------------------------------------------------
// Integer steps: 2^M signed taps (Table 1 signs (-1)^popcount), exact.
// ----------------------------------------------------------------------------
template <typename V, int MT, bool BATCH>
__global__ __launch_bounds__(256) void k_gather_int(GatherArgs one, const GatherArgs *__restrict__ table,
                                                    const int64_t *__restrict__ prefix, int B) {
    GatherArgs a;
    int64_t bx, by, x, y;
    if (!tile_of_block_xcd<BATCH>(one, table, prefix, B, kTile, kTile, a, bx, by)) return;
    // wavefronts of 16 x 4 pixels: a tap of 16 neighbours in a row reads one
    // 128-byte line of the window
    if (!pixel_wx<16>(a, bx, by, x, y) || !selected(a, y * a.W + x)) return;
    const int M = MT > 0 ? MT : a.M;
    const int64_t HW = a.H * a.W, idx = y * a.W + x;
    const V *G = static_cast<const V *>(a.G) + (y + a.pad_top) * a.Wp + (x + a.pad_left);
    int64_t pa[BSF_MAX_FACTORS], pb[BSF_MAX_FACTORS];
    int64_t den = 1;
    bool bad = false;
    double prod = 1.0;
#pragma unroll
    for (int j = 0; j < (MT > 0 ? MT : BSF_MAX_FACTORS); ++j) {
        if (j >= M) break;
        const float s_raw = a.steps[a.plane[j] * HW + idx];
        step_check(s_raw, a.max_step, BSF_STEPS_INT, 1, bad, prod);
        const float s = clamp_step(s_raw, a.max_step);
        const int si = min((int)rintf(s), (int)a.max_step);   // stays inside the window's reach
        const int c = (si - 1) >> 1;
        pa[j] = (int64_t)c * a.off[j];
        pb[j] = (int64_t)(c - si) * a.off[j];
        den *= si;
    }
    report_steps(a, bad, prod);
    V num = V(0);
    const int n = 1 << M;
    if constexpr (MT > 0) {
#pragma unroll
        for (int e = 0; e < (1 << MT); ++e) {
            int64_t o = 0;
#pragma unroll
            for (int j = 0; j < MT; ++j) o += (e >> j & 1) ? pb[j] : pa[j];
            if (__builtin_popcount(e) & 1) num -= G[o];
            else num += G[o];
        }
    } else {
        for (int e = 0; e < n; ++e) {
            int64_t o = 0;
            for (int j = 0; j < M; ++j) o += (e >> j & 1) ? pb[j] : pa[j];
            if (__builtin_popcount(e) & 1) num -= G[o];
            else num += G[o];
        }
    }
    if constexpr (std::is_integral_v<V>) {
        const int F = a.status[ST_F_USED];
        if (a.out_num) a.out_num[idx] = num;
        if (a.out_den) a.out_den[idx] = den;
        if (a.out) a.out[idx] = (float)(ldexp_neg((double)num, F) / (double)den);
    } else {
        if (a.out_den) a.out_den[idx] = den;
        if (a.out) a.out[idx] = (float)(num / (double)den);
    }
}

// ----------------------------------------------------------------------------
// Continuous steps, any factor count: per factor two integer boxes; 2^M box
// choices e, each an exact 2^M-tap combination J_e, weighted by
// prod_j (e_j ? phi_j : 1 - phi_j).  4^M loads per pixel: the reference path
// for configurations without a specialised kernel.
// ----------------------------------------------------------------------------
// MT > 0 fixes the factor count at compile time (M = 4 is the order-1
// filter of four directions): the loops unroll and the per-factor arrays live
// in registers.  MT = 0 takes any M up to BSF_MAX_FACTORS.
template <typename V, int MT, bool BATCH>
__global__ __launch_bounds__(256) void k_gather_real_generic(GatherArgs one, const GatherArgs *__restrict__ table,
                                                             const int64_t *__restrict__ prefix, int B) {
    constexpr int MAXF = MT > 0 ? MT : BSF_MAX_FACTORS;
    GatherArgs a;
    int64_t bx, by, x, y;
    if (!tile_of_block_xcd<BATCH>(one, table, prefix, B, kTile, kTile, a, bx, by)) return;
    if (!pixel_wx<16>(a, bx, by, x, y) || !selected(a, y * a.W + x)) return;  // rows of 16: whole lines
    check_pixel_steps(a, y * a.W + x);
    const int M = MT > 0 ? MT : a.M;
    const int64_t HW = a.H * a.W, idx = y * a.W + x;
    const V *G = static_cast<const V *>(a.G) + (y + a.pad_top) * a.Wp + (x + a.pad_left);
    int64_t pos[MAXF][4];  // [j][2*e + t]: e = box (0 narrow, 1 wide), t = end (0 top, 1 bottom)
    double ph[MAXF];
    double den = 1.0;
#pragma unroll
    for (int j = 0; j < MAXF; ++j) {
        if (j >= M) break;
        const float s = clamp_step(a.steps[a.plane[j] * HW + idx], a.max_step);
        const float t = (s - 1.0f) * 0.5f;
        const float R = floorf(t);
        ph[j] = (double)(t - R);
        const int64_t Ri = (int64_t)R;
        pos[j][0] = Ri * a.off[j];
        pos[j][1] = (-Ri - 1) * a.off[j];
        pos[j][2] = (Ri + 1) * a.off[j];
        pos[j][3] = (-Ri - 2) * a.off[j];
        den *= (double)s;
    }
    double tot = 0.0;
    double dtot[MAXF];
#pragma unroll
    for (int j = 0; j < MAXF; ++j) dtot[j] = 0.0;
    const bool want_d = a.dsteps != nullptr;
    const int n = 1 << M;
    // one box choice e at a time (its 2^M loads in flight together)
#pragma unroll 1
    for (int e = 0; e < n; ++e) {
        double w = 1.0;
#pragma unroll
        for (int j = 0; j < MAXF; ++j)
            if (j < M) w *= (e >> j & 1) ? ph[j] : 1.0 - ph[j];
        if (MT == 0 && w == 0.0 && !want_d) continue;
        V J = V(0);
#pragma unroll
        for (int t = 0; t < (MT > 0 ? (1 << MT) : n); ++t) {
            int64_t o = 0;
#pragma unroll
            for (int j = 0; j < MAXF; ++j)
                if (j < M) o += pos[j][2 * (e >> j & 1) + (t >> j & 1)];
            if (__builtin_popcount(t) & 1) J -= G[o];
            else J += G[o];
        }
        tot += w * (double)J;
        if (want_d) {
            // d w / d phi_j: the product over the other factors, signed by the box choice
#pragma unroll
            for (int j = 0; j < MAXF; ++j) {
                if (j >= M) break;
                double dw = (e >> j & 1) ? 1.0 : -1.0;
#pragma unroll
                for (int l = 0; l < MAXF; ++l)
                    if (l != j && l < M) dw *= (e >> l & 1) ? ph[l] : 1.0 - ph[l];
                dtot[j] += dw * (double)J;
            }
        }
    }
    int F = 0;
    if constexpr (std::is_integral_v<V>) F = a.status[ST_F_USED];
    const double outv = ldexp_neg(tot, F) / den;
    if (a.out) a.out[idx] = (float)outv;
    if (want_d) {
        // plane q collects its factors: d out / d s_j = (1/2) dJ-term / den - out / s_j
        const int planes = a.tied ? a.n_dirs : M;
        for (int q = 0; q < planes; ++q) {
            double d = 0.0;
#pragma unroll
            for (int j = 0; j < MAXF; ++j) {
                if (j >= M) break;
                if (a.plane[j] != q) continue;
                const double s = (double)clamp_step(a.steps[a.plane[j] * HW + idx], a.max_step);
                d += 0.5 * ldexp_neg(dtot[j], F) / den - outv / s;
            }
            a.dsteps[q * HW + idx] = (float)d;
        }
    }
}

// ----------------------------------------------------------------------------
// Continuous steps, four directions, order 2, steps tied per direction.
//
// Per direction k the squared difference D_k^2 =
//   (1-phi)^2 P_a^2 + 2 phi (1-phi) P_a P_b + phi^2 P_b^2
// touches 9 lattice positions in three clusters of three consecutive points,
//   T = 2R + {0,1,2},  M = -2 + {0,1,2},  B = -2R - 4 + {0,1,2},
// and the three integer operators read them as
//   aa = P_a^2    = T0 - 2 M1 + B2
//   ab = P_a P_b  = T1 - M0 - M2 + B1
//   bb = P_b^2    = T2 - 2 M1 + B0.
// The 3^4 = 81 products J[a0][a1][a2][a3] are contracted one direction at a
// time (innermost first) in exact int64; the innermost direction is the one
// with window offset +1 when the set has it, so each cluster is three
// consecutive int64.
// ----------------------------------------------------------------------------

// One 8-byte running-sum value.  Offsets are 32-bit byte offsets from the
// window base (the launcher checks the window is below 4 GiB); forming the
// address as base pointer + offset lets constant deltas become load
// immediates, so a cluster of three consecutive taps costs one address add.
__device__ __forceinline__ int64_t ldG(const char *__restrict__ p) {
    return *reinterpret_cast<const int64_t *>(p);
}

// acc[a1][a2][a3] += sum over the 9 x 9 x 9 taps (p1, p2, p3) of directions
// 1..3 of C1 C2 C3 G[b + o1(p1) + o2(p2) + o3(p3)], direction 3 innermost.
// Tap index p = 3 * cluster + sub.  The two inner levels keep positive and
// negative parts apart so that every fold is an add; the sign of the
// direction-1 tap is applied once per p1.
template <bool CONTIG>
__device__ __forceinline__ void contract3(const char *__restrict__ Gb, uint32_t b, const int32_t cT[4],
                                          const int32_t cB[4], const int32_t st[4], int64_t acc[27]) {
    const int32_t st3 = CONTIG ? 8 : st[3];
#pragma unroll
    for (int p1 = 0; p1 < 9; ++p1) {
        const int c1 = p1 / 3, s1 = p1 % 3;
        const uint32_t b1 = b + (uint32_t)((c1 == 0 ? cT[1] : c1 == 1 ? -2 * st[1] : cB[1]) + s1 * st[1]);
        int64_t ipos[9], ineg[9];  // [a2][a3]
#pragma unroll
        for (int q = 0; q < 9; ++q) { ipos[q] = 0; ineg[q] = 0; }
#pragma unroll
        for (int p2 = 0; p2 < 9; ++p2) {
            const int c2 = p2 / 3, s2 = p2 % 3;
            const uint32_t b2 = b1 + (uint32_t)((c2 == 0 ? cT[2] : c2 == 1 ? -2 * st[2] : cB[2]) + s2 * st[2]);
            const char *pT = Gb + (uint32_t)(b2 + (uint32_t)cT[3]);
            const char *pM = Gb + b2;
            const char *pB = Gb + (uint32_t)(b2 + (uint32_t)cB[3]);
            const int64_t T0 = ldG(pT), T1 = ldG(pT + st3), T2 = ldG(pT + 2 * st3);
            const int64_t M0 = ldG(pM - 2 * st3), M1 = ldG(pM - st3), M2 = ldG(pM);
            const int64_t B0 = ldG(pB), B1 = ldG(pB + st3), B2 = ldG(pB + 2 * st3);
            const int64_t P0 = T0 + B2, P1 = T1 + B1, P2 = T2 + B0, N1 = M0 + M2;
            if (c2 != 1) {  // T or B tap: +1 on operator a2
                const int a2 = (c2 == 0) ? s2 : 2 - s2;
                ipos[a2 * 3 + 0] += P0; ipos[a2 * 3 + 1] += P1; ipos[a2 * 3 + 2] += P2;
                ineg[a2 * 3 + 0] += 2 * M1; ineg[a2 * 3 + 1] += N1; ineg[a2 * 3 + 2] += 2 * M1;
            } else if (s2 != 1) {  // M0, M2: -1 on ab
                ipos[3] += 2 * M1; ipos[4] += N1; ipos[5] += 2 * M1;
                ineg[3] += P0; ineg[4] += P1; ineg[5] += P2;
            } else {  // M1: -2 on aa and bb
                ipos[0] += 4 * M1; ipos[1] += 2 * N1; ipos[2] += 4 * M1;
                ineg[0] += 2 * P0; ineg[1] += 2 * P1; ineg[2] += 2 * P2;
                ipos[6] += 4 * M1; ipos[7] += 2 * N1; ipos[8] += 4 * M1;
                ineg[6] += 2 * P0; ineg[7] += 2 * P1; ineg[8] += 2 * P2;
            }
        }
        if (c1 != 1) {
            const int a1 = (c1 == 0) ? s1 : 2 - s1;
#pragma unroll
            for (int q = 0; q < 9; ++q) acc[a1 * 9 + q] += ipos[q] - ineg[q];
        } else if (s1 != 1) {
#pragma unroll
            for (int q = 0; q < 9; ++q) acc[9 + q] += ineg[q] - ipos[q];
        } else {
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int64_t d = ineg[q] - ipos[q];
                acc[q] += 2 * d;
                acc[18 + q] += 2 * d;
            }
        }
    }
}

// Phase weights of one tied order-2 direction, (1-phi)^2, 2 phi (1-phi), phi^2
// for the operators aa, ab, bb, and their derivatives with respect to phi.
__device__ __forceinline__ void phase_weights(float phf, double w[3], double dw[3]) {
    const double p = (double)phf, q = 1.0 - p;
    w[0] = q * q;
    w[1] = 2.0 * p * q;
    w[2] = p * p;
    dw[0] = -2.0 * q;
    dw[1] = 2.0 - 4.0 * p;
    dw[2] = 2.0 * p;
}

__device__ __forceinline__ double contract_fp(const int64_t acc[27], const double w1[3], const double w2[3],
                                              const double w3[3]) {
    double r = 0.0;
#pragma unroll
    for (int a1 = 0; a1 < 3; ++a1) {
        double r1 = 0.0;
#pragma unroll
        for (int a2 = 0; a2 < 3; ++a2) {
            double r2 = 0.0;
#pragma unroll
            for (int a3 = 0; a3 < 3; ++a3) r2 += w3[a3] * (double)acc[(a1 * 3 + a2) * 3 + a3];
            r1 += w2[a2] * r2;
        }
        r += w1[a1] * r1;
    }
    return r;
}

// One pixel of the tied order-2 four-direction filter, taps read straight
// from the window.  Direction 0 is outermost: its taps are visited in an order
// that finishes one operator at a time, so only the 27 values J[a0][.][.][.] of
// the current operator a0 are live:
//   aa: -2 M1, + T0, + B2;   bb: -2 M1, + T2, + B0;   ab: -(M0 + M2), + T1, + B1
// (M1 is visited twice, 10 steps in all).
template <bool CONTIG, bool DERIV = true>
__device__ __forceinline__ void t2n4_pixel(const GatherArgs &a, int64_t x, int64_t y) {
    const int64_t HW = a.H * a.W, idx = y * a.W + x;
    const char *Gb = static_cast<const char *>(a.G);
    const uint32_t base = (uint32_t)(((y + a.pad_top) * a.Wp + (x + a.pad_left)) * 8);
    // contraction direction k is config factor 2k (tied: both copies share a plane)
    int32_t cT[4], cB[4], st[4];
    float ph[4], sk[4];
    double den = 1.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float s = clamp_step(a.steps[a.plane[2 * k] * HW + idx], a.max_step);
        const float t = (s - 1.0f) * 0.5f;
        const float Rf = floorf(t);
        const int32_t R = (int32_t)Rf;
        st[k] = a.off[2 * k] * 8;
        ph[k] = t - Rf;
        sk[k] = s;
        cT[k] = 2 * R * st[k];
        cB[k] = (-2 * R - 4) * st[k];
        den *= (double)s * (double)s;
    }
    double dtot[4] = {0.0, 0.0, 0.0, 0.0};
    constexpr int kSeq[10] = {4, 0, 8, 4, 2, 6, 3, 5, 1, 7};
    double tot = 0.0;
    int64_t acc[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) acc[q] = 0;
    for (int i = 0; i < 10; ++i) {
        const int p0 = kSeq[i];
        if (i == 0 || i == 3 || i == 6) {
#pragma unroll
            for (int q = 0; q < 27; ++q) acc[q] = 0;
        }
        const int c0 = p0 / 3, s0 = p0 % 3;
        const int32_t o0 = (c0 == 0 ? cT[0] : c0 == 1 ? -2 * st[0] : cB[0]) + s0 * st[0];
        contract3<CONTIG>(Gb, base + (uint32_t)o0, cT, cB, st, acc);
        if (i == 0 || i == 3) {
#pragma unroll
            for (int q = 0; q < 27; ++q) acc[q] = -2 * acc[q];
        }
        if (i == 7) {
#pragma unroll
            for (int q = 0; q < 27; ++q) acc[q] = -acc[q];
        }
        if (i == 2 || i == 5 || i == 9) {
            double w[4][3], dw[4][3];
#pragma unroll
            for (int k = 0; k < 4; ++k) phase_weights(ph[k], w[k], dw[k]);
            const int a0 = (i == 2) ? 0 : (i == 5) ? 2 : 1;
            const double r = contract_fp(acc, w[1], w[2], w[3]);
            tot += w[0][a0] * r;
            if (DERIV && a.dsteps) {
                dtot[0] += dw[0][a0] * r;
                dtot[1] += w[0][a0] * contract_fp(acc, dw[1], w[2], w[3]);
                dtot[2] += w[0][a0] * contract_fp(acc, w[1], dw[2], w[3]);
                dtot[3] += w[0][a0] * contract_fp(acc, w[1], w[2], dw[3]);
            }
        }
    }
    const int F = a.status[ST_F_USED];
    const double outv = ldexp_neg(tot, F) / den;
    if (a.out) a.out[idx] = (float)outv;
    if (DERIV && a.dsteps) {
        // d phi / d s = 1/2, and the step of direction k enters prod s twice
#pragma unroll
        for (int k = 0; k < 4; ++k)
            a.dsteps[a.plane[2 * k] * HW + idx] = (float)(0.5 * ldexp_neg(dtot[k], F) / den - 2.0 * outv / sk[k]);
    }
}

// WAVES bounds the registers so that that many wavefronts fit on a SIMD; WX
// is the wavefront's pixel width.
template <bool CONTIG, int WAVES, int WX, bool BATCH, bool DERIV = true>
__global__ __launch_bounds__(256, WAVES) void k_gather_t2n4(GatherArgs one, const GatherArgs *__restrict__ table,
                                                            const int64_t *__restrict__ prefix, int B) {
    GatherArgs a;
    int64_t bx, by, x, y;
    if (!tile_of_block<BATCH>(one, table, prefix, B, WX, 256 / WX, a, bx, by)) return;
    if (!pixel_wx<WX>(a, bx, by, x, y) || !selected(a, y * a.W + x)) return;
    check_pixel_steps(a, y * a.W + x);
    t2n4_pixel<CONTIG, DERIV>(a, x, y);
}

// ----------------------------------------------------------------------------
// Tied order-2 filter along (1,0), (0,1), (1,1), (1,-1) from LDS cluster boxes.
// A 16 x 16 tile visits the 81 cluster combinations; for each it stages the
// combination's box of the window in LDS with row-contiguous loads, and every
// pixel reads its 37 distinct sub-patch points at static offsets from its
// anchor and adds them into the 81 exact values J.  Combinations with an even
// number of M clusters come first; J is then negated once, so the odd ones
// (whose taps are all negative) are added too, and the FP64 combination
// negates the result back.  A tile whose step range would not fit the LDS box
// falls back to reading its taps from the window.
// ----------------------------------------------------------------------------
// acc += v << sh as one v_lshl_add_u64 (sh <= 4), also when the same shifted
// value feeds two accumulators (the compiler would shift once and add twice).
__device__ __forceinline__ void shl_add(uint64_t &acc, uint64_t v, int sh) {
    switch (sh) {
    case 0: acc += v; break;
    case 1: asm("v_lshl_add_u64 %0, %1, 1, %2" : "=v"(acc) : "v"(v), "v"(acc)); break;
    case 2: asm("v_lshl_add_u64 %0, %1, 2, %2" : "=v"(acc) : "v"(v), "v"(acc)); break;
    case 3: asm("v_lshl_add_u64 %0, %1, 3, %2" : "=v"(acc) : "v"(v), "v"(acc)); break;
    default: asm("v_lshl_add_u64 %0, %1, 4, %2" : "=v"(acc) : "v"(v), "v"(acc)); break;
    }
}

// The lane number, computed anew at every use (not shared between uses).
__device__ __forceinline__ int fresh_lane_id() {
    int lo, id;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0" : "=v"(lo));
    asm volatile("v_mbcnt_hi_u32_b32 %0, -1, %1" : "=v"(id) : "v"(lo));
    return id;
}

// Tiles of the forward cluster-box kernel: 16 columns by TH rows of pixels, one
// wavefront per 16 x 4 block of them, and the LDS box rows each stages: 16 x 8
// tiles of two wavefronts with 38-row boxes (four workgroups per CU in 158 KB of
// LDS), or 16 x 4 tiles of one wavefront with 18-row boxes (eight workgroups per
// CU in 150 KB).  Narrower boxes waste less of every copy, but tiles whose step
// range needs more rows fall back to direct window reads, so the best shape
// depends on how fast the step field varies (the tuner times both).
constexpr int kFwdTileW = 16;
template <int TH>
struct FwdShape {
    static_assert(TH == 4 || TH == 8, "tile heights");
    static constexpr int H = TH;
    static constexpr int Waves = TH / 4;
    static constexpr int Rows = TH == 8 ? 38 : 18;
    static constexpr int Elems = cbox::kPitch * Rows;
    static_assert(kFwdTileW + 64 * (TH - 1) < 1024 && Rows % 2 == 0, "tile shape");
};
// Position of thread i's pixel in the tile.
__device__ __forceinline__ int fwd_tx(int i) { return i & 15; }
__device__ __forceinline__ int fwd_ty(int i) { return 4 * (i >> 6) + ((i >> 4) & 3); }

// Patch row (Y + 2) of the lowest sub-tap a row tuple of combination C reads.
__host__ __device__ constexpr int tuple_max_row(int C, int r0, int r1, int r2, int r3) {
    using namespace cbox;
    const int c0 = cl(C, 0), c1 = cl(C, 1), c2 = cl(C, 2), c3 = cl(C, 3);
    int m = 0;
    for (int i0 = 0; i0 < n_sub(c0, r0); ++i0)
        for (int i1 = 0; i1 < n_sub(c1, r1); ++i1)
            for (int i2 = 0; i2 < n_sub(c2, r2); ++i2)
                for (int i3 = 0; i3 < n_sub(c3, r3); ++i3) {
                    const int y = sub_q(c1, r1, i1) + sub_q(c2, r2, i2) - sub_q(c3, r3, i3) + 2;
                    m = y > m ? y : m;
                }
    return m;
}

// Adds of the row tuples of combination C selected by PASS: 0 = those reading
// patch rows 0-3 only with r0 == 0, 1 = the same with r0 > 0, 2 = the rest.
template <int C, int PASS>
__device__ __forceinline__ void box_fwd_pass(const uint64_t val[49], uint64_t J[81]) {
    using namespace cbox;
    constexpr int c0 = cl(C, 0), c1 = cl(C, 1), c2 = cl(C, 2), c3 = cl(C, 3);
#pragma unroll
    for (int r0 = 0; r0 < n_rows(c0); ++r0)
#pragma unroll
        for (int r1 = 0; r1 < n_rows(c1); ++r1)
#pragma unroll
            for (int r2 = 0; r2 < n_rows(c2); ++r2)
#pragma unroll
                for (int r3 = 0; r3 < n_rows(c3); ++r3) {
                    const bool upper = tuple_max_row(C, r0, r1, r2, r3) <= 3;
                    const int pass = !upper ? 2 : r0 == 0 ? 0 : 1;
                    if (pass != PASS) continue;
                    uint64_t v = 0;
#pragma unroll
                    for (int i0 = 0; i0 < n_sub(c0, r0); ++i0)
#pragma unroll
                        for (int i1 = 0; i1 < n_sub(c1, r1); ++i1)
#pragma unroll
                            for (int i2 = 0; i2 < n_sub(c2, r2); ++i2)
#pragma unroll
                                for (int i3 = 0; i3 < n_sub(c3, r3); ++i3) {
                                    const int q0 = sub_q(c0, r0, i0), q1 = sub_q(c1, r1, i1);
                                    const int q2 = sub_q(c2, r2, i2), q3 = sub_q(c3, r3, i3);
                                    v += val[(q0 + q2 + q3) + 7 * (q1 + q2 - q3 + 2)];
                                }
                    const int sh = doubled(c0, r0) + doubled(c1, r1) + doubled(c2, r2) + doubled(c3, r3);
#pragma unroll
                    for (int j0 = 0; j0 < n_out(c0, r0); ++j0)
#pragma unroll
                        for (int j1 = 0; j1 < n_out(c1, r1); ++j1)
#pragma unroll
                            for (int j2 = 0; j2 < n_out(c2, r2); ++j2)
#pragma unroll
                                for (int j3 = 0; j3 < n_out(c3, r3); ++j3)
                                    shl_add(J[jidx(out_o(c0, r0, j0), out_o(c1, r1, j1), out_o(c2, r2, j2),
                                                   out_o(c3, r3, j3))],
                                            v, sh);
                }
}

// One combination: the 22 patch points of rows 0-3 are loaded together, the
// tuples reading only those start, the 15 points of rows 4-6 are loaded
// (kept below that first part by a scheduling barrier, so that not all 37
// values are live at once), and the remaining tuples follow.
template <int C>
__device__ __forceinline__ void box_fwd_combo(const uint64_t *__restrict__ p, const uint64_t *__restrict__ p_hi,
                                              uint64_t J[81]) {
    using namespace cbox;
    uint64_t val[49];
#pragma unroll
    for (int P = 0; P < 4 * 7; ++P)
        if (kPatch.count[P] > 0) val[P] = p[point_elem(P)];
    box_fwd_pass<C, 0>(val, J);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int P = 4 * 7; P < 49; ++P)
        if (kPatch.count[P] > 0) val[P] = p_hi[point_elem(P) - 4 * kPitch];
    box_fwd_pass<C, 1>(val, J);
    box_fwd_pass<C, 2>(val, J);
}

// Frame 1 (the directions of Table 1, (2,1), (1,2), (1,-2), (2,-1)): the
// 81 sub-taps of a combination fall on 73 distinct points of a 13 x 13 patch,
// one or two per point, so each sub-tap is added into its targets on its own
// (a T tap q feeds o = q, a B tap o = 2 - q, M1 both aa and bb doubled, M0 and
// M2 ab).  The patch is read in four batches of rows, each from its own
// opaque LDS base, and a batch's sub-taps are added before the next batch is
// loaded, so that at most 23 values wait in registers beside J.
struct F1Points {
    bool hit[13 * 13];  // point X + 13 Y of the patch is some sub-tap's
};
__host__ __device__ constexpr F1Points make_f1_points() {
    F1Points t{};
    for (int q = 0; q < 81; ++q) {
        const int q0 = q % 3, q1 = (q / 3) % 3, q2 = (q / 9) % 3, q3 = q / 27;
        t.hit[cbox::sub_dx<1>(q0, q1, q2, q3) + 13 * cbox::sub_row<1>(q0, q1, q2, q3)] = true;
    }
    return t;
}
constexpr F1Points kF1Points = make_f1_points();

// Target j of sub-tap q in combination C (its J index, or -1 past the last):
// a T tap q feeds o = q, a B tap o = 2 - q, M0 and M2 ab, and M1 both aa and
// bb (bit b of j picks between them for the b-th such direction); f1_shift is
// the number of those doublings.  Everything here is a template constant, so
// that every J index is known at compile time.
__host__ __device__ constexpr int f1_target(int C, int q, int j) {
    int idx = 0, bit = 0;
    for (int k = 0; k < 4; ++k) {
        const int c = cbox::cl(C, k), qk = k == 0 ? q % 3 : k == 1 ? (q / 3) % 3 : k == 2 ? (q / 9) % 3 : q / 27;
        int o = 0;
        if (c == 1 && qk == 1) {
            o = ((j >> bit) & 1) ? 2 : 0;
            ++bit;
        } else {
            o = c == 0 ? qk : c == 2 ? 2 - qk : 1;
        }
        idx = idx * 3 + o;
    }
    return j < (1 << bit) ? idx : -1;
}
__host__ __device__ constexpr int f1_shift(int C, int q) {
    int n = 0;
    for (int k = 0; k < 4; ++k) {
        const int qk = k == 0 ? q % 3 : k == 1 ? (q / 3) % 3 : k == 2 ? (q / 9) % 3 : q / 27;
        n += cbox::cl(C, k) == 1 && qk == 1;
    }
    return n;
}

template <int T, int SH>
__device__ __forceinline__ void f1_add(uint64_t J[81], uint64_t v) {
    if constexpr (T >= 0) shl_add(J[T], v, SH);
}

template <int C, int Y_BEGIN, int Y_END, int Q, int... Js>
__device__ __forceinline__ void f1_subtap(const uint64_t *val, uint64_t J[81], std::integer_sequence<int, Js...>) {
    constexpr int q0 = Q % 3, q1 = (Q / 3) % 3, q2 = (Q / 9) % 3, q3 = Q / 27;
    constexpr int Y = cbox::sub_row<1>(q0, q1, q2, q3);
    if constexpr (Y >= Y_BEGIN && Y < Y_END) {
        const uint64_t v = val[(Y - Y_BEGIN) * cbox::patch_w<1>() + cbox::sub_dx<1>(q0, q1, q2, q3)];
        (f1_add<f1_target(C, Q, Js), f1_shift(C, Q)>(J, v), ...);
    }
}

template <int C, int Y_BEGIN, int Y_END, int... Qs>
__device__ __forceinline__ void f1_subtaps(const uint64_t *val, uint64_t J[81], std::integer_sequence<int, Qs...>) {
    (f1_subtap<C, Y_BEGIN, Y_END, Qs>(val, J, std::make_integer_sequence<int, 16>{}), ...);
}

template <int C, int Y_BEGIN, int Y_END>
__device__ __forceinline__ void box_fwd_rows_f1(const uint64_t *__restrict__ p, uint64_t J[81]) {
    using namespace cbox;
    constexpr int PW = patch_w<1>();
    uint64_t val[(Y_END - Y_BEGIN) * PW];
#pragma unroll
    for (int Y = Y_BEGIN; Y < Y_END; ++Y)
#pragma unroll
        for (int X = 0; X < PW; ++X)
            if (kF1Points.hit[X + PW * Y]) val[(Y - Y_BEGIN) * PW + X] = p[X + kPitch * (Y - Y_BEGIN)];
    f1_subtaps<C, Y_BEGIN, Y_END>(val, J, std::make_integer_sequence<int, 81>{});
}

template <int C, int Y_BEGIN, int Y_END>
__device__ __forceinline__ void box_fwd_batch_f1(int base, const uint64_t *__restrict__ s_box, uint64_t J[81]) {
    int b = base + cbox::kPitch * Y_BEGIN;
    asm("" : "+v"(b));
    box_fwd_rows_f1<C, Y_BEGIN, Y_END>(s_box + b, J);
    __builtin_amdgcn_sched_barrier(0);
}

template <int C>
__device__ __forceinline__ void box_fwd_combo_f1(int base, const uint64_t *__restrict__ s_box, uint64_t J[81]) {
    static_assert(cbox::patch_h<1>() == 13, "four row batches cover the patch");
    box_fwd_batch_f1<C, 0, 5>(base, s_box, J);
    box_fwd_batch_f1<C, 5, 7>(base, s_box, J);
    box_fwd_batch_f1<C, 7, 9>(base, s_box, J);
    box_fwd_batch_f1<C, 9, 13>(base, s_box, J);
}

// Start copying box b of the window into the LDS buffer dst (rows of kPitch
// elements) with LDS-direct loads: one instruction moves two box rows as 64
// aligned pairs of elements (lane l: row l / 32, elements 2 (l % 32) and the
// next), wavefront w of WAVES taking the row pairs w, w + WAVES, ...; lanes whose pair
// lies right of the box idle, as do the second-row lanes of a last, unpaired
// row.  The loop runs on wavefront-uniform values only: a pair's window row
// and LDS row advance by scalar adds.  Completion is waited for (vmcnt)
// before the barrier that publishes the box.
template <int WAVES>
__device__ __forceinline__ void box_stage_async(const GatherArgs &a, uint64_t *__restrict__ dst,
                                                const cbox::Box &b, int w) {
    static_assert(cbox::kPitch == 64, "two box rows per 64-lane copy");
    const int lane = threadIdx.x & 63;
    const int col = 2 * (lane & 31);
    const bool upper = lane >= 32;
    if (col >= b.bw) return;
    const int64_t Wp = a.Wp;
    const uint32_t lane_off = (uint32_t)(((upper ? Wp : 0) + col) * 8);
    const char *__restrict__ row =
        reinterpret_cast<const char *>(static_cast<const uint64_t *>(a.G) +
                                       ((int64_t)(b.oy + a.pad_top + 2 * w) * Wp + (b.ox + a.pad_left)));
    const int64_t row_step = 2 * WAVES * Wp * 8;             // WAVES pairs of window rows, bytes
    uint64_t *l = dst + 2 * w * cbox::kPitch;
    const int full = b.bh >> 1;                                  // pairs with both rows in the box
    int pr = w;
    for (; pr < full; pr += WAVES, row += row_step, l += 2 * WAVES * cbox::kPitch)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(row + lane_off),
                                         (__attribute__((address_space(3))) void *)l, 16, 0, 0);
    if ((b.bh & 1) && pr == full && !upper)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(row + lane_off),
                                         (__attribute__((address_space(3))) void *)l, 16, 0, 0);
}

struct BoxTile {
    int x, y;              // pixel
    int R[4];
    int x_lo, x_hi, y_lo, y_hi;
    int Rlo[4], Rhi[4];
    int pad_left;
    int wave;              // wavefront of the pixel in its workgroup (uniform)
    const uint32_t *state; // cbox::pack_state of every thread of the tile, in LDS
};



// Combination I reads buffer I % 2 while combination I + 1 is copied into the
// other one; one barrier per combination publishes the next box and frees the
// current one.
template <int I, class S, int D>
__device__ __forceinline__ void box_fwd_all(const GatherArgs &a, uint64_t *__restrict__ s_box, bool active,
                                            const BoxTile &t, uint64_t J[81]) {
    constexpr int C = cbox::order_at(I);
    const cbox::Box b = cbox::box_of<C, D>(t.x_lo, t.x_hi, t.y_lo, t.y_hi, t.Rlo, t.Rhi, t.pad_left);
    if constexpr (I + 1 < cbox::kCombos) {
        constexpr int Cn = cbox::order_at(I + 1);
        const cbox::Box bn = cbox::box_of<Cn, D>(t.x_lo, t.x_hi, t.y_lo, t.y_hi, t.Rlo, t.Rhi, t.pad_left);
        box_stage_async<S::Waves>(a, s_box + ((I + 1) & 1) * S::Elems, bn, t.wave);
    }
    if constexpr (I == cbox::kEven) {
#pragma unroll
        for (int q = 0; q < 81; ++q) J[q] = 0 - J[q];
    }
    if (active) {
        // the state is read from LDS in every combination, at an index formed
        // afresh from the lane number: neither the state, its decoded fields
        // nor its address stay live across combinations
        const uint32_t st = t.state[64 * t.wave + fresh_lane_id()];
        const int base = (I & 1) * S::Elems + cbox::packed_base<C, D>(st, t.x_lo, t.y_lo, t.Rlo, b);
        if constexpr (D == 0) {
            int lo = base, hi = base + 4 * cbox::kPitch;
            asm("" : "+v"(lo), "+v"(hi));
            box_fwd_combo<C>(s_box + lo, s_box + hi, J);
        } else {
            box_fwd_combo_f1<C>(base, s_box, J);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if constexpr (I + 1 < cbox::kCombos) box_fwd_all<I + 1, S, D>(a, s_box, active, t, J);
}

// The 81-term contraction of J with the phase weights: the value (weights w
// for every direction) and, with DA / DB set, the derivatives with dw_A / dw_B
// in place of w_A / w_B, in one sweep over J that converts each sum to FP64
// as it is consumed (no FP64 copy of J is ever held).  S_L are the partial
// sums over the directions from L on; every result is the nested sum over o0
// (outermost) to o3 (innermost) of the weights times J.  The value and four
// derivatives together need more registers than a wavefront has beside J, so
// a pixel takes two sweeps of two results each (and the value).
template <int DA, int DB, int KEEP, int THREADS>
__device__ __forceinline__ void contract81_sweep(const uint64_t Jr[81], const uint64_t *park, const double w[4][3],
                                                 const double dw[4][3], double &out, double &dA, double &dB) {
    constexpr bool A = DA >= 0, B = DB >= 0;
    // weights of level L: plain, or the derivative's where L is its direction
    auto wt = [&](int which, int L, int o) -> double { return which == L ? dw[L][o] : w[L][o]; };
    double r = 0.0, ra = 0.0, rb = 0.0;
#pragma unroll
    for (int o0 = 0; o0 < 3; ++o0) {
        // sums J[q], q >= KEEP, wait in LDS at park[(q - KEEP) * THREADS + thread]: the
        // index is formed afresh for each third, so that fewer of their loads
        // are hoisted ahead of the sums before them (the registers would not
        // hold them all)
        int own = (int)threadIdx.x;
        asm volatile("" : "+v"(own));
        const auto J = [&](int q) -> uint64_t { return q < KEEP ? Jr[q] : park[(q - KEEP) * THREADS + own]; };
        double s1 = 0.0, s1a = 0.0, s1b = 0.0;
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1) {
            double s2 = 0.0, s2a = 0.0, s2b = 0.0;
#pragma unroll
            for (int o2 = 0; o2 < 3; ++o2) {
                double s3 = 0.0, s3a = 0.0, s3b = 0.0;
#pragma unroll
                for (int o3 = 0; o3 < 3; ++o3) {
                    const double j = -(double)(int64_t)J(cbox::jidx(o0, o1, o2, o3));
                    s3 += w[3][o3] * j;
                    if (A) s3a += wt(DA, 3, o3) * j;
                    if (B) s3b += wt(DB, 3, o3) * j;
                }
                s2 += w[2][o2] * s3;
                if (A) s2a += wt(DA, 2, o2) * (DA == 3 ? s3a : s3);
                if (B) s2b += wt(DB, 2, o2) * (DB == 3 ? s3b : s3);
            }
            s1 += w[1][o1] * s2;
            if (A) s1a += wt(DA, 1, o1) * (DA >= 2 ? s2a : s2);
            if (B) s1b += wt(DB, 1, o1) * (DB >= 2 ? s2b : s2);
        }
        r += w[0][o0] * s1;
        if (A) ra += wt(DA, 0, o0) * (DA >= 1 ? s1a : s1);
        if (B) rb += wt(DB, 0, o0) * (DB >= 1 ? s1b : s1);
        // the next third of J is not touched before this one is consumed
        __builtin_amdgcn_sched_barrier(0);
    }
    out = r;
    dA = ra;
    dB = rb;
}

// Tile-wide min / max of R per direction over the active pixels.
template <int WAVES>
__device__ __forceinline__ void tile_R_range(const int R[4], bool active, int Rlo[4], int Rhi[4]) {
    __shared__ int s_red[WAVES][8];
    int lo[4], hi[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        lo[k] = active ? R[k] : 0x7fffffff;
        hi[k] = active ? R[k] : -0x7fffffff;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            lo[k] = min(lo[k], __shfl_xor(lo[k], d, 64));
            hi[k] = max(hi[k], __shfl_xor(hi[k], d, 64));
        }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s_red[w][k] = lo[k];
            s_red[w][4 + k] = hi[k];
        }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int l = s_red[0][k], h = s_red[0][4 + k];
#pragma unroll
        for (int v = 1; v < WAVES; ++v) {
            l = min(l, s_red[v][k]);
            h = max(h, s_red[v][4 + k]);
        }
        Rlo[k] = __builtin_amdgcn_readfirstlane(l);
        Rhi[k] = __builtin_amdgcn_readfirstlane(h);
    }
}

// DERIV: the call asks for the step derivatives (their sweeps need registers
// the value alone does not, so the kernel without them is its own instance).
// D: the direction frame (cluster_box.h); canon_plane[k] is the step plane of
// the frame's k-th direction.
template <bool BATCH, int TH, bool DERIV, int D = 0>
__global__ __launch_bounds__(64 * FwdShape<TH>::Waves, 2) void k_gather_t2n4_box(
    GatherArgs one, const GatherArgs *__restrict__ table, const int64_t *__restrict__ prefix, int B) {
    using S = FwdShape<TH>;
    __shared__ uint64_t s_box[2 * S::Elems];
    __shared__ uint32_t s_state[64 * S::Waves];
    GatherArgs a;
    int64_t bx, by;
    if (!tile_of_block_xcd<BATCH>(one, table, prefix, B, kFwdTileW, TH, a, bx, by)) return;
    BoxTile t;
    t.x = (int)(bx * kFwdTileW) + fwd_tx(threadIdx.x);
    t.y = (int)(by * TH) + fwd_ty(threadIdx.x);
    const bool active = t.x < a.W && t.y < a.H && selected(a, (int64_t)t.y * a.W + t.x);
    {
        const int64_t HW = a.H * a.W, idx = (int64_t)t.y * a.W + t.x;
        bool bad = false;
        double prod = 1.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float s_raw = active ? a.steps[a.canon_plane[k] * HW + idx] : 1.0f;
            step_check(s_raw, a.max_step, BSF_STEPS_REAL, 2, bad, prod);
            const float s = clamp_step(s_raw, a.max_step);
            t.R[k] = (int)floorf((s - 1.0f) * 0.5f);
        }
        if (active) report_steps(a, bad, prod);
    }
    tile_R_range<S::Waves>(t.R, active, t.Rlo, t.Rhi);
    // no pixel of the tile to filter (outside the image, or in Alg. 2 on the
    // other direction set): the range is empty and the tile is done
    if (t.Rlo[0] > t.Rhi[0]) return;
    t.x_lo = (int)(bx * kFwdTileW);
    t.y_lo = (int)(by * TH);
    t.x_hi = (int)min((int64_t)t.x_lo + kFwdTileW - 1, a.W - 1);
    t.y_hi = (int)min((int64_t)t.y_lo + TH - 1, a.H - 1);
    t.pad_left = (int)a.pad_left;
    t.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    s_state[threadIdx.x] = cbox::pack_state(fwd_tx(threadIdx.x), fwd_ty(threadIdx.x), t.R, t.Rlo, active);
    t.state = s_state;
    if (!cbox::boxes_fit<D>(t.x_lo, t.x_hi, t.y_lo, t.y_hi, t.Rlo, t.Rhi, S::Rows)) {
        if (active) {
            if (a.off[6] == 1) t2n4_pixel<true>(a, t.x, t.y);
            else t2n4_pixel<false>(a, t.x, t.y);
        }
        return;
    }
    uint64_t J[81];
#pragma unroll
    for (int q = 0; q < 81; ++q) J[q] = 0;
    box_stage_async<S::Waves>(
        a, s_box, cbox::box_of<cbox::order_at(0), D>(t.x_lo, t.x_hi, t.y_lo, t.y_hi, t.Rlo, t.Rhi, t.pad_left),
        t.wave);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    box_fwd_all<0, S, D>(a, s_box, active, t, J);
    // The last kPark sums wait in the box buffers, idle now (the last
    // combination ended with a barrier), so that the epilogue's own values fit
    // in registers beside the rest; each thread reads back only its own.
    constexpr int kPark = 36, kKeep = 81 - kPark, kThreads = 64 * S::Waves;
    static_assert(kPark * kThreads <= 2 * S::Elems, "parking space");
#pragma unroll
    for (int q = kKeep; q < 81; ++q) s_box[(q - kKeep) * kThreads + threadIdx.x] = J[q];
    // the pixel's position and phases are formed again here rather than held
    // through the loop
    const int px = t.x_lo + fwd_tx(threadIdx.x), py = t.y_lo + fwd_ty(threadIdx.x);
    if (px >= a.W || py >= a.H || !selected(a, (int64_t)py * a.W + px)) return;
    const int64_t HW = a.H * a.W, idx = (int64_t)py * a.W + px;
    float ph[4], sk[4];
    double den = 1.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float s = clamp_step(a.steps[a.canon_plane[k] * HW + idx], a.max_step);
        const float tt = (s - 1.0f) * 0.5f;
        ph[k] = tt - floorf(tt);
        sk[k] = s;
        den *= (double)s * (double)s;
    }
    const int F = a.status[ST_F_USED];
    // With the derivatives: two sweeps of two derivatives each (directions 0
    // and 1, then 2 and 3; the first also forms the value).  The second reads
    // J and the phases afresh (registers laundered, the parked sums re-read),
    // so that neither its weights nor any conversion of the first are held
    // across the first.  Both epilogues fit in registers beside J.
    double r, d[4], unused;
    {
        double w[4][3], dw[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k) phase_weights(ph[k], w[k], dw[k]);
        if constexpr (DERIV) contract81_sweep<0, 1, kKeep, kThreads>(J, s_box, w, dw, r, d[0], d[1]);
        else contract81_sweep<-1, -1, kKeep, kThreads>(J, s_box, w, dw, r, unused, unused);
    }
    if constexpr (DERIV) {
#pragma unroll
        for (int q = 0; q < kKeep; ++q) asm volatile("" : "+v"(J[q]));
#pragma unroll
        for (int k = 0; k < 4; ++k) asm volatile("" : "+v"(ph[k]));
        asm volatile("" ::: "memory");
        double w[4][3], dw[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k) phase_weights(ph[k], w[k], dw[k]);
        contract81_sweep<2, 3, kKeep, kThreads>(J, s_box, w, dw, unused, d[2], d[3]);
    }
    const double outv = ldexp_neg(r, F) / den;
    if (a.out) a.out[idx] = (float)outv;
    if (DERIV && a.dsteps) {
        // d phi / d s = 1/2, and each step enters prod s twice
#pragma unroll
        for (int k = 0; k < 4; ++k)
            a.dsteps[a.canon_plane[k] * HW + idx] = (float)(0.5 * ldexp_neg(d[k], F) / den - 2.0 * outv / sk[k]);
    }
}

// Plain FP64 counterpart: FP64 running sums and FP64 tap weights
//   T0:(1-p)^2 T1:2p(1-p) T2:p^2 M0:-2p(1-p) M1:-2((1-p)^2+p^2) M2:-2p(1-p) B0:p^2 B1:2p(1-p) B2:(1-p)^2
__device__ __forceinline__ void offsets9(int32_t R, int32_t off, int32_t o[9]) {
    const int32_t t = 2 * R * off, m = -2 * off, b = (-2 * R - 4) * off;
    o[0] = t; o[1] = t + off; o[2] = t + 2 * off;
    o[3] = m; o[4] = m + off; o[5] = m + 2 * off;
    o[6] = b; o[7] = b + off; o[8] = b + 2 * off;
}

template <bool BATCH>
__global__ __launch_bounds__(256) void k_gather_t2n4_fp64(GatherArgs one, const GatherArgs *__restrict__ table,
                                                          const int64_t *__restrict__ prefix, int B) {
    GatherArgs a;
    int64_t bx, by, x, y;
    if (!tile_of_block<BATCH>(one, table, prefix, B, kTile, kTile, a, bx, by)) return;
    if (!pixel_16x16(a, bx, by, x, y) || !selected(a, y * a.W + x)) return;
    check_pixel_steps(a, y * a.W + x);
    const int64_t HW = a.H * a.W, idx = y * a.W + x;
    const double *G = static_cast<const double *>(a.G);
    const int32_t base = (int32_t)((y + a.pad_top) * a.Wp + (x + a.pad_left));
    int32_t o[4][9];
    double w[4][9];
    double den = 1.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float s = clamp_step(a.steps[a.plane[2 * k] * HW + idx], a.max_step);
        const float t = (s - 1.0f) * 0.5f;
        const float Rf = floorf(t);
        const double p = (double)(t - Rf), q = 1.0 - p;
        offsets9((int32_t)Rf, a.off[2 * k], o[k]);
        w[k][0] = q * q; w[k][1] = 2 * p * q; w[k][2] = p * p;
        w[k][3] = -2 * p * q; w[k][4] = -2 * (q * q + p * p); w[k][5] = -2 * p * q;
        w[k][6] = p * p; w[k][7] = 2 * p * q; w[k][8] = q * q;
        den *= (double)s * (double)s;
    }
    double tot = 0.0;
    for (int p0 = 0; p0 < 9; ++p0) {
        double t1 = 0.0;
#pragma unroll
        for (int p1 = 0; p1 < 9; ++p1) {
            double t2 = 0.0;
#pragma unroll
            for (int p2 = 0; p2 < 9; ++p2) {
                const int32_t bb = base + o[0][p0] + o[1][p1] + o[2][p2];
                double t3 = 0.0;
#pragma unroll
                for (int p3 = 0; p3 < 9; ++p3) t3 += w[3][p3] * G[(uint32_t)(bb + o[3][p3])];
                t2 += w[2][p2] * t3;
            }
            t1 += w[1][p1] * t2;
        }
        tot += w[0][p0] * t1;
    }
    if (a.out) a.out[idx] = (float)(tot / den);
}

#ifndef BSF_GATHER_FRAME1_UNIT
// Pixel-tile shape of the kernel run_gather picks for a plan.
struct GatherShape {
    int kind;  // 0 int, 1 generic real, 2 tied order-2 exact, 3 tied order-2 fp64, 4 cluster boxes,
               // 5 cluster boxes of Table 1's directions
    int tile_w, tile_h;
};

GatherShape gather_shape(const Plan &p, const GatherArgs &a) {
    GatherShape s{1, kTile, kTile};
    if (p.mode == BSF_STEPS_INT) {
        s.kind = 0;
    } else if (p.n_dirs == 4 && p.order == 2 && p.tied && p.Hp * p.Wp * 8 < (int64_t(1) << 32)) {
        if (p.arith == BSF_ARITH_FP64) {
            s.kind = 3;
        } else if (a.canon == 1) {
            s.kind = 4;
            s.tile_w = kFwdTileW;
            s.tile_h = tuning().box_h;
        } else if (a.canon == 2) {
            s.kind = 5;
            s.tile_w = kFwdTileW;
            s.tile_h = 8;  // the 13-row patch needs the 38-row boxes
        } else {
            s.kind = 2;
            const bool contig = a.off[6] == 1;
            const int wx = contig ? tuning().gather_wx : 16;
            s.tile_w = wx;
            s.tile_h = 256 / wx;
        }
    }
    return s;
}

template <bool BATCH>
bsf_status launch_gather(const Plan &p, const GatherArgs &one, const GatherArgs *table, const int64_t *prefix, int B,
                         int64_t total_tiles, hipStream_t st) {
    const GatherShape s = gather_shape(p, one);
    dim3 grid;
    if (s.kind == 4 || s.kind == 5 || s.kind == 0 || s.kind == 1) {  // tiles in XCD order (tile_of_block_xcd)
        const int64_t tiles = BATCH ? total_tiles
                                    : ((p.W + s.tile_w - 1) / s.tile_w) * ((p.H + s.tile_h - 1) / s.tile_h);
        grid = dim3((unsigned)xcd_grid(tiles));
    } else if (BATCH) {
        grid = dim3((unsigned)total_tiles);
    } else {
        grid = dim3((unsigned)((p.W + s.tile_w - 1) / s.tile_w), (unsigned)((p.H + s.tile_h - 1) / s.tile_h));
    }
    dim3 block(s.kind == 4 || s.kind == 5 ? 16 * s.tile_h : 256);
    const bool fp64 = p.arith == BSF_ARITH_FP64;
    if (s.kind == 0) {
        if (p.M == 4) {
            if (fp64) hipLaunchKernelGGL((k_gather_int<double, 4, BATCH>), grid, block, 0, st, one, table, prefix, B);
            else hipLaunchKernelGGL((k_gather_int<int64_t, 4, BATCH>), grid, block, 0, st, one, table, prefix, B);
        } else {
            if (fp64) hipLaunchKernelGGL((k_gather_int<double, 0, BATCH>), grid, block, 0, st, one, table, prefix, B);
            else hipLaunchKernelGGL((k_gather_int<int64_t, 0, BATCH>), grid, block, 0, st, one, table, prefix, B);
        }
    } else if (s.kind == 3) {
        hipLaunchKernelGGL((k_gather_t2n4_fp64<BATCH>), grid, block, 0, st, one, table, prefix, B);
    } else if (s.kind == 4) {
        // the batched forward never asks for step derivatives
        const bool deriv = !BATCH && one.dsteps;
        if (s.tile_h == 4) {
            if (deriv) hipLaunchKernelGGL((k_gather_t2n4_box<false, 4, true>), grid, block, 0, st, one, table, prefix, B);
            else hipLaunchKernelGGL((k_gather_t2n4_box<BATCH, 4, false>), grid, block, 0, st, one, table, prefix, B);
        } else {
            if (deriv) hipLaunchKernelGGL((k_gather_t2n4_box<false, 8, true>), grid, block, 0, st, one, table, prefix, B);
            else hipLaunchKernelGGL((k_gather_t2n4_box<BATCH, 8, false>), grid, block, 0, st, one, table, prefix, B);
        }
    } else if (s.kind == 5) {
        if (BATCH) return BSF_E_INVALID;  // the batched forward takes kind 2 for these directions
        return launch_gather_f1(one, grid, block, st);
    } else if (s.kind == 2) {
        const bool contig = one.off[6] == 1;
        if (!contig) {
            if (one.dsteps) hipLaunchKernelGGL((k_gather_t2n4<false, 2, 16, BATCH>), grid, block, 0, st, one, table, prefix, B);
            else hipLaunchKernelGGL((k_gather_t2n4<false, 2, 16, BATCH, false>), grid, block, 0, st, one, table, prefix, B);
        }
        else if (s.tile_w == 8) hipLaunchKernelGGL((k_gather_t2n4<true, 2, 8, BATCH>), grid, block, 0, st, one, table, prefix, B);
        else if (s.tile_w == 32) hipLaunchKernelGGL((k_gather_t2n4<true, 2, 32, BATCH>), grid, block, 0, st, one, table, prefix, B);
        else if (s.tile_w == 64) hipLaunchKernelGGL((k_gather_t2n4<true, 2, 64, BATCH>), grid, block, 0, st, one, table, prefix, B);
        else hipLaunchKernelGGL((k_gather_t2n4<true, 2, 16, BATCH>), grid, block, 0, st, one, table, prefix, B);
    } else {
        if (p.M == 4) {
            if (fp64) hipLaunchKernelGGL((k_gather_real_generic<double, 4, BATCH>), grid, block, 0, st, one, table, prefix, B);
            else hipLaunchKernelGGL((k_gather_real_generic<int64_t, 4, BATCH>), grid, block, 0, st, one, table, prefix, B);
        } else {
            if (fp64) hipLaunchKernelGGL((k_gather_real_generic<double, 0, BATCH>), grid, block, 0, st, one, table, prefix, B);
            else hipLaunchKernelGGL((k_gather_real_generic<int64_t, 0, BATCH>), grid, block, 0, st, one, table, prefix, B);
        }
    }
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

}  // namespace

bsf_status run_bound(const Plan &p, const Src &src, const float *steps, int32_t F_request, int32_t *status,
                     hipStream_t st) {
    BoundJob job{steps, src.kind == SRC_F32 ? static_cast<const float *>(src.img) : nullptr, p.H, p.W, src.pitch,
                 status};
    hipLaunchKernelGGL((k_status_begin<false>), dim3(1), dim3(64), 0, st, job, nullptr, F_request);
    BSF_HIP_CHECK(hipGetLastError());
    int64_t blocks = p.H < 2048 ? p.H : 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_bound<false>), dim3((unsigned)blocks), dim3(256), 0, st, job, nullptr, nullptr, 1, p.planes,
                       p.tied ? p.order : 1, p.mode, p.max_step);
    BSF_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL((k_choose_F<false>), dim3(1), dim3(64), 0, st, job, nullptr, src.kind, p.arith);
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

bsf_status run_gather(const Plan &p, const GatherArgs &a, hipStream_t st) {
    if (p.H == 0 || p.W == 0) return BSF_OK;
    return launch_gather<false>(p, a, nullptr, nullptr, 1, 0, st);
}

int gather_variant(const Plan &p, const GatherArgs &a) {
    const GatherShape s = gather_shape(p, a);
    return s.kind | (s.tile_w << 4) | ((a.off[6] == 1) << 12) | ((p.M == 4) << 13) | (p.arith << 14) |
           (s.tile_h << 16);
}

int64_t gather_tiles(const Plan &p, const GatherArgs &a) {
    const GatherShape s = gather_shape(p, a);
    return ((p.W + s.tile_w - 1) / s.tile_w) * ((p.H + s.tile_h - 1) / s.tile_h);
}

bsf_status run_gather_batch(const Plan &p0, const GatherArgs &a0, const GatherArgs *table, const int64_t *prefix,
                            int B, int64_t total_tiles, hipStream_t st) {
    if (total_tiles <= 0) return BSF_OK;
    return launch_gather<true>(p0, a0, table, prefix, B, total_tiles, st);
}

bsf_status run_bound_batch(const Plan &p0, int img_kind, int32_t F_request, const void *jobs, const int64_t *prefix,
                           int B, int64_t total_rows, hipStream_t st) {
    const BoundJob *bj = static_cast<const BoundJob *>(jobs);
    BoundJob none{};
    hipLaunchKernelGGL((k_status_begin<true>), dim3((unsigned)B), dim3(64), 0, st, none, bj, F_request);
    BSF_HIP_CHECK(hipGetLastError());
    if (total_rows > 0) {
        hipLaunchKernelGGL((k_bound<true>), dim3((unsigned)total_rows), dim3(256), 0, st, none, bj, prefix, B,
                           p0.planes, p0.tied ? p0.order : 1, p0.mode, p0.max_step);
        BSF_HIP_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL((k_choose_F<true>), dim3((unsigned)B), dim3(64), 0, st, none, bj, img_kind, p0.arith);
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

size_t bound_job_bytes() { return sizeof(BoundJob); }

void make_bound_job(const float *steps, const float *img, int64_t H, int64_t W, int64_t pitch, int32_t *status,
                    void *out) {
    BoundJob j{steps, img, H, W, pitch, status};
    memcpy(out, &j, sizeof(j));
}

}  // namespace bsf

#else  // BSF_GATHER_FRAME1_UNIT: the cluster-box kernels of Table 1's directions
}  // namespace

bsf_status launch_gather_f1(const GatherArgs &a, dim3 grid, dim3 block, hipStream_t st) {
    if (a.dsteps) hipLaunchKernelGGL((k_gather_t2n4_box<false, 8, true, 1>), grid, block, 0, st, a, nullptr, nullptr, 1);
    else hipLaunchKernelGGL((k_gather_t2n4_box<false, 8, false, 1>), grid, block, 0, st, a, nullptr, nullptr, 1);
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

}  // namespace bsf
#endif
