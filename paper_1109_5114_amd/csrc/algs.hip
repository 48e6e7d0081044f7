// Algorithms 1 and 2 of the paper on top of the space-variant filter.
//
// Alg. 1 (better accuracy): sigma^2 is half the bound of condition2, taken as
// the smallest over the image because its first filtering pass is one global
// convolution; the image is filtered with the isotropic box spline of scales
// sqrt(6) sigma, then with every pixel's scales for C - sigma^2 I (minimum
// kurtosis).  By Prop. 1 and Prop. 2 this is one space-variant filter whose
// kernels have covariance C.
//
// Alg. 2 (improved elongation): running sums along both four-direction sets,
// the one of Section 1.1 and the one of Alg. 3; each pixel takes the box spline
// whose axes lie nearer its orientation (the sector rule), its scales for C in
// that box spline, and its finite difference on that set's running sums.
#include <math.h>
#include <string.h>

#include <mutex>

#include "bsf_common.h"

namespace bsf {
namespace {

enum AlgStatusWord : int {
    ST_ALG_BMIN_BITS = 24,  // scratch: float bits of min over pixels of the condition2 bound (clamped at 0)
    ST_ALG_SIGMA2 = 25,     // float bits of the sigma^2 of Alg. 1
};

// The status blocks of the passes start clean on every call; the caller's
// block keeps its sticky flags and gets the reduction words reset.
__global__ void k_alg_begin(int32_t *top, int32_t *s1, int32_t *s2) {
    const int i = threadIdx.x;
    if (blockIdx.x != 0 || i >= ST_WORDS) return;
    if (s1) s1[i] = 0;
    if (s2) s2[i] = 0;
    if (i == 0) {
        top[ST_ALG_BMIN_BITS] = 0x7f800000;  // +infinity
        top[ST_ALG_SIGMA2] = 0;
    }
}

__global__ void k_alg_clear_block(int32_t *s) {
    if (blockIdx.x == 0 && threadIdx.x < ST_WORDS) s[threadIdx.x] = 0;
}

// The top status word of a composed call: flags OR-ed, the smallest F and the
// largest bound of its passes.
__global__ void k_alg_merge(int32_t *top, const int32_t *s1, const int32_t *s2) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    top[ST_FLAGS] |= s1[ST_FLAGS] | s2[ST_FLAGS];
    top[ST_F_USED] = min(s1[ST_F_USED], s2[ST_F_USED]);
    top[ST_LOG2_BOUND] = max(s1[ST_LOG2_BOUND], s2[ST_LOG2_BOUND]);
}

// condition2 at every pixel: half of C11 + C22 - (e + 1)/(e - 1) sqrt(D), with
// e = e(phi) of eq. boundE at C's orientation phi; min-reduced (clamped at 0,
// non-finite covariances raise the range flag and count as 0).
__global__ __launch_bounds__(256) void k_alg1_bound(const float *__restrict__ cov, int64_t HW, int32_t *top) {
    __shared__ unsigned s_m[4];
    unsigned m = 0x7f800000u;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < HW; i += (int64_t)gridDim.x * blockDim.x) {
        const double c11 = cov[i], c12 = cov[HW + i], c22 = cov[2 * HW + i];
        const double phi = 0.5 * atan2(2.0 * c12, c11 - c22);
        const double sn = sin(phi), cs = cos(phi);
        double f = 1.0;  // (e + 1)/(e - 1); e is infinite along the axes
        if (sn != 0.0 && cs != 0.0) {
            const double t = 0.5 * fabs(sn / cs - cs / sn), q = sqrt(1.0 + t * t);
            const double den = 1.0 + t - q;
            if (den > 0.0) {
                const double e = (1.0 + t + q) / den;
                f = (e + 1.0) / (e - 1.0);
            }
        }
        double b = 0.5 * (c11 + c22 - f * sqrt((c11 - c22) * (c11 - c22) + 4.0 * c12 * c12));
        if (!(b == b) || !(fabs(c11) + fabs(c12) + fabs(c22) < 1e300)) {
            bad = true;
            b = 0.0;
        }
        m = min(m, __float_as_uint((float)fmax(b, 0.0)));
    }
    for (int d = 32; d >= 1; d >>= 1) m = min(m, (unsigned)__shfl_xor((int)m, d, 64));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr((unsigned *)&top[ST_FLAGS], BSF_FLAG_RANGE);
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; ++k) m = min(m, s_m[k]);
        atomicMin((unsigned *)&top[ST_ALG_BMIN_BITS], m);
    }
}

// sigma^2 = half the smallest bound; the isotropic pass's steps: scales
// sqrt(6) sigma per direction, i.e. sqrt(6 sigma^2 / r) lattice steps on the
// axes and sqrt(3 sigma^2 / r) on the diagonals for each of r copies.
__global__ __launch_bounds__(256) void k_alg1_iso_steps(int32_t *top, float *__restrict__ steps, int64_t HW,
                                                        int planes, int order, int diag_plane_mask, float max_step) {
    const float bmin = __uint_as_float((unsigned)top[ST_ALG_BMIN_BITS]);
    const float s2 = (bmin <= 3.4e38f) ? 0.5f * bmin : 0.0f;
    if (blockIdx.x == 0 && threadIdx.x == 0) top[ST_ALG_SIGMA2] = __float_as_int(s2);
    const float axis = fminf(fmaxf(sqrtf(6.0f * s2 / order), 1.0f), max_step);
    const float diag = fminf(fmaxf(sqrtf(3.0f * s2 / order), 1.0f), max_step);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < HW * planes;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(i / HW);
        steps[i] = (diag_plane_mask >> q) & 1 ? diag : axis;
    }
}

struct AlgLayout {
    int32_t *top;
    char *ws1, *ws2;
    float *steps1, *steps2, *mid;
    uint8_t *sel;
    size_t bytes;
};

size_t plane_bytes(const Plan &p) { return align_up((size_t)p.planes * p.H * p.W * sizeof(float)); }

AlgLayout alg_layout(const Plan &p1, const Plan *p2, bool want_mid, bool want_sel, char *base) {
    AlgLayout L{};
    size_t off = kStatusBytes;
    const size_t w1 = align_up(ws_bytes_for(p1, true));
    L.ws1 = base + off;
    off += w1;
    if (p2) {
        L.ws2 = base + off;
        off += align_up(ws_bytes_for(*p2, true));
    }
    L.steps1 = reinterpret_cast<float *>(base + off);
    off += plane_bytes(p1);
    L.steps2 = reinterpret_cast<float *>(base + off);
    off += plane_bytes(p2 ? *p2 : p1);
    if (want_mid) {
        L.mid = reinterpret_cast<float *>(base + off);
        off += align_up((size_t)p1.H * p1.W * sizeof(float));
    }
    if (want_sel) {
        L.sel = reinterpret_cast<uint8_t *>(base + off);
        off += align_up((size_t)p1.H * p1.W);
    }
    L.top = reinterpret_cast<int32_t *>(base);
    L.bytes = off;
    return L;
}

// One forward pass of the filter through a single-image workspace region.
bsf_status one_pass(const Plan &p, int src_kind, int32_t frac_bits, const void *img, int64_t pitch,
                    const float *steps, float *out, const uint8_t *sel, int sel_id, char *ws, hipStream_t st) {
    int32_t *status = reinterpret_cast<int32_t *>(ws);
    void *G = ws + kStatusBytes;
    void *aux = ws + kStatusBytes + align_up(p.g_bytes);
    Src src{img, src_kind, p.H, p.W, pitch, p.pad_top, p.pad_left};
    bsf_status r = run_bound(p, src, steps, src_kind == SRC_F32 ? frac_bits : 0, status, st);
    if (r != BSF_OK) return r;
    r = run_preintegrate(p, src, G, aux, status, st);
    if (r != BSF_OK) return r;
    GatherArgs a = gather_args(p, G, steps, out, nullptr, nullptr, nullptr, status);
    a.sel = sel;
    a.sel_id = sel_id;
    return run_gather(p, a, st);
}

// A second stream per device, on which Alg. 2 runs its second direction set
// beside the first: forked from the caller's stream and joined back into it by
// events (graph capture follows the fork and the join too).  Created on the
// first call on a device and kept for the process, at the default priority.
// The lock keeps the record / wait pairs of concurrent calls from
// interleaving.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
constexpr int kMaxDevices = 64;
std::mutex g_side_lock;
SideStream g_side[kMaxDevices];

bsf_status side_stream_locked(SideStream *&out) {
    int dev = 0;
    BSF_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return BSF_E_UNSUPPORTED;
    SideStream &ss = g_side[dev];
    if (!ss.s) {
        BSF_HIP_CHECK(hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking));
        BSF_HIP_CHECK(hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming));
        BSF_HIP_CHECK(hipEventCreateWithFlags(&ss.join, hipEventDisableTiming));
    }
    out = &ss;
    return BSF_OK;
}

int src_kind(bsf_dtype d) { return d == BSF_U8 ? SRC_U8 : d == BSF_U16 ? SRC_U16 : d == BSF_F32 ? SRC_F32 : -1; }

bsf_config with_dirs(const bsf_config &c, const int dirs[8]) {
    bsf_config o = c;
    o.n_dirs = 4;
    memset(o.dirs, 0, sizeof(o.dirs));
    for (int i = 0; i < 8; ++i) o.dirs[i] = dirs[i];
    return o;
}

const int kBank1[8] = {1, 0, 0, 1, 1, 1, 1, -1};
const int kBank2[8] = {2, 1, 1, 2, 1, -2, 2, -1};

bool is_bank1(const Plan &p) {
    // any order of the four directions of Section 1.1
    int found = 0;
    for (int k = 0; k < 4 && p.n_dirs == 4; ++k)
        for (int c = 0; c < 4; ++c)
            if (p.dx[k] == kBank1[2 * c] && p.dy[k] == kBank1[2 * c + 1]) ++found;
    return found == 4;
}

bsf_status alg1_plan(const bsf_config *cfg, int64_t H, int64_t W, Plan &p) {
    bsf_status r = make_plan(cfg, H, W, &p);
    if (r != BSF_OK) return r;
    if (!is_bank1(p) || p.mode != BSF_STEPS_REAL) return BSF_E_UNSUPPORTED;
    return BSF_OK;
}

bsf_status alg2_plans(const bsf_config *cfg, int64_t H, int64_t W, Plan &p1, Plan &p2) {
    if (!cfg) return BSF_E_INVALID;
    const bsf_config c1 = with_dirs(*cfg, kBank1), c2 = with_dirs(*cfg, kBank2);
    bsf_status r = make_plan(&c1, H, W, &p1);
    if (r != BSF_OK) return r;
    r = make_plan(&c2, H, W, &p2);
    if (r != BSF_OK) return r;
    if (p1.mode != BSF_STEPS_REAL) return BSF_E_UNSUPPORTED;
    return BSF_OK;
}

int64_t grid_of(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return b < 1 ? 1 : b > 8192 ? 8192 : b;
}

}  // namespace
}  // namespace bsf

using namespace bsf;

extern "C" {

size_t bsf_alg1_workspace_bytes(const bsf_config *cfg, int64_t H, int64_t W) {
    Plan p;
    if (alg1_plan(cfg, H, W, p) != BSF_OK) return 0;
    return alg_layout(p, nullptr, true, false, nullptr).bytes;
}

bsf_status bsf_filter_alg1(const bsf_config *cfg, const float *img, int64_t H, int64_t W, int64_t pitch,
                           const float *cov, float *out, void *ws, size_t ws_bytes, void *stream) {
    Plan p;
    bsf_status r = alg1_plan(cfg, H, W, p);
    if (r != BSF_OK) return r;
    if (!ws || pitch < W || (H * W > 0 && (!img || !cov || !out))) return BSF_E_INVALID;
    AlgLayout L = alg_layout(p, nullptr, true, false, static_cast<char *>(ws));
    if (ws_bytes < L.bytes) return BSF_E_WORKSPACE;
    if (H * W == 0) return BSF_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t HW = H * W;
    int32_t *s1 = reinterpret_cast<int32_t *>(L.ws1);
    int32_t *top = L.top;
    // sigma^2 from the smallest condition2 bound
    hipLaunchKernelGGL(k_alg_begin, dim3(1), dim3(64), 0, st, top, s1, (int32_t *)nullptr);
    BSF_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_alg1_bound, dim3((unsigned)grid_of(HW)), dim3(256), 0, st, cov, HW, top);
    BSF_HIP_CHECK(hipGetLastError());
    // pass 1: the isotropic box spline of scales sqrt(6) sigma
    int diag_mask = 0;
    const int per = p.tied ? 1 : p.order;
    for (int k = 0; k < 4; ++k)
        if (p.dx[k] != 0 && p.dy[k] != 0)
            for (int q = 0; q < per; ++q) diag_mask |= 1 << (k * per + q);
    hipLaunchKernelGGL(k_alg1_iso_steps, dim3((unsigned)grid_of(HW * p.planes)), dim3(256), 0, st, top, L.steps1, HW,
                       p.planes, p.order, diag_mask, p.max_step);
    BSF_HIP_CHECK(hipGetLastError());
    r = one_pass(p, SRC_F32, cfg->frac_bits, img, pitch, L.steps1, L.mid, nullptr, 0, L.ws1, st);
    if (r != BSF_OK) return r;
    // pass 2: every pixel's scales for C - sigma^2 I
    CovBank b;
    r = make_cov_bank(p, &b);
    if (r != BSF_OK) return r;
    r = run_cov_to_steps(p, b, nullptr, cov, reinterpret_cast<const float *>(top + ST_ALG_SIGMA2), 0.0f, L.steps2,
                         nullptr, nullptr, top, st);
    if (r != BSF_OK) return r;
    hipLaunchKernelGGL(k_alg_merge, dim3(1), dim3(64), 0, st, top, s1, s1);
    BSF_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_alg_clear_block, dim3(1), dim3(64), 0, st, s1);
    BSF_HIP_CHECK(hipGetLastError());
    r = one_pass(p, SRC_F32, cfg->frac_bits, L.mid, W, L.steps2, out, nullptr, 0, L.ws1, st);
    if (r != BSF_OK) return r;
    hipLaunchKernelGGL(k_alg_merge, dim3(1), dim3(64), 0, st, top, s1, s1);
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

size_t bsf_alg2_workspace_bytes(const bsf_config *cfg, int64_t H, int64_t W) {
    Plan p1, p2;
    if (alg2_plans(cfg, H, W, p1, p2) != BSF_OK) return 0;
    return alg_layout(p1, &p2, false, true, nullptr).bytes;
}

bsf_status bsf_filter_alg2(const bsf_config *cfg, bsf_dtype dtype, const void *img, int64_t H, int64_t W,
                           int64_t pitch, const float *cov, float *out, uint8_t *bank_out, void *ws, size_t ws_bytes,
                           void *stream) {
    Plan p1, p2;
    bsf_status r = alg2_plans(cfg, H, W, p1, p2);
    if (r != BSF_OK) return r;
    const int kind = src_kind(dtype);
    if (kind < 0 || !ws || pitch < W || (H * W > 0 && (!img || !cov || !out))) return BSF_E_INVALID;
    AlgLayout L = alg_layout(p1, &p2, false, true, static_cast<char *>(ws));
    if (ws_bytes < L.bytes) return BSF_E_WORKSPACE;
    if (H * W == 0) return BSF_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int32_t *s1 = reinterpret_cast<int32_t *>(L.ws1), *s2 = reinterpret_cast<int32_t *>(L.ws2);
    uint8_t *sel = bank_out ? bank_out : L.sel;
    hipLaunchKernelGGL(k_alg_begin, dim3(1), dim3(64), 0, st, L.top, s1, s2);
    BSF_HIP_CHECK(hipGetLastError());
    CovBank b1, b2;
    r = make_cov_bank(p1, &b1);
    if (r != BSF_OK) return r;
    r = make_cov_bank(p2, &b2);
    if (r != BSF_OK) return r;
    // sector, scales of the pixel's own box spline; the other set's steps are 1
    r = run_cov_to_steps(p1, b1, &b2, cov, nullptr, 0.0f, L.steps1, L.steps2, sel, L.top, st);
    if (r != BSF_OK) return r;
    // the two sets' passes touch disjoint workspace regions and output pixels:
    // the second runs on the side stream while the first runs on st
    {
        std::lock_guard<std::mutex> lock(g_side_lock);
        SideStream *ss = nullptr;
        r = side_stream_locked(ss);
        if (r != BSF_OK) return r;
        BSF_HIP_CHECK(hipEventRecord(ss->fork, st));
        BSF_HIP_CHECK(hipStreamWaitEvent(ss->s, ss->fork, 0));
        r = one_pass(p2, kind, cfg->frac_bits, img, pitch, L.steps2, out, sel, 1, L.ws2, ss->s);
        const bsf_status r1 = one_pass(p1, kind, cfg->frac_bits, img, pitch, L.steps1, out, sel, 0, L.ws1, st);
        // join even when a launch failed, so that st never runs ahead of work on the side stream
        BSF_HIP_CHECK(hipEventRecord(ss->join, ss->s));
        BSF_HIP_CHECK(hipStreamWaitEvent(st, ss->join, 0));
        if (r != BSF_OK) return r;
        if (r1 != BSF_OK) return r1;
    }
    hipLaunchKernelGGL(k_alg_merge, dim3(1), dim3(64), 0, st, L.top, s1, s2);
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

}  // extern "C"
