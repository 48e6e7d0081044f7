// C ABI of libbsf: validation, planning of the running-sum window, workspace
// layout and launch sequencing.  Declarations and contracts: include/bsf.h.
#include <math.h>
#include <string.h>

#include <mutex>

#include "bsf_common.h"

namespace bsf {

namespace {

int gcd_int(int a, int b) {
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
        int t = a % b;
        a = b;
        b = t;
    }
    return a;
}

__global__ void k_set_F(int32_t *status, int32_t F) {
    if (threadIdx.x == 0 && blockIdx.x == 0) status[ST_F_USED] = F;
}

__global__ void k_clear_status(int32_t *status) {
    if (blockIdx.x == 0 && threadIdx.x < ST_WORDS) status[threadIdx.x] = 0;
}

int src_kind_of(bsf_dtype d) {
    switch (d) {
    case BSF_U8: return SRC_U8;
    case BSF_U16: return SRC_U16;
    case BSF_F32: return SRC_F32;
    }
    return -1;
}

}  // namespace

bsf_status make_plan(const bsf_config *cfg, int64_t H, int64_t W, Plan *p) {
    if (!cfg || !p) return BSF_E_INVALID;
    memset(p, 0, sizeof(*p));
    if (cfg->n_dirs < 1 || cfg->n_dirs > BSF_MAX_DIRS) return BSF_E_INVALID;
    if (cfg->order < 1) return BSF_E_INVALID;
    if (cfg->order > 4) return BSF_E_UNSUPPORTED;
    if (cfg->n_dirs * cfg->order > BSF_MAX_FACTORS) return BSF_E_INVALID;
    if (cfg->mode != BSF_STEPS_INT && cfg->mode != BSF_STEPS_REAL) return BSF_E_INVALID;
    if (cfg->arith != BSF_ARITH_EXACT && cfg->arith != BSF_ARITH_FP64) return BSF_E_INVALID;
    if (!(cfg->max_step >= 1.0f) || !isfinite(cfg->max_step) || cfg->max_step > 1.0e6f) return BSF_E_INVALID;
    if (cfg->frac_bits < -1 || cfg->frac_bits > 62) return BSF_E_INVALID;
    if (H < 0 || W < 0 || H > (int64_t(1) << 18) || W > (int64_t(1) << 18)) return BSF_E_INVALID;
    // Any directions, in any order: a line of a running sum starts at zero
    // where it enters the window, and what that truncation leaves out is, on
    // the window, a polynomial of degree < r along the pass's own lines,
    // carried through the later passes in a form that every tap combination
    // (r-th differences along every direction) cancels, as long as all taps
    // lie in the window.
    for (int k = 0; k < cfg->n_dirs; ++k) {
        const int dx = cfg->dirs[2 * k], dy = cfg->dirs[2 * k + 1];
        if (dx == 0 && dy == 0) return BSF_E_INVALID;
        if (gcd_int(dx, dy) != 1) return BSF_E_INVALID;              // primitive
        if (dx < 0 || (dx == 0 && dy < 0)) return BSF_E_INVALID;     // canonical sign
        if (dx > 64 || dy > 64 || dy < -64) return BSF_E_INVALID;
        for (int l = 0; l < k; ++l)
            if (p->dx[l] == dx && p->dy[l] == dy) return BSF_E_INVALID;  // each direction once
        p->dx[k] = dx;
        p->dy[k] = dy;
    }
    p->n_dirs = cfg->n_dirs;
    p->order = cfg->order;
    p->M = cfg->n_dirs * cfg->order;
    p->tied = cfg->tied ? 1 : 0;
    p->mode = cfg->mode;
    p->arith = cfg->arith;
    p->planes = p->tied ? p->n_dirs : p->M;
    p->max_step = cfg->max_step;
    p->R_max = (int)floorf((cfg->max_step - 1.0f) * 0.5f);
    p->H = H;
    p->W = W;
    // Every tap of factor j lies at m u_j with m in [-(R+2), R+1] (both step
    // modes), so direction k reaches [-r(R+2), r(R+1)] lattice steps.
    const int64_t lo = (int64_t)p->order * (p->R_max + 2), hi = (int64_t)p->order * (p->R_max + 1);
    int64_t left = 0, right = 0, top = 0, bottom = 0;
    for (int k = 0; k < p->n_dirs; ++k) {
        const int64_t dx = p->dx[k], dy = p->dy[k];
        left += lo * dx;
        right += hi * dx;
        if (dy > 0) {
            top += lo * dy;
            bottom += hi * dy;
        } else {
            top += hi * (-dy);
            bottom += lo * (-dy);
        }
    }
    p->pad_top = top;
    p->pad_bottom = bottom;
    p->pad_left = left;
    // one spare column past the rightmost tap: the gather copies boxes of the
    // window in aligned pairs of elements
    int64_t Wp = W + left + right + 1;
    Wp = (Wp + 15) / 16 * 16;
    p->pad_right = Wp - W - left;
    p->Wp = Wp;
    p->Hp = H + top + bottom;
    p->g_bytes = (size_t)p->Hp * (size_t)p->Wp * 8;
    p->scan_aux_bytes = scan_aux_bytes(*p);
    return BSF_OK;
}

}  // namespace bsf

namespace bsf {

Tuning g_tuning{16, 64, 8};
const Tuning &tuning() { return g_tuning; }

size_t ws_bytes_for(const Plan &p, bool g_internal) {
    return kStatusBytes + (g_internal ? align_up(p.g_bytes) : 0) + p.scan_aux_bytes;
}

GatherArgs gather_args(const Plan &p, const void *G, const float *steps, float *out, int64_t *num, int64_t *den,
                       float *dsteps, const int32_t *status) {
    GatherArgs a;
    memset(&a, 0, sizeof(a));
    a.G = G;
    a.Wp = p.Wp;
    a.pad_top = p.pad_top;
    a.pad_left = p.pad_left;
    a.H = p.H;
    a.W = p.W;
    a.steps = steps;
    a.out = out;
    a.out_num = num;
    a.out_den = den;
    a.dsteps = dsteps;
    a.status = status;
    a.max_step = p.max_step;
    a.M = p.M;
    a.order = p.order;
    a.tied = p.tied;
    a.n_dirs = p.n_dirs;
    a.mode = p.mode;
    // Factor order: directions in config order, except that for the tied
    // four-direction order-2 kernel a direction with window offset +1 goes last,
    // so its taps are contiguous.  The result does not depend on the order.
    int perm[BSF_MAX_DIRS];
    for (int k = 0; k < p.n_dirs; ++k) perm[k] = k;
    if (p.n_dirs == 4 && p.order == 2 && p.tied) {
        for (int k = 0; k < p.n_dirs; ++k)
            if (p.dx[k] == 1 && p.dy[k] == 0) {
                perm[k] = perm[3];
                perm[3] = k;
                break;
            }
    }
    if (p.n_dirs == 4) {
        // the two frames of the cluster-box kernels: Section 1.1's directions
        // and those of Table 1
        static const int kFrame[2][4][2] = {{{1, 0}, {0, 1}, {1, 1}, {1, -1}}, {{2, 1}, {1, 2}, {1, -2}, {2, -1}}};
        for (int f = 0; f < 2 && !a.canon; ++f) {
            int found = 0;
            for (int c = 0; c < 4; ++c)
                for (int k = 0; k < 4; ++k)
                    if (p.dx[k] == kFrame[f][c][0] && p.dy[k] == kFrame[f][c][1]) {
                        a.canon_plane[c] = k;
                        ++found;
                    }
            if (found == 4) a.canon = f + 1;
        }
    }
    for (int kk = 0; kk < p.n_dirs; ++kk) {
        const int k = perm[kk];
        for (int q = 0; q < p.order; ++q) {
            const int j = kk * p.order + q;
            a.off[j] = (int32_t)(p.dy[k] * p.Wp + p.dx[k]);
            a.plane[j] = p.tied ? k : k * p.order + q;
        }
    }
    return a;
}

}  // namespace bsf

using namespace bsf;

extern "C" {

bsf_status bsf_workspace_init(void *ws, size_t ws_bytes, void *stream) {
    if (!ws || ws_bytes < kStatusBytes) return BSF_E_WORKSPACE;
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                       static_cast<int32_t *>(ws));
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

bsf_status bsf_plan(const bsf_config *cfg, int64_t H, int64_t W, bsf_geometry *geo) {
    if (!geo) return BSF_E_INVALID;
    Plan p;
    bsf_status r = make_plan(cfg, H, W, &p);
    if (r != BSF_OK) return r;
    geo->pad_top = p.pad_top;
    geo->pad_bottom = p.pad_bottom;
    geo->pad_left = p.pad_left;
    geo->pad_right = p.pad_right;
    geo->win_h = p.Hp;
    geo->win_w = p.Wp;
    geo->g_bytes = p.g_bytes;
    geo->workspace_bytes = ws_bytes_for(p, true);
    geo->workspace_bytes_g_external = ws_bytes_for(p, false);
    return BSF_OK;
}

bsf_status bsf_preintegrate(const bsf_config *cfg, bsf_dtype dtype, const void *img, int64_t H, int64_t W,
                            int64_t pitch, int32_t F, void *G, void *ws, size_t ws_bytes, void *stream) {
    Plan p;
    bsf_status r = make_plan(cfg, H, W, &p);
    if (r != BSF_OK) return r;
    const int kind = src_kind_of(dtype);
    if (kind < 0) return BSF_E_INVALID;
    if (pitch < W || !G || !ws || (H * W > 0 && !img)) return BSF_E_INVALID;
    if (F < 0 || F > 62) return BSF_E_INVALID;
    if (ws_bytes < ws_bytes_for(p, false)) return BSF_E_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int32_t *status = static_cast<int32_t *>(ws);
    void *aux = static_cast<char *>(ws) + kStatusBytes;
    hipLaunchKernelGGL(k_set_F, dim3(1), dim3(64), 0, st, status, kind == SRC_F32 ? F : 0);
    BSF_HIP_CHECK(hipGetLastError());
    Src src{img, kind, H, W, pitch, p.pad_top, p.pad_left};
    return run_preintegrate(p, src, G, aux, status, st);
}

}  // extern "C"

namespace {

// Workspace layout: [status 256 B][G when internal][scan carries].
struct WsLayout {
    int32_t *status;
    void *G;
    void *aux;
};

WsLayout ws_layout(const Plan &p, void *ws, void *G_ext) {
    WsLayout L;
    char *wsp = static_cast<char *>(ws);
    L.status = reinterpret_cast<int32_t *>(wsp);
    wsp += kStatusBytes;
    L.G = G_ext;
    if (!L.G) {
        L.G = wsp;
        wsp += align_up(p.g_bytes);
    }
    L.aux = wsp;
    return L;
}

bsf_status prepare_impl(const bsf_config *cfg, bsf_dtype dtype, const void *img, int64_t H, int64_t W,
                        int64_t pitch, const float *steps, void *G_ext, void *ws, size_t ws_bytes, void *stream,
                        Plan &p, WsLayout &L) {
    bsf_status r = make_plan(cfg, H, W, &p);
    if (r != BSF_OK) return r;
    const int kind = src_kind_of(dtype);
    if (kind < 0) return BSF_E_INVALID;
    if (pitch < W || !ws) return BSF_E_INVALID;
    if (H * W > 0 && (!img || !steps)) return BSF_E_INVALID;
    if (ws_bytes < ws_bytes_for(p, G_ext == nullptr)) return BSF_E_WORKSPACE;
    L = ws_layout(p, ws, G_ext);
    if (H * W == 0) return BSF_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Src src{img, kind, H, W, pitch, p.pad_top, p.pad_left};
    r = run_bound(p, src, steps, kind == SRC_F32 ? cfg->frac_bits : 0, L.status, st);
    if (r != BSF_OK) return r;
    return run_preintegrate(p, src, L.G, L.aux, L.status, st);
}

bsf_status apply_checks(const Plan &p, bsf_dtype dtype, int64_t *out_num, int64_t *out_den, float *dsteps) {
    if (src_kind_of(dtype) < 0) return BSF_E_INVALID;
    if (out_num && (p.mode != BSF_STEPS_INT || p.arith != BSF_ARITH_EXACT)) return BSF_E_INVALID;
    if (out_den && p.mode != BSF_STEPS_INT) return BSF_E_INVALID;
    if (dsteps && p.mode != BSF_STEPS_REAL) return BSF_E_INVALID;
    return BSF_OK;
}

}  // namespace

extern "C" {

bsf_status bsf_forward_prepare(const bsf_config *cfg, bsf_dtype dtype, const void *img, int64_t H, int64_t W,
                               int64_t pitch, const float *steps, void *G, void *ws, size_t ws_bytes,
                               void *stream) {
    Plan p;
    WsLayout L;
    return prepare_impl(cfg, dtype, img, H, W, pitch, steps, G, ws, ws_bytes, stream, p, L);
}

bsf_status bsf_forward_apply(const bsf_config *cfg, bsf_dtype dtype, int64_t H, int64_t W, const float *steps,
                             const void *G, float *out, int64_t *out_num, int64_t *out_den, float *dout_dsteps,
                             void *ws, size_t ws_bytes, void *stream) {
    Plan p;
    bsf_status r = make_plan(cfg, H, W, &p);
    if (r != BSF_OK) return r;
    r = apply_checks(p, dtype, out_num, out_den, dout_dsteps);
    if (r != BSF_OK) return r;
    if (!ws || (H * W > 0 && !steps)) return BSF_E_INVALID;
    if (ws_bytes < ws_bytes_for(p, G == nullptr)) return BSF_E_WORKSPACE;
    WsLayout L = ws_layout(p, ws, const_cast<void *>(G));
    if (H * W == 0) return BSF_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the taps check these steps themselves (range, and headroom at the stored F)
    GatherArgs a = gather_args(p, L.G, steps, out, out_num, out_den, dout_dsteps, L.status);
    return run_gather(p, a, st);
}

bsf_status bsf_filter_varying(const bsf_config *cfg, bsf_dtype dtype, const void *img, int64_t H, int64_t W,
                              int64_t pitch, const float *steps, float *out, int64_t *out_num, int64_t *out_den,
                              float *dout_dsteps, void *G_save, void *ws, size_t ws_bytes, void *stream) {
    Plan p;
    bsf_status r = make_plan(cfg, H, W, &p);
    if (r != BSF_OK) return r;
    r = apply_checks(p, dtype, out_num, out_den, dout_dsteps);
    if (r != BSF_OK) return r;
    WsLayout L;
    r = prepare_impl(cfg, dtype, img, H, W, pitch, steps, G_save, ws, ws_bytes, stream, p, L);
    if (r != BSF_OK || H * W == 0) return r;
    GatherArgs a = gather_args(p, L.G, steps, out, out_num, out_den, dout_dsteps, L.status);
    return run_gather(p, a, static_cast<hipStream_t>(stream));
}

size_t bsf_backward_workspace_bytes(const bsf_config *cfg, int64_t H, int64_t W) {
    Plan p;
    if (make_plan(cfg, H, W, &p) != BSF_OK) return 0;
    return ws_bytes_for(p, true);
}

bsf_status bsf_filter_backward(const bsf_config *cfg, int64_t H, int64_t W, const float *steps, const float *gout,
                               const float *dout_dsteps, float *grad_img, float *grad_steps, void *ws,
                               size_t ws_bytes, void *stream) {
    Plan p;
    bsf_status r = make_plan(cfg, H, W, &p);
    if (r != BSF_OK) return r;
    if (p.mode != BSF_STEPS_REAL || p.arith != BSF_ARITH_EXACT) return BSF_E_UNSUPPORTED;
    if (!ws) return BSF_E_INVALID;
    if (H * W > 0 && (!steps || !gout)) return BSF_E_INVALID;
    if (grad_steps && !dout_dsteps) return BSF_E_INVALID;
    if (ws_bytes < ws_bytes_for(p, true)) return BSF_E_WORKSPACE;
    if (H * W == 0 || (!grad_img && !grad_steps)) return BSF_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    WsLayout L = ws_layout(p, ws, nullptr);
    if (grad_img) {
        AdjointArgs a;
        memset(&a, 0, sizeof(a));
        const GatherArgs ga = gather_args(p, nullptr, steps, nullptr, nullptr, nullptr, nullptr, L.status);
        a.Ghat = static_cast<int64_t *>(L.G);
        a.Wp = p.Wp;
        a.pad_top = p.pad_top;
        a.pad_left = p.pad_left;
        a.H = H;
        a.W = W;
        a.steps = steps;
        a.gout = gout;
        a.status = L.status;
        a.max_step = p.max_step;
        a.M = p.M;
        a.order = p.order;
        a.tied = p.tied;
        a.n_dirs = p.n_dirs;
        memcpy(a.off, ga.off, sizeof(a.off));
        memcpy(a.plane, ga.plane, sizeof(a.plane));
        a.canon = ga.canon;
        memcpy(a.canon_plane, ga.canon_plane, sizeof(a.canon_plane));
        for (int k = 0; k < p.n_dirs; ++k) {
            a.adx[k] = p.dx[k] < 0 ? -p.dx[k] : p.dx[k];
            a.ady[k] = p.dy[k] < 0 ? -p.dy[k] : p.dy[k];
        }
        r = run_adjoint_scatter(p, a, L.status, L.aux, st);
        if (r != BSF_OK) return r;
        r = run_preintegrate_transpose(p, L.G, L.aux, L.status, st);
        if (r != BSF_OK) return r;
    }
    return run_adjoint_finish(p, static_cast<const int64_t *>(L.G), L.status, grad_img, gout, dout_dsteps,
                              grad_steps, st);
}

bsf_status bsf_cov_to_steps(const bsf_config *cfg, const float *cov, int64_t H, int64_t W, float sub, float *steps,
                            void *ws, size_t ws_bytes, void *stream) {
    Plan p;
    bsf_status r = make_plan(cfg, H, W, &p);
    if (r != BSF_OK) return r;
    if (p.n_dirs != 4) return BSF_E_UNSUPPORTED;
    if (!ws) return BSF_E_INVALID;
    if (ws_bytes < kStatusBytes) return BSF_E_WORKSPACE;
    if (H * W > 0 && (!cov || !steps)) return BSF_E_INVALID;
    if (!isfinite(sub)) return BSF_E_INVALID;
    CovBank b;
    r = make_cov_bank(p, &b);
    if (r != BSF_OK) return r;
    return run_cov_to_steps(p, b, nullptr, cov, nullptr, sub, steps, nullptr, nullptr, static_cast<int32_t *>(ws),
                            static_cast<hipStream_t>(stream));
}

bsf_status bsf_set_tuning(int32_t gather_wx, int32_t line_tl) {
    if (gather_wx != 8 && gather_wx != 16 && gather_wx != 32 && gather_wx != 64) return BSF_E_INVALID;
    if (line_tl < 16 || line_tl > 4096 || (line_tl & (line_tl - 1)) != 0) return BSF_E_INVALID;
    g_tuning.gather_wx = gather_wx;
    g_tuning.line_tl = line_tl;
    return BSF_OK;
}

bsf_status bsf_set_box_tile(int32_t tile_h) {
    if (tile_h != 4 && tile_h != 8) return BSF_E_INVALID;
    g_tuning.box_h = tile_h;
    return BSF_OK;
}

int32_t bsf_get_box_tile(void) { return g_tuning.box_h; }

void bsf_get_tuning(int32_t *gather_wx, int32_t *line_tl) {
    if (gather_wx) *gather_wx = g_tuning.gather_wx;
    if (line_tl) *line_tl = g_tuning.line_tl;
}

bsf_status bsf_read_device_status(void *ws, void *stream, uint32_t *flags, int32_t *F_used, int32_t *log2_bound,
                                  int32_t clear) {
    if (!ws) return BSF_E_INVALID;
    BSF_HIP_CHECK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    int32_t h[ST_WORDS];
    BSF_HIP_CHECK(hipMemcpy(h, ws, sizeof(int32_t) * 8, hipMemcpyDeviceToHost));
    if (flags) *flags = (uint32_t)h[ST_FLAGS];
    if (F_used) *F_used = h[ST_F_USED];
    if (log2_bound) *log2_bound = h[ST_LOG2_BOUND];
    if (clear) {
        int32_t z = 0;
        BSF_HIP_CHECK(hipMemcpy(ws, &z, sizeof(z), hipMemcpyHostToDevice));
    }
    return BSF_OK;
}

}  // extern "C"

namespace {

// Scratch of bsf_filter_varying_noalloc: one array per GPU, in the code object
// (no allocation at run time).  Host code never uses the symbol's name as an
// address: the device address is looked up once per device and kept.
__device__ __align__(256) unsigned char scratch[BSF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mutex;

bsf_status scratch_of_current_device(void **ptr) {
    int dev = -1;
    BSF_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return BSF_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        BSF_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return BSF_E_DEVICE;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return BSF_OK;
}

__global__ void k_copy_status(const int32_t *status, int32_t *out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        out[0] = status[ST_FLAGS];
        out[1] = status[ST_F_USED];
        out[2] = status[ST_LOG2_BOUND];
        out[3] = 0;
    }
}

}  // namespace

extern "C" {

bsf_status bsf_filter_varying_noalloc(const bsf_config *cfg, bsf_dtype dtype, const void *img, int64_t H, int64_t W,
                                      int64_t pitch, const float *steps, float *out, int64_t *out_num,
                                      int64_t *out_den, float *dout_dsteps, int32_t *status_out, void *stream) {
    Plan p;
    bsf_status r = make_plan(cfg, H, W, &p);
    if (r != BSF_OK) return r;
    if (ws_bytes_for(p, true) > BSF_NOALLOC_SCRATCH_BYTES) return BSF_E_WORKSPACE;
    r = apply_checks(p, dtype, out_num, out_den, dout_dsteps);
    if (r != BSF_OK) return r;
    void *ws = nullptr;
    r = scratch_of_current_device(&ws);
    if (r != BSF_OK) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // this call's flags only: the array keeps the previous call's words
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, st, static_cast<int32_t *>(ws));
    BSF_HIP_CHECK(hipGetLastError());
    r = bsf_filter_varying(cfg, dtype, img, H, W, pitch, steps, out, out_num, out_den, dout_dsteps, nullptr, ws,
                           BSF_NOALLOC_SCRATCH_BYTES, stream);
    if (r != BSF_OK) return r;
    if (status_out) {
        hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, st, static_cast<const int32_t *>(ws), status_out);
        BSF_HIP_CHECK(hipGetLastError());
    }
    return BSF_OK;
}

const char *bsf_status_string(bsf_status s) {
    switch (s) {
    case BSF_OK: return "ok";
    case BSF_E_INVALID: return "invalid argument";
    case BSF_E_RANGE: return "step out of range";
    case BSF_E_OVERFLOW: return "fixed-point overflow";
    case BSF_E_WORKSPACE: return "workspace too small";
    case BSF_E_DEVICE: return "device error";
    case BSF_E_UNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

const char *bsf_version(void) { return "bsf 0.1 gfx950"; }

}  // extern "C"
