// Alg. 3 as the paper computes it: the box spline of four directions with
// continuous scales, from running sums read between lattice points through the
// interpolation of eq. interpolation, in FP64.
//
// The image is filtered tile by tile.  A 16 x 16 tile (or, when its steps need
// a larger rectangle than the LDS buffer holds, each b x b sub-tile in turn,
// b = 8, 4, 2, 1) loads into LDS, in FP64, the rectangle of lattice points that
// its taps read, takes the running sums of step 2 inside that rectangle, each
// line starting at zero where it enters it, and then evaluates every pixel's
// 16 taps of Table 1 at the shifts of eq. shifts (bit k of the tap index moves
// the tap by -s_k u_k, tau = (1/2) sum_k (s_k - 1) u_k, the sign is the parity
// of the bits, the weight 1 / prod s_k).  What a line's late start leaves out
// is cancelled by the taps' differences along every direction, because the
// rectangle holds the convex hull of all the points the taps read.  Each tap is
// F(q) = sum_m g(m) beta_b(q - m) over the lattice points m within half the sum
// of |u_k| of q (eq. interpolation), with beta_b the box spline of one lattice
// step along each direction and unit mass (the paper's beta'_b with all scales
// sqrt(5) for its directions).  The result is the image convolved with the
// centred box spline of the pixel's own scales.
//
// beta_b is the parallelogram of the first two directions convolved with that of
// the last two, so beta_b(p) = |P ^ (p + Q)| / (|P| |Q|).  The area of the
// overlap of two convex polygons is, by Green's theorem, half the sum over the
// edges a + t d (t in [0, 1]) of either polygon of (t1 - t0) (a x d) over the
// part [t0, t1] of the edge inside the other one; with four directions no edge
// of P is parallel to one of Q, and each part is the edge's parameter range
// clipped by the other parallelogram's two slabs: no vertex lists, no branches
// beyond min and max.  The area is the paper's "area of overlap" of two
// rotated boxes; the paper tabulates its quadratic pieces, here it is
// evaluated directly.
#include <limits.h>
#include <math.h>

#include <algorithm>
#include <cstdlib>

#include "bsf_common.h"

namespace bsf {
namespace {

constexpr int kA3Tile = 16;             // pixels per tile side
constexpr int kA3Threads = 256;         // one thread per pixel of a whole tile
constexpr size_t kA3CapDefault = 8192;  // window elements (64 KiB) when the steps allow it
constexpr size_t kA3CapMax = 18944;     // window elements (148 KiB): the largest LDS buffer

// Constants of the unit box spline of four directions.
struct A3Geom {
    double u[4][2];        // P spans (u0, u1), Q spans (u2, u3), each pair counter-clockwise
    double inv01, inv23;   // 1 / det(u0, u1), 1 / det(u2, u3)
    double pg[4], pd[4];   // P's edge starts a_i in Q's frame: gamma(a_i), delta(a_i)
    double prg[4], prd[4]; // 1 / gamma(d_i), 1 / delta(d_i) of P's edge directions
    double pc[4];          // a_i x d_i
    double qa[4], qb[4];   // Q's edge starts b_j (about Q's centre) in P's frame: alpha(b_j), beta(b_j)
    double qra[4], qrb[4]; // 1 / alpha(e_j), 1 / beta(e_j) of Q's edge directions
    double qc[4];          // b_j x e_j
    double qe[4][2];       // e_j
    double ex, ey;         // reach of beta_b: half the sums of |dx| and of |dy|
};

struct A3Args {
    const void *img;
    int kind;  // SrcKind of the image
    int64_t H, W, pitch;
    const float *steps;  // [4][H][W]
    float *out;          // nullable
    double *out64;       // nullable
    int32_t *status;
    int dx[4], dy[4];
    float max_step;
    int cap;               // window elements the LDS buffer holds
    int64_t tiles_x, tiles;
    A3Geom g;
};

__device__ __forceinline__ double cross2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

// Narrow [t0, t1] to the t with |v + t dv| <= 1/2 (r = 1 / dv, dv != 0).
__device__ __forceinline__ void slab(double v, double r, double &t0, double &t1) {
    const double ta = (-0.5 - v) * r, tb = (0.5 - v) * r;
    t0 = fmax(t0, fmin(ta, tb));
    t1 = fmin(t1, fmax(ta, tb));
}

// beta_b(p): the overlap of P (about 0) and Q (about p), over |P| |Q|.
__device__ double unit_box_spline(const A3Geom &G, double px, double py) {
    // p in Q's frame and in P's frame
    const double gp = cross2(px, py, G.u[3][0], G.u[3][1]) * G.inv23;
    const double dp = cross2(G.u[2][0], G.u[2][1], px, py) * G.inv23;
    const double ap = cross2(px, py, G.u[1][0], G.u[1][1]) * G.inv01;
    const double bp = cross2(G.u[0][0], G.u[0][1], px, py) * G.inv01;
    double twice = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // P's edges inside Q
        double t0 = 0.0, t1 = 1.0;
        slab(G.pg[i] - gp, G.prg[i], t0, t1);
        slab(G.pd[i] - dp, G.prd[i], t0, t1);
        twice += fmax(t1 - t0, 0.0) * G.pc[i];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {  // Q's edges inside P
        double t0 = 0.0, t1 = 1.0;
        slab(G.qa[j] + ap, G.qra[j], t0, t1);
        slab(G.qb[j] + bp, G.qrb[j], t0, t1);
        twice += fmax(t1 - t0, 0.0) * (G.qc[j] + cross2(px, py, G.qe[j][0], G.qe[j][1]));
    }
    return 0.5 * twice * G.inv01 * G.inv23;
}

__device__ __forceinline__ double a3_sample(const A3Args &a, int64_t x, int64_t y, bool &nonfinite) {
    if (x < 0 || y < 0 || x >= a.W || y >= a.H) return 0.0;
    const int64_t i = y * a.pitch + x;
    double v;
    if (a.kind == SRC_U8) v = static_cast<const uint8_t *>(a.img)[i];
    else if (a.kind == SRC_U16) v = static_cast<const uint16_t *>(a.img)[i];
    else v = static_cast<const float *>(a.img)[i];
    if (!isfinite(v)) nonfinite = true;
    return v;
}

// Offsets of tap e from its pixel (exact: s is a float, the directions small).
__device__ __forceinline__ void tap_offset(const A3Args &a, const double s[4], int e, double &qx, double &qy) {
    qx = 0.0;
    qy = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double t = 0.5 * (s[k] - 1.0) - ((e >> k) & 1) * s[k];
        qx += t * a.dx[k];
        qy += t * a.dy[k];
    }
}

struct Ext {
    int lx, hx, ly, hy;
};

__global__ __launch_bounds__(kA3Threads) void k_alg3(A3Args a) {
    extern __shared__ double win[];
    __shared__ double s_red[kA3Threads];
    __shared__ Ext s_wave[kA3Threads / 64];
    __shared__ unsigned char s_live[kA3Threads];
    __shared__ int s_nonfinite;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tile = xcd_item(blockIdx.x, a.tiles);
    if (tile >= a.tiles) return;
    const int64_t x0 = (tile % a.tiles_x) * kA3Tile, y0 = (tile / a.tiles_x) * kA3Tile;
    const int64_t HW = a.H * a.W;
    const double ex = a.g.ex, ey = a.g.ey;

    // 1. each pixel's steps and the offsets of the lattice points its taps read
    Ext e{INT_MAX, INT_MIN, INT_MAX, INT_MIN};
    bool live = false;
    {
        const int64_t x = x0 + (tid % kA3Tile), y = y0 + (tid / kA3Tile);
        if (x < a.W && y < a.H) {
            const int64_t p = y * a.W + x;
            double s[4];
            bool ok = true;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s[k] = a.steps[k * HW + p];
                ok = ok && s[k] >= 1.0 && s[k] <= (double)a.max_step;  // false for NaN
            }
            if (ok) {
                for (int t = 0; t < 16; ++t) {
                    double qx, qy;
                    tap_offset(a, s, t, qx, qy);
                    e.lx = min(e.lx, (int)ceil(qx - ex));
                    e.hx = max(e.hx, (int)floor(qx + ex));
                    e.ly = min(e.ly, (int)ceil(qy - ey));
                    e.hy = max(e.hy, (int)floor(qy + ey));
                }
                ok = (int64_t)(e.hx - e.lx + 1) * (e.hy - e.ly + 1) <= a.cap;
            }
            if (!ok) {
                atomicOr((unsigned *)&a.status[ST_FLAGS], BSF_FLAG_RANGE);
                if (a.out) a.out[p] = __builtin_nanf("");
                if (a.out64) a.out64[p] = __builtin_nan("");
                e = Ext{INT_MAX, INT_MIN, INT_MAX, INT_MIN};
            }
            live = ok;
        }
    }
    s_live[tid] = live;
    Ext t = e;
    for (int d = 32; d >= 1; d >>= 1) {
        t.lx = min(t.lx, __shfl_xor(t.lx, d, 64));
        t.hx = max(t.hx, __shfl_xor(t.hx, d, 64));
        t.ly = min(t.ly, __shfl_xor(t.ly, d, 64));
        t.hy = max(t.hy, __shfl_xor(t.hy, d, 64));
    }
    if (lane == 0) s_wave[wave] = t;
    if (tid == 0) s_nonfinite = 0;
    __syncthreads();
    Ext T = s_wave[0];
    for (int w = 1; w < kA3Threads / 64; ++w) {
        T.lx = min(T.lx, s_wave[w].lx);
        T.hx = max(T.hx, s_wave[w].hx);
        T.ly = min(T.ly, s_wave[w].ly);
        T.hy = max(T.hy, s_wave[w].hy);
    }
    if (T.lx == INT_MAX) return;  // no live pixel in the tile (block-uniform)

    // 2. the largest sub-tile whose rectangle, with the tile's offsets, fits.
    //    One pixel always fits: the offsets of any pixel with steps up to
    //    max_step lie within the span the buffer was sized for.
    int b = kA3Tile;
    while (b > 1 && (int64_t)(b + T.hx - T.lx) * (b + T.hy - T.ly) > a.cap) b >>= 1;
    const int per_side = kA3Tile / b, tpp = min(16, kA3Threads / (b * b));
    bool nonfinite = false;
    for (int sub = 0; sub < per_side * per_side; ++sub) {
        const int sx0 = (sub % per_side) * b, sy0 = (sub / per_side) * b;
        if (x0 + sx0 >= a.W || y0 + sy0 >= a.H) continue;  // block-uniform
        const Ext E = T;
        const int64_t wx0 = x0 + sx0 + E.lx, wy0 = y0 + sy0 + E.ly;
        const int WX = b + E.hx - E.lx, WY = b + E.hy - E.ly;
        if ((int64_t)WX * WY > a.cap) {  // not reached for steps within max_step; never overrun the buffer
            const int64_t x = x0 + sx0 + tid % b, y = y0 + sy0 + tid / b;
            if (tid < b * b && x < a.W && y < a.H) {
                if (a.out) a.out[y * a.W + x] = __builtin_nanf("");
                if (a.out64) a.out64[y * a.W + x] = __builtin_nan("");
            }
            if (tid == 0) atomicOr((unsigned *)&a.status[ST_FLAGS], BSF_FLAG_RANGE);
            continue;
        }
        __syncthreads();  // the previous sub-tile is done with the buffer
        for (int i = tid; i < WX * WY; i += kA3Threads)
            win[i] = a3_sample(a, wx0 + i % WX, wy0 + i / WX, nonfinite);
        __syncthreads();
        // step 2: g <- g + g(. - u_k), one direction after another
        for (int k = 0; k < 4; ++k) {
            const int dx = a.dx[k], dy = a.dy[k];
            const int cA = min(dx, WX), rB = min(abs(dy), WY);
            const int nA = cA * WY, nB = max(WX - dx, 0) * rB;
            for (int j = tid; j < nA + nB; j += kA3Threads) {
                int mx, my;  // where the line enters the rectangle
                if (j < nA) {
                    mx = j / WY;
                    my = j % WY;
                } else {
                    const int jj = j - nA, r = jj % rB;
                    mx = dx + jj / rB;
                    my = dy > 0 ? r : WY - 1 - r;
                }
                double acc = 0.0;
                while (mx < WX && my >= 0 && my < WY) {
                    acc += win[my * WX + mx];
                    win[my * WX + mx] = acc;
                    mx += dx;
                    my += dy;
                }
            }
            __syncthreads();
        }
        // step 3: the taps, tpp threads per pixel
        const int pi = tid / tpp, grp = tid % tpp;
        const int lx_ = pi % b, ly_ = pi / b;
        const int64_t px = x0 + sx0 + lx_, py = y0 + sy0 + ly_;
        const bool mine = pi < b * b && px < a.W && py < a.H && s_live[(sy0 + ly_) * kA3Tile + sx0 + lx_];
        double acc = 0.0, den = 1.0;
        if (mine) {
            const int64_t p = py * a.W + px;
            double s[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s[k] = a.steps[k * HW + p];
                den *= s[k];
            }
            // the pixel's offset inside the rectangle
            const int ox = (int)(px - wx0), oy = (int)(py - wy0);
            for (int tap = grp; tap < 16; tap += tpp) {
                double qx, qy;
                tap_offset(a, s, tap, qx, qy);
                const int mx0 = (int)ceil(qx - ex), mx1 = (int)floor(qx + ex);
                const int my0 = (int)ceil(qy - ey), my1 = (int)floor(qy + ey);
                double F = 0.0;
                for (int my = my0; my <= my1; ++my) {
                    const int iy = oy + my;
                    if ((unsigned)iy >= (unsigned)WY) continue;
                    for (int mx = mx0; mx <= mx1; ++mx) {
                        const int ix = ox + mx;
                        if ((unsigned)ix >= (unsigned)WX) continue;
                        F += win[iy * WX + ix] * unit_box_spline(a.g, qx - mx, qy - my);
                    }
                }
                acc += (__builtin_popcount(tap) & 1) ? -F : F;
            }
        }
        s_red[tid] = acc;
        __syncthreads();
        if (mine && grp == 0) {
            double v = 0.0;
            for (int j = 0; j < tpp; ++j) v += s_red[tid + j];
            v /= den;
            const int64_t p = py * a.W + px;
            if (a.out) a.out[p] = (float)v;
            if (a.out64) a.out64[p] = v;
        }
    }
    if (nonfinite) s_nonfinite = 1;
    __syncthreads();
    if (tid == 0 && s_nonfinite) atomicOr((unsigned *)&a.status[ST_FLAGS], BSF_FLAG_NONFINITE);
}

// Host: the constants of beta_b for four directions (the first two span P, the
// last two Q; each pair turned counter-clockwise).
bsf_status make_a3_geom(const int dx[4], const int dy[4], A3Geom *G) {
    double u[4][2];
    for (int k = 0; k < 4; ++k) {
        u[k][0] = dx[k];
        u[k][1] = dy[k];
    }
    for (int pair = 0; pair < 2; ++pair) {
        double *v0 = u[2 * pair], *v1 = u[2 * pair + 1];
        const double det = v0[0] * v1[1] - v0[1] * v1[0];
        if (det == 0.0) return BSF_E_INVALID;
        if (det < 0.0)
            for (int c = 0; c < 2; ++c) {
                const double t = v0[c];
                v0[c] = v1[c];
                v1[c] = t;
            }
    }
    for (int k = 0; k < 4; ++k)
        for (int c = 0; c < 2; ++c) G->u[k][c] = u[k][c];
    const double det01 = u[0][0] * u[1][1] - u[0][1] * u[1][0];
    const double det23 = u[2][0] * u[3][1] - u[2][1] * u[3][0];
    G->inv01 = 1.0 / det01;
    G->inv23 = 1.0 / det23;
    auto cr = [](const double *a, const double *b) { return a[0] * b[1] - a[1] * b[0]; };
    // corners (-,-), (+,-), (+,+), (-,+) and edges +v0, +v1, -v0, -v1: counter-clockwise
    const double sg[4][2] = {{-0.5, -0.5}, {0.5, -0.5}, {0.5, 0.5}, {-0.5, 0.5}};
    const double sd[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
    for (int i = 0; i < 4; ++i) {
        const double a[2] = {sg[i][0] * u[0][0] + sg[i][1] * u[1][0], sg[i][0] * u[0][1] + sg[i][1] * u[1][1]};
        const double d[2] = {sd[i][0] * u[0][0] + sd[i][1] * u[1][0], sd[i][0] * u[0][1] + sd[i][1] * u[1][1]};
        G->pg[i] = cr(a, u[3]) * G->inv23;
        G->pd[i] = cr(u[2], a) * G->inv23;
        const double gd = cr(d, u[3]) * G->inv23, dd = cr(u[2], d) * G->inv23;
        if (gd == 0.0 || dd == 0.0) return BSF_E_INVALID;  // parallel edges
        G->prg[i] = 1.0 / gd;
        G->prd[i] = 1.0 / dd;
        G->pc[i] = cr(a, d);
        const double b[2] = {sg[i][0] * u[2][0] + sg[i][1] * u[3][0], sg[i][0] * u[2][1] + sg[i][1] * u[3][1]};
        const double e[2] = {sd[i][0] * u[2][0] + sd[i][1] * u[3][0], sd[i][0] * u[2][1] + sd[i][1] * u[3][1]};
        G->qa[i] = cr(b, u[1]) * G->inv01;
        G->qb[i] = cr(u[0], b) * G->inv01;
        const double ad = cr(e, u[1]) * G->inv01, bd = cr(u[0], e) * G->inv01;
        if (ad == 0.0 || bd == 0.0) return BSF_E_INVALID;
        G->qra[i] = 1.0 / ad;
        G->qrb[i] = 1.0 / bd;
        G->qc[i] = cr(b, e);
        G->qe[i][0] = e[0];
        G->qe[i][1] = e[1];
    }
    G->ex = 0.0;
    G->ey = 0.0;
    for (int k = 0; k < 4; ++k) {
        G->ex += 0.5 * fabs((double)dx[k]);
        G->ey += 0.5 * fabs((double)dy[k]);
    }
    return BSF_OK;
}

// Window elements for b x b pixels at the largest step: every pixel's taps read
// offsets within a span of floor(S sum|dx|) + sum|dx| columns (and rows alike).
int64_t a3_window(const Plan &p, int b) {
    int64_t sx = 0, sy = 0;
    for (int k = 0; k < 4; ++k) {
        sx += std::abs(p.dx[k]);
        sy += std::abs(p.dy[k]);
    }
    const double S = p.max_step;
    return (b + (int64_t)floor(S * sx) + sx) * (b + (int64_t)floor(S * sy) + sy);
}

bsf_status a3_check(const bsf_config *cfg, int64_t H, int64_t W, Plan &p, size_t &cap) {
    bsf_status r = make_plan(cfg, H, W, &p);
    if (r != BSF_OK) return r;
    if (p.n_dirs != 4 || p.order != 1 || p.mode != BSF_STEPS_REAL || !p.tied) return BSF_E_UNSUPPORTED;
    const int64_t one = a3_window(p, 1), whole = a3_window(p, kA3Tile);
    if (one > (int64_t)kA3CapMax) return BSF_E_UNSUPPORTED;  // max_step too large for the LDS buffer
    cap = (size_t)std::max<int64_t>(std::min<int64_t>(whole, kA3CapDefault), one);
    return BSF_OK;
}

}  // namespace
}  // namespace bsf

using namespace bsf;

extern "C" {

size_t bsf_alg3_workspace_bytes(const bsf_config *cfg, int64_t H, int64_t W) {
    Plan p;
    size_t cap;
    if (a3_check(cfg, H, W, p, cap) != BSF_OK) return 0;
    return kStatusBytes;
}

bsf_status bsf_filter_alg3(const bsf_config *cfg, bsf_dtype dtype, const void *img, int64_t H, int64_t W,
                           int64_t pitch, const float *steps, float *out, double *out_f64, void *ws, size_t ws_bytes,
                           void *stream) {
    Plan p;
    size_t cap;
    bsf_status r = a3_check(cfg, H, W, p, cap);
    if (r != BSF_OK) return r;
    const int kind = dtype == BSF_U8 ? SRC_U8 : dtype == BSF_U16 ? SRC_U16 : dtype == BSF_F32 ? SRC_F32 : -1;
    if (kind < 0 || !ws || pitch < W || (H * W > 0 && (!img || !steps || (!out && !out_f64))))
        return BSF_E_INVALID;
    if (ws_bytes < kStatusBytes) return BSF_E_WORKSPACE;
    if (H * W == 0) return BSF_OK;
    A3Args a{};
    a.img = img;
    a.kind = kind;
    a.H = H;
    a.W = W;
    a.pitch = pitch;
    a.steps = steps;
    a.out = out;
    a.out64 = out_f64;
    a.status = static_cast<int32_t *>(ws);
    for (int k = 0; k < 4; ++k) {
        a.dx[k] = p.dx[k];
        a.dy[k] = p.dy[k];
    }
    a.max_step = p.max_step;
    a.cap = (int)cap;
    r = make_a3_geom(a.dx, a.dy, &a.g);
    if (r != BSF_OK) return r;
    a.tiles_x = (W + kA3Tile - 1) / kA3Tile;
    a.tiles = a.tiles_x * ((H + kA3Tile - 1) / kA3Tile);
    hipStream_t st = static_cast<hipStream_t>(stream);
    static bool s_big_lds = false;  // allow the largest buffer once per process
    if (!s_big_lds) {
        BSF_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(k_alg3),
                                          hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)(kA3CapMax * sizeof(double))));
        s_big_lds = true;
    }
    hipLaunchKernelGGL(k_alg3, dim3((unsigned)xcd_grid(a.tiles)), dim3(kA3Threads), cap * sizeof(double), st, a);
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

}  // extern "C"
