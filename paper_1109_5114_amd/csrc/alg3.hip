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
#include <utility>

#include "bsf_common.h"

namespace bsf {
namespace {

constexpr int kA3Tile = 16;        // pixels per tile side
constexpr int kA3Threads = 256;    // one thread per pixel of a whole tile
constexpr int kA3CapMax = 18944;   // window elements (148 KiB): the largest LDS buffer
// Launch tiers: a tile first goes to a launch whose LDS buffer holds kA3Tier[0]
// elements (four blocks per CU); a tile whose rectangle does not fit there,
// even in 4 x 4 pieces, is queued for the next tier, whose buffer is larger
// and whose blocks work through the queue.  The last tier's buffer holds any
// one pixel's rectangle at max_step.
constexpr int kA3Tier[2] = {4096, 8192};
constexpr int kA3MinPiece = 4;     // smallest piece of a tile outside the last tier

enum A3StatusWord : int {
    ST_A3_QUEUED0 = 28,  // tiles queued by the first tier
    ST_A3_QUEUED1 = 29,  // tiles queued by the second
};

// Constants of the unit box spline of four directions.  P is the
// parallelogram of the first two directions, Q that of the last two, each
// about its centre with its pair turned counter-clockwise; frame coordinates
// of a point x: (alpha, beta) in P's frame, (gamma, delta) in Q's, so that P
// and Q are [-1/2, 1/2]^2 there.  Each parallelogram's edges come in mirror
// pairs (edge i + 2 is edge i through the centre).  For P's edge a_i + t d_i
// (and its mirror) with Q about p, |gamma| <= 1/2 holds for t in
// [K + lg, K + ug] (mirror: [-K + lg, -K + ug]) with K = kg . p, and the same
// for delta; for Q's edge p + b_j + t e_j the range is [-A + la, -A + ua]
// (mirror: [A + la, A + ua]) with A = ka . p.  An edge's part inside the
// other parallelogram adds (t1 - t0) (start x direction) to twice the area.
struct A3Beta {
    double kg[2][2], kd[2][2], lg[2], ug[2], ld[2], ud[2], pc[2];  // P's edge pairs
    double ka[2][2], kb[2][2], la[2], ua[2], lb[2], ub[2], qc[2];  // Q's edge pairs
    double xe[2][2];          // p x e_j = xe[j] . p
    double scale;             // 1 / (2 det01 det23)
    // the support: |n_k . p| < h_k, n_k normal to u_k, h_k = (1/2) sum_j |n_k . u_j|
    double ny[4], h[4], rnx[4];  // rnx = 1 / n_k.x (0 when n_k.x = 0)
    double ex, ey;               // half the sums of |dx| and of |dy|
    int ok;                      // 0 when two directions are parallel
};

__host__ __device__ constexpr double a3_abs(double v) { return v < 0 ? -v : v; }
__host__ __device__ constexpr double a3_min(double a, double b) { return a < b ? a : b; }
__host__ __device__ constexpr double a3_max(double a, double b) { return a < b ? b : a; }

__host__ __device__ constexpr A3Beta make_beta(int x0, int y0, int x1, int y1, int x2, int y2, int x3, int y3) {
    A3Beta G{};
    const int dx[4] = {x0, x1, x2, x3}, dy[4] = {y0, y1, y2, y3};
    double u[4][2] = {{(double)x0, (double)y0}, {(double)x1, (double)y1}, {(double)x2, (double)y2},
                      {(double)x3, (double)y3}};
    for (int pr = 0; pr < 2; ++pr) {
        const double det = u[2 * pr][0] * u[2 * pr + 1][1] - u[2 * pr][1] * u[2 * pr + 1][0];
        if (det == 0.0) return G;
        if (det < 0.0)
            for (int c = 0; c < 2; ++c) {
                const double t = u[2 * pr][c];
                u[2 * pr][c] = u[2 * pr + 1][c];
                u[2 * pr + 1][c] = t;
            }
    }
    const double det01 = u[0][0] * u[1][1] - u[0][1] * u[1][0];
    const double det23 = u[2][0] * u[3][1] - u[2][1] * u[3][0];
    // alpha = fa . x = (x ^ u1) / det01, beta = (u0 ^ x) / det01, gamma = (x ^ u3) / det23, delta = (u2 ^ x) / det23
    const double fa[2] = {u[1][1] / det01, -u[1][0] / det01}, fb[2] = {-u[0][1] / det01, u[0][0] / det01};
    const double fg[2] = {u[3][1] / det23, -u[3][0] / det23}, fd[2] = {-u[2][1] / det23, u[2][0] / det23};
    // edges 0 and 1: from corner (-1/2, -1/2) along +v0, from (+1/2, -1/2) along +v1
    const double sg[2][2] = {{-0.5, -0.5}, {0.5, -0.5}}, sd[2][2] = {{1, 0}, {0, 1}};
    for (int i = 0; i < 2; ++i) {
        for (int side = 0; side < 2; ++side) {
            const double *v0 = u[2 * side], *v1 = u[2 * side + 1];
            const double a[2] = {sg[i][0] * v0[0] + sg[i][1] * v1[0], sg[i][0] * v0[1] + sg[i][1] * v1[1]};
            const double d[2] = {sd[i][0] * v0[0] + sd[i][1] * v1[0], sd[i][0] * v0[1] + sd[i][1] * v1[1]};
            // the other parallelogram's two frame coordinates
            const double *f1 = side == 0 ? fg : fa, *f2 = side == 0 ? fd : fb;
            const double c1 = f1[0] * a[0] + f1[1] * a[1], c2 = f2[0] * a[0] + f2[1] * a[1];
            const double e1 = f1[0] * d[0] + f1[1] * d[1], e2 = f2[0] * d[0] + f2[1] * d[1];
            if (e1 == 0.0 || e2 == 0.0) return G;  // an edge of one parallel to an edge of the other
            const double r1 = 1.0 / e1, r2 = 1.0 / e2;
            const double lo1 = a3_min((-0.5 - c1) * r1, (0.5 - c1) * r1), hi1 = a3_max((-0.5 - c1) * r1, (0.5 - c1) * r1);
            const double lo2 = a3_min((-0.5 - c2) * r2, (0.5 - c2) * r2), hi2 = a3_max((-0.5 - c2) * r2, (0.5 - c2) * r2);
            const double cr = a[0] * d[1] - a[1] * d[0];
            if (side == 0) {
                G.kg[i][0] = fg[0] * r1;
                G.kg[i][1] = fg[1] * r1;
                G.kd[i][0] = fd[0] * r2;
                G.kd[i][1] = fd[1] * r2;
                G.lg[i] = lo1;
                G.ug[i] = hi1;
                G.ld[i] = lo2;
                G.ud[i] = hi2;
                G.pc[i] = cr;
            } else {
                G.ka[i][0] = fa[0] * r1;
                G.ka[i][1] = fa[1] * r1;
                G.kb[i][0] = fb[0] * r2;
                G.kb[i][1] = fb[1] * r2;
                G.la[i] = lo1;
                G.ua[i] = hi1;
                G.lb[i] = lo2;
                G.ub[i] = hi2;
                G.qc[i] = cr;
                // p x d = p.x d.y - p.y d.x
                G.xe[i][0] = d[1];
                G.xe[i][1] = -d[0];
            }
        }
    }
    G.scale = 0.5 / (det01 * det23);
    for (int k = 0; k < 4; ++k) {
        G.ex += 0.5 * a3_abs(dx[k]);
        G.ey += 0.5 * a3_abs(dy[k]);
        const double nx = -dy[k], ny = dx[k];
        double h = 0.0;
        for (int j = 0; j < 4; ++j) h += 0.5 * a3_abs(nx * dx[j] + ny * dy[j]);
        G.ny[k] = ny;
        G.h[k] = h;
        G.rnx[k] = nx != 0.0 ? 1.0 / nx : 0.0;
    }
    G.ok = 1;
    return G;
}

// The direction sets with constants built into the kernels: 1 for those of
// Alg. 3 and Table 1 (canonical sign), 2 for those of Section 1.1; 0 reads
// them from the launch arguments.
__host__ __device__ constexpr A3Beta beta_of_set(int set) {
    return set == 1 ? make_beta(2, 1, 1, 2, 1, -2, 2, -1) : make_beta(1, 0, 0, 1, 1, 1, 1, -1);
}

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
    int64_t tiles_x, tiles;
    A3Beta g;  // for other direction sets
};

// beta_b(p): the overlap of P (about 0) and Q (about p), over |P| |Q|.
__device__ __forceinline__ double unit_box_spline(const A3Beta &G, double px, double py) {
    double twice = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double K = G.kg[i][0] * px + G.kg[i][1] * py, J = G.kd[i][0] * px + G.kd[i][1] * py;
        const double t0 = fmax(fmax(K + G.lg[i], J + G.ld[i]), 0.0), t1 = fmin(fmin(K + G.ug[i], J + G.ud[i]), 1.0);
        const double m0 = fmax(fmax(G.lg[i] - K, G.ld[i] - J), 0.0), m1 = fmin(fmin(G.ug[i] - K, G.ud[i] - J), 1.0);
        twice += (fmax(t1 - t0, 0.0) + fmax(m1 - m0, 0.0)) * G.pc[i];
        const double A = G.ka[i][0] * px + G.ka[i][1] * py, B = G.kb[i][0] * px + G.kb[i][1] * py;
        const double s0 = fmax(fmax(G.la[i] - A, G.lb[i] - B), 0.0), s1 = fmin(fmin(G.ua[i] - A, G.ub[i] - B), 1.0);
        const double n0 = fmax(fmax(G.la[i] + A, G.lb[i] + B), 0.0), n1 = fmin(fmin(G.ua[i] + A, G.ub[i] + B), 1.0);
        const double pe = G.xe[i][0] * px + G.xe[i][1] * py;
        twice += fmax(s1 - s0, 0.0) * (G.qc[i] + pe) + fmax(n1 - n0, 0.0) * (G.qc[i] - pe);
    }
    return twice * G.scale;
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

struct A3Shared {
    double red[kA3Threads];
    Ext wave[kA3Threads / 64];
    unsigned char live[kA3Threads];
};

// F(q) of eq. interpolation at the tap q = pixel + (qx, qy): the running sums
// at the lattice points of beta_b's support around q, row by row (the
// support's cross-section at each row bounds the columns), weighted by
// beta_b(q - m).  (ox, oy) is the pixel inside the WX x WY rectangle.
__device__ __forceinline__ double interpolate(const A3Beta &G, const double *win, int WX, int WY, int ox, int oy,
                                              double qx, double qy) {
    const int mx0 = (int)ceil(qx - G.ex), mx1 = (int)floor(qx + G.ex);
    const int my0 = (int)ceil(qy - G.ey), my1 = (int)floor(qy + G.ey);
    double F = 0.0;
    for (int my = my0; my <= my1; ++my) {
        const int iy = oy + my;
        if ((unsigned)iy >= (unsigned)WY) continue;
        const double py = qy - my;
        double xl = -G.ex, xr = G.ex;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (G.rnx[k] != 0.0) {
                const double c = -G.ny[k] * py;
                const double t1 = (c - G.h[k]) * G.rnx[k], t2 = (c + G.h[k]) * G.rnx[k];
                xl = fmax(xl, fmin(t1, t2));
                xr = fmin(xr, fmax(t1, t2));
            } else if (fabs(G.ny[k] * py) >= G.h[k]) {
                xr = xl - 1.0;  // the row misses the support
            }
        }
        const int lo = max(mx0, (int)ceil(qx - xr)), hi = min(mx1, (int)floor(qx - xl));
        for (int mx = lo; mx <= hi; ++mx) {
            const int ix = ox + mx;
            if ((unsigned)ix >= (unsigned)WX) continue;
            F += win[iy * WX + ix] * unit_box_spline(G, qx - mx, py);
        }
    }
    return F;
}

// One tile: the rectangle of every piece of it that fits `cap` window
// elements, at pieces of at least b_min pixels a side; a tile that fits no
// such piece goes to q_out (NULL in the last tier, whose buffer fits one pixel).
__device__ __forceinline__ void a3_tile_body(const A3Args &a, const A3Beta &G, int64_t tile, int cap, int b_min,
                                             int32_t *q_out, int32_t *n_out, double *win, A3Shared &sh,
                                             bool &nonfinite) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t x0 = (tile % a.tiles_x) * kA3Tile, y0 = (tile / a.tiles_x) * kA3Tile;
    const int64_t HW = a.H * a.W;

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
                    e.lx = min(e.lx, (int)ceil(qx - G.ex));
                    e.hx = max(e.hx, (int)floor(qx + G.ex));
                    e.ly = min(e.ly, (int)ceil(qy - G.ey));
                    e.hy = max(e.hy, (int)floor(qy + G.ey));
                }
            } else {
                atomicOr((unsigned *)&a.status[ST_FLAGS], BSF_FLAG_RANGE);
                if (a.out) a.out[p] = __builtin_nanf("");
                if (a.out64) a.out64[p] = __builtin_nan("");
            }
            live = ok;
        }
    }
    sh.live[tid] = live;
    Ext t = e;
    for (int d = 32; d >= 1; d >>= 1) {
        t.lx = min(t.lx, __shfl_xor(t.lx, d, 64));
        t.hx = max(t.hx, __shfl_xor(t.hx, d, 64));
        t.ly = min(t.ly, __shfl_xor(t.ly, d, 64));
        t.hy = max(t.hy, __shfl_xor(t.hy, d, 64));
    }
    if (lane == 0) sh.wave[wave] = t;
    __syncthreads();
    Ext T = sh.wave[0];
    for (int w = 1; w < kA3Threads / 64; ++w) {
        T.lx = min(T.lx, sh.wave[w].lx);
        T.hx = max(T.hx, sh.wave[w].hx);
        T.ly = min(T.ly, sh.wave[w].ly);
        T.hy = max(T.hy, sh.wave[w].hy);
    }
    if (T.lx == INT_MAX) {  // no live pixel in the tile (block-uniform)
        __syncthreads();
        return;
    }

    // 2. the largest piece whose rectangle, with the tile's offsets, fits
    int b = kA3Tile;
    while (b > b_min && (int64_t)(b + T.hx - T.lx) * (b + T.hy - T.ly) > cap) b >>= 1;
    if ((int64_t)(b + T.hx - T.lx) * (b + T.hy - T.ly) > cap) {
        if (q_out) {
            if (tid == 0) q_out[atomicAdd(n_out, 1)] = (int32_t)tile;
        } else {
            // not reached: the last buffer holds one pixel's rectangle at max_step
            if (live) {
                const int64_t p = (y0 + tid / kA3Tile) * a.W + x0 + tid % kA3Tile;
                if (a.out) a.out[p] = __builtin_nanf("");
                if (a.out64) a.out64[p] = __builtin_nan("");
            }
            if (tid == 0) atomicOr((unsigned *)&a.status[ST_FLAGS], BSF_FLAG_RANGE);
        }
        __syncthreads();
        return;
    }
    const int per_side = kA3Tile / b, tpp = min(16, kA3Threads / (b * b));
    const int WX = b + T.hx - T.lx, WY = b + T.hy - T.ly;
    for (int sub = 0; sub < per_side * per_side; ++sub) {
        const int sx0 = (sub % per_side) * b, sy0 = (sub / per_side) * b;
        if (x0 + sx0 >= a.W || y0 + sy0 >= a.H) continue;  // block-uniform
        const int64_t wx0 = x0 + sx0 + T.lx, wy0 = y0 + sy0 + T.ly;
        __syncthreads();  // the previous piece is done with the buffer
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
        const int lx = pi % b, ly = pi / b;
        const int64_t px = x0 + sx0 + lx, py = y0 + sy0 + ly;
        const bool mine = pi < b * b && px < a.W && py < a.H && sh.live[(sy0 + ly) * kA3Tile + sx0 + lx];
        double acc = 0.0, den = 1.0;
        if (mine) {
            const int64_t p = py * a.W + px;
            double s[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s[k] = a.steps[k * HW + p];
                den *= s[k];
            }
            const int ox = (int)(px - wx0), oy = (int)(py - wy0);
            for (int tap = grp; tap < 16; tap += tpp) {
                double qx, qy;
                tap_offset(a, s, tap, qx, qy);
                const double F = interpolate(G, win, WX, WY, ox, oy, qx, qy);
                acc += (__builtin_popcount(tap) & 1) ? -F : F;
            }
        }
        sh.red[tid] = acc;
        __syncthreads();
        if (mine && grp == 0) {
            double v = 0.0;
            for (int j = 0; j < tpp; ++j) v += sh.red[tid + j];
            v /= den;
            const int64_t p = py * a.W + px;
            if (a.out) a.out[p] = (float)v;
            if (a.out64) a.out64[p] = v;
        }
    }
    __syncthreads();  // the shared words are free for the next tile
}

// SET 1 and 2 build the constants of their direction set into the code.
template <int SET>
__device__ __forceinline__ void a3_tile(const A3Args &a, int64_t tile, int cap, int b_min, int32_t *q_out,
                                        int32_t *n_out, double *win, A3Shared &sh, bool &nonfinite) {
    if constexpr (SET == 0) {
        a3_tile_body(a, a.g, tile, cap, b_min, q_out, n_out, win, sh, nonfinite);
    } else {
        constexpr A3Beta G = beta_of_set(SET);
        a3_tile_body(a, G, tile, cap, b_min, q_out, n_out, win, sh, nonfinite);
    }
}

__global__ void k_alg3_begin(int32_t *status) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        status[ST_A3_QUEUED0] = 0;
        status[ST_A3_QUEUED1] = 0;
    }
}

__device__ __forceinline__ void flag_nonfinite(const A3Args &a, bool nonfinite) {
    if (__any(nonfinite) && (threadIdx.x & 63) == 0) atomicOr((unsigned *)&a.status[ST_FLAGS], BSF_FLAG_NONFINITE);
}

// First tier: one block per tile, in XCD order.
template <int SET>
__global__ __launch_bounds__(kA3Threads) void k_alg3_tiles(A3Args a, int cap, int b_min, int32_t *q_out,
                                                           int32_t *n_out) {
    extern __shared__ double win[];
    __shared__ A3Shared sh;
    const int64_t tile = xcd_item(blockIdx.x, a.tiles);
    bool nonfinite = false;
    if (tile < a.tiles) a3_tile<SET>(a, tile, cap, b_min, q_out, n_out, win, sh, nonfinite);
    flag_nonfinite(a, nonfinite);
}

// Later tiers: blocks work through the tiles the previous tier queued.
template <int SET>
__global__ __launch_bounds__(kA3Threads) void k_alg3_queue(A3Args a, int cap, int b_min, const int32_t *q_in,
                                                           const int32_t *n_in, int32_t *q_out, int32_t *n_out) {
    extern __shared__ double win[];
    __shared__ A3Shared sh;
    const int n = *n_in;
    bool nonfinite = false;
    for (int i = blockIdx.x; i < n; i += gridDim.x) a3_tile<SET>(a, q_in[i], cap, b_min, q_out, n_out, win, sh, nonfinite);
    flag_nonfinite(a, nonfinite);
}

// The launch tiers for a plan: buffer sizes in window elements, the last one
// holding any single pixel's rectangle (and a whole tile's when it is small).
struct A3Tiers {
    int n;
    int cap[3];
};

// Which direction set's constants are built in (0: none).
int a3_set(const Plan &p) {
    const int sets[2][8] = {{2, 1, 1, 2, 1, -2, 2, -1}, {1, 0, 0, 1, 1, 1, 1, -1}};
    for (int k = 0; k < 2; ++k) {
        int found = 0;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j)
                if (p.dx[i] == sets[k][2 * j] && p.dy[i] == sets[k][2 * j + 1]) ++found;
        if (found == 4) return k + 1;
    }
    return 0;
}

template <int SET>
bsf_status a3_launch(const A3Args &a, const A3Tiers &tiers, int32_t *const queue[2], int32_t *const queued[2],
                     hipStream_t st) {
    static bool s_big_lds = false;  // allow the largest buffer, once per process
    if (!s_big_lds) {
        for (const void *k : {reinterpret_cast<const void *>(k_alg3_tiles<SET>),
                              reinterpret_cast<const void *>(k_alg3_queue<SET>)})
            BSF_HIP_CHECK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                              (int)(kA3CapMax * sizeof(double))));
        s_big_lds = true;
    }
    for (int i = 0; i < tiers.n; ++i) {
        const bool last = i == tiers.n - 1;
        const int cap = tiers.cap[i], b_min = last ? 1 : kA3MinPiece;
        int32_t *q_out = last ? nullptr : queue[i % 2], *n_out = last ? nullptr : queued[i % 2];
        const size_t lds = (size_t)cap * sizeof(double);
        if (i == 0) {
            hipLaunchKernelGGL(k_alg3_tiles<SET>, dim3((unsigned)xcd_grid(a.tiles)), dim3(kA3Threads), lds, st, a,
                               cap, b_min, q_out, n_out);
        } else {
            const unsigned grid = (unsigned)std::min<int64_t>(a.tiles, 2048);
            hipLaunchKernelGGL(k_alg3_queue<SET>, dim3(grid), dim3(kA3Threads), lds, st, a, cap, b_min,
                               queue[(i - 1) % 2], queued[(i - 1) % 2], q_out, n_out);
        }
        BSF_HIP_CHECK(hipGetLastError());
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

bsf_status a3_check(const bsf_config *cfg, int64_t H, int64_t W, Plan &p, A3Tiers &t) {
    bsf_status r = make_plan(cfg, H, W, &p);
    if (r != BSF_OK) return r;
    if (p.n_dirs != 4 || p.order != 1 || p.mode != BSF_STEPS_REAL || !p.tied) return BSF_E_UNSUPPORTED;
    const int64_t one = a3_window(p, 1), whole = a3_window(p, kA3Tile);
    if (one > kA3CapMax) return BSF_E_UNSUPPORTED;  // max_step too large for the LDS buffer
    const int last = (int)std::max<int64_t>(std::min<int64_t>(whole, kA3Tier[1]), one);
    t.n = 0;
    for (int c : kA3Tier)
        if (c < last) t.cap[t.n++] = c;
    t.cap[t.n++] = last;
    return BSF_OK;
}

size_t a3_queue_bytes(int64_t tiles) { return align_up((size_t)tiles * sizeof(int32_t)); }

}  // namespace
}  // namespace bsf

using namespace bsf;

extern "C" {

size_t bsf_alg3_workspace_bytes(const bsf_config *cfg, int64_t H, int64_t W) {
    Plan p;
    A3Tiers t;
    if (a3_check(cfg, H, W, p, t) != BSF_OK) return 0;
    const int64_t tiles = ((W + kA3Tile - 1) / kA3Tile) * ((H + kA3Tile - 1) / kA3Tile);
    return kStatusBytes + 2 * a3_queue_bytes(tiles);
}

bsf_status bsf_filter_alg3(const bsf_config *cfg, bsf_dtype dtype, const void *img, int64_t H, int64_t W,
                           int64_t pitch, const float *steps, float *out, double *out_f64, void *ws, size_t ws_bytes,
                           void *stream) {
    Plan p;
    A3Tiers tiers;
    bsf_status r = a3_check(cfg, H, W, p, tiers);
    if (r != BSF_OK) return r;
    const int kind = dtype == BSF_U8 ? SRC_U8 : dtype == BSF_U16 ? SRC_U16 : dtype == BSF_F32 ? SRC_F32 : -1;
    if (kind < 0 || !ws || pitch < W || (H * W > 0 && (!img || !steps || (!out && !out_f64))))
        return BSF_E_INVALID;
    if (ws_bytes < bsf_alg3_workspace_bytes(cfg, H, W)) return BSF_E_WORKSPACE;
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
    a.g = make_beta(p.dx[0], p.dy[0], p.dx[1], p.dy[1], p.dx[2], p.dy[2], p.dx[3], p.dy[3]);
    if (!a.g.ok) return BSF_E_INVALID;
    a.tiles_x = (W + kA3Tile - 1) / kA3Tile;
    a.tiles = a.tiles_x * ((H + kA3Tile - 1) / kA3Tile);
    int32_t *const queue[2] = {reinterpret_cast<int32_t *>(static_cast<char *>(ws) + kStatusBytes),
                               reinterpret_cast<int32_t *>(static_cast<char *>(ws) + kStatusBytes +
                                                           a3_queue_bytes(a.tiles))};
    int32_t *const queued[2] = {a.status + ST_A3_QUEUED0, a.status + ST_A3_QUEUED1};
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_alg3_begin, dim3(1), dim3(64), 0, st, a.status);
    BSF_HIP_CHECK(hipGetLastError());
    switch (a3_set(p)) {
    case 1: return a3_launch<1>(a, tiers, queue, queued, st);
    case 2: return a3_launch<2>(a, tiers, queue, queued, st);
    default: return a3_launch<0>(a, tiers, queue, queued, st);
    }
}

}  // extern "C"
