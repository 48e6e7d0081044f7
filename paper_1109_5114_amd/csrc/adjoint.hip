// Adjoint of the space-variant filter with respect to the image.
//
// Forward, per pixel x:  out(x) = 2^-F / prod s(x) * sum_J c_J(x) J(x), where J
// are the integer tap combinations of the running sums G = S f (one per choice
// of operator per direction) and c_J the FP64 phase products.  Its transpose
// sends the upstream gradient g back through the same taps and then through the
// transposed running sums:
//     grad_f = S^T  sum_x  sum_J  omega_J(x) B_J(. - x),
// with B_J the integer tap pattern of J and omega_J(x) = g(x) c_J(x) / prod s(x).
//
// To keep the cancellation exact the weights are fixed point in the J basis,
// omega_J = nearest(2^Fg g c_J / prod s), and everything after that is int64
// modulo 2^64: the scatter of sum_J omega_J B_J into a window-sized array, and
// the suffix sums S^T (the transposed, window-truncated running sums, last
// direction first).  Only the final value at each image pixel p has to fit in
// 63 bits, and it is bounded by
//     |V(p)| <= sum_x sum_J |round(omega_J(x))| K_J(p - x)
//            <= 2 * 2^Fg max|g| * sum_x k_x(p - x)
// (K_J >= 0 are the integer component kernels, k_x the pixel's normalised
// kernel, and |round(w)| <= 2|w| for every w).  The column sum
// sum_x k_x(p - x) has no fixed bound (pixels with long steps pointing at p
// pile up), so it is bounded from the data before the scatter: every pixel's
// kernel is at most kmax(x) = min(1, 1/S_(1), 1/(S_(1) S_(2))) (S_(1) >= S_(2)
// the largest steps of two different directions: the factors of two
// non-parallel directions meet at every lattice point at most once, and
// further factors only spread mass) on the rectangle that holds its support,
// and the sum of those rectangles, a 2-D prefix sum of a difference array, is
// maximised over the image.  Fg = 62 - ceil(log2(max|g| * bound)), unclamped,
// so the weights keep their bits whatever the scale of g.  The only error is
// the rounding of omega_J.
#include "bsf_common.h"
#include "cluster_box.h"

namespace bsf {

// The cluster-box scatter in the frame of Table 1's directions (canon = 2),
// launched on the given grid; defined by adjoint_f1.hip, which compiles this
// file's kernels for that frame only.
bsf_status launch_adj_scatter_f1(const AdjointArgs &a, dim3 grid, hipStream_t st);

namespace {

constexpr int kTile = 16;
constexpr int kKmaxBits = 24;  // fixed-point scale of the per-pixel kernel bounds

__device__ __forceinline__ bool pixel_of_thread(int64_t H, int64_t W, int64_t &x, int64_t &y) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    x = (int64_t)blockIdx.x * kTile + (w & 1) * 8 + (lane & 7);
    y = (int64_t)blockIdx.y * kTile + (w >> 1) * 8 + (lane >> 3);
    return x < W && y < H;
}

__device__ __forceinline__ float clamp_step(float s, float max_step) { return fminf(fmaxf(s, 1.0f), max_step); }

__device__ __forceinline__ int64_t fixed(double v) { return (int64_t)__builtin_rint(v); }

__device__ __forceinline__ void atomic_add_i64(int64_t *p, int64_t v) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}

// A finite, nonzero upstream gradient scatters; zero scatters nothing and a
// NaN or infinity is reported (and poisons grad_img) instead.
__device__ __forceinline__ bool scatters(float g) { return g != 0.0f && fabsf(g) <= 3.402823466e38f; }

__global__ void k_adj_begin(int32_t *status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        status[ST_G_ABSMAX_BITS] = 0;
        status[ST_COLSUM_MAX] = 0;
        status[ST_COLSUM_MAX + 1] = 0;
        status[ST_G_NONFINITE] = 0;
    }
}

__global__ __launch_bounds__(256) void k_adj_gmax(const float *__restrict__ g, int64_t H, int64_t W,
                                                  int32_t *status) {
    __shared__ unsigned s_b[4];
    __shared__ int s_nf[4];
    unsigned b = 0;
    int nf = 0;
    for (int64_t y = blockIdx.x; y < H; y += gridDim.x)
        for (int64_t x = threadIdx.x; x < W; x += blockDim.x) {
            const float v = fabsf(g[y * W + x]);
            if (v <= 3.402823466e38f) b = max(b, __float_as_uint(v));
            else nf = 1;
        }
    for (int d = 32; d >= 1; d >>= 1) {
        b = max(b, (unsigned)__shfl_xor((int)b, d, 64));
        nf |= __shfl_xor(nf, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_b[threadIdx.x >> 6] = b;
        s_nf[threadIdx.x >> 6] = nf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            b = max(b, s_b[k]);
            nf |= s_nf[k];
        }
        atomicMax((unsigned *)&status[ST_G_ABSMAX_BITS], b);
        if (nf) {
            atomicOr((unsigned *)&status[ST_G_NONFINITE], 1u);
            atomicOr((unsigned *)&status[ST_FLAGS], BSF_FLAG_NONFINITE);
        }
    }
}

// Peak bound of the 1-D factor kernels.  For a continuous step s (clamped to
// >= 1), R = floor((s - 1)/2) and lambda = (s - 2R - 1)/2, the normalised
// factor is phi = alpha U + beta V with U, V the normalised odd boxes of
// lengths 2R + 1 and 2R + 3, alpha = (1 - lambda)(2R + 1)/s, beta =
// lambda (2R + 3)/s; max phi = 1/s, and phi * phi (symmetric) peaks at
// sum phi^2 = (2R + 1 + 2 lambda^2)/s^2.  ||U * U||_2 = sqrt((2L^2 + 1)/(3L^3))
// for a box of odd length L, so ||phi * phi||_2 <= (alpha sqrt||U*U|| +
// beta sqrt||V*V||)^2 by the triangle and Cauchy-Schwarz inequalities.
struct FactorBound {
    double peak1;  // max phi
    double peak2;  // max phi * phi = ||phi||_2^2
    double l2sq2;  // bound on ||phi * phi||_2^2
};

__device__ __forceinline__ double box2_norm(double L) { return sqrt((2.0 * L * L + 1.0) / (3.0 * L * L * L)); }

__device__ __forceinline__ FactorBound factor_bound(float s) {
    const double sd = (double)s;
    const double R = floor((sd - 1.0) * 0.5), lam = (sd - 2.0 * R - 1.0) * 0.5;
    const double L = 2.0 * R + 1.0;
    const double al = (1.0 - lam) * L / sd, be = lam * (L + 2.0) / sd;
    const double m = al * sqrt(box2_norm(L)) + be * sqrt(box2_norm(L + 2.0));
    FactorBound b;
    b.peak1 = 1.0 / sd;
    b.peak2 = (L + 2.0 * lam * lam) / (sd * sd);
    b.l2sq2 = m * m * m * m;
    return b;
}

// Column-sum bound, first part: each scattering pixel adds ceil(kmax 2^24) on
// the rectangle of the image that holds its kernel's support, as the four
// corners of a difference array D[(H + 1) x (W + 1)].  Along factor j the
// kernel reaches |i| <= R_j + 1 lattice steps.  kmax bounds the pixel's
// kernel, the convolution of the direction kernels A_k (each the convolution
// of its factors), by the smallest of
//   - max A_a max A_b for two directions (factors of non-parallel directions
//     meet at a lattice point at most once; further factors only spread mass),
//   - ||A_a * A_b||_2 ||A_c * A_d||_2 = sqrt(prod ||A||_2^2) over up to four
//     directions (Cauchy-Schwarz), and 1;
// max A_k is at most 1/s of any of its factors, and max(phi * phi) of a
// repeated (tied) factor; ||A_k||_2^2 is at most ||phi||_2^2 of any factor and
// the bound on ||phi * phi||_2^2 of a repeated one.
__global__ __launch_bounds__(256) void k_adj_colsum_scatter(AdjointArgs a, uint64_t *__restrict__ D) {
    int64_t x, y;
    if (!pixel_of_thread(a.H, a.W, x, y)) return;
    const int64_t HW = a.H * a.W, idx = y * a.W + x;
    if (!scatters(a.gout[idx])) return;
    double pk[BSF_MAX_DIRS], l2[BSF_MAX_DIRS];
    int64_t ex = 0, ey = 0;
    for (int k = 0; k < a.n_dirs; ++k) {
        pk[k] = 1.0;
        l2[k] = 1.0;
        for (int q = 0; q < a.order; ++q) {
            const int j = k * a.order + q;
            const float s = clamp_step(a.steps[a.plane[j] * HW + idx], a.max_step);
            const FactorBound fb = factor_bound(s);
            pk[k] = fmin(pk[k], fb.peak1);
            l2[k] = fmin(l2[k], fb.peak2);
            if (a.tied && a.order >= 2) {
                pk[k] = fmin(pk[k], fb.peak2);
                l2[k] = fmin(l2[k], fb.l2sq2);
            }
            const int64_t reach = (int64_t)floorf((s - 1.0f) * 0.5f) + 1;
            ex += reach * a.adx[k];
            ey += reach * a.ady[k];
        }
    }
    // the two smallest peaks, and the product of up to four smallest L2 norms
    double p1 = 1.0, p2 = 1.0;
    for (int k = 0; k < a.n_dirs; ++k) {
        if (pk[k] < p1) {
            p2 = p1;
            p1 = pk[k];
        } else if (pk[k] < p2) {
            p2 = pk[k];
        }
    }
    double lprod = 1.0;
    bool used[BSF_MAX_DIRS] = {};
    for (int n = 0; n < 4 && n < a.n_dirs; ++n) {
        int best = -1;
        for (int k = 0; k < a.n_dirs; ++k)
            if (!used[k] && (best < 0 || l2[k] < l2[best])) best = k;
        used[best] = true;
        lprod *= l2[best];
    }
    double kmax = fmin(1.0, fmin(p1 * p2, sqrt(lprod)));
    kmax *= 1.0 + 0x1p-30;  // stays an upper bound through the rounding above
    const uint64_t v = (uint64_t)ceil(__builtin_ldexp(kmax, kKmaxBits));
    const int64_t W1 = a.W + 1;
    const int64_t x0 = max(x - ex, (int64_t)0), x1 = min(x + ex, a.W - 1) + 1;
    const int64_t y0 = max(y - ey, (int64_t)0), y1 = min(y + ey, a.H - 1) + 1;
    atomicAdd((unsigned long long *)&D[y0 * W1 + x0], (unsigned long long)v);
    atomicAdd((unsigned long long *)&D[y0 * W1 + x1], (unsigned long long)(0 - v));
    atomicAdd((unsigned long long *)&D[y1 * W1 + x0], (unsigned long long)(0 - v));
    atomicAdd((unsigned long long *)&D[y1 * W1 + x1], (unsigned long long)v);
}

// Column-sum bound, last part: after the 2-D prefix sum D(p) bounds
// 2^24 sum_x k_x(p - x); its largest value over the image.
__global__ __launch_bounds__(256) void k_adj_colsum_max(const uint64_t *__restrict__ D, int64_t H, int64_t W,
                                                        int32_t *status) {
    __shared__ uint64_t s_m[4];
    uint64_t m = 0;
    const int64_t W1 = W + 1;
    for (int64_t y = blockIdx.x; y < H; y += gridDim.x)
        for (int64_t x = threadIdx.x; x < W; x += blockDim.x) m = max(m, D[y * W1 + x]);
    for (int d = 32; d >= 1; d >>= 1) m = max(m, (uint64_t)__shfl_xor((unsigned long long)m, d, 64));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) m = max(m, s_m[k]);
        atomicMax(reinterpret_cast<unsigned long long *>(status + ST_COLSUM_MAX), (unsigned long long)m);
    }
}

__global__ void k_adj_choose_Fg(int32_t *status) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const float gmax = __uint_as_float((unsigned)status[ST_G_ABSMAX_BITS]);
    const uint64_t dmax = *reinterpret_cast<const uint64_t *>(status + ST_COLSUM_MAX);
    int Fg = 0;
    if (gmax > 0.0f && dmax > 0) {
        // |V| <= 2 * 2^Fg * max|g| * max_p sum_x k_x(p - x) < 2^63, and every
        // |omega| <= 2^Fg max|g| kmax stays below that too
        const double P = (double)gmax * __builtin_ldexp((double)dmax, -kKmaxBits) * (1.0 + 0x1p-40);
        int e;
        const double m = __builtin_frexp(P, &e);
        const int ceil_log2_P = (m == 0.5) ? e - 1 : e;
        Fg = 62 - ceil_log2_P;
    }
    status[ST_FG] = Fg;
}

__global__ __launch_bounds__(256) void k_fill_zero(int64_t *__restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

// Tap patterns of the tied order-2 operators along one direction, tap index
// p = 3 * cluster + sub (clusters T = 2R + sub, M = -2 + sub, B = -2R - 4 + sub):
//   aa = T0 - 2 M1 + B2,  ab = T1 - M0 - M2 + B1,  bb = T2 - 2 M1 + B0.
// expand3 gives the weight of tap p from the three operator weights.
__device__ __forceinline__ int64_t expand3(int p, const int64_t v[3]) {
    switch (p) {
    case 0: return v[0];
    case 1: return v[1];
    case 2: return v[2];
    case 3: return -v[1];
    case 4: return -2 * (v[0] + v[2]);
    case 5: return -v[1];
    case 6: return v[2];
    case 7: return v[1];
    default: return v[0];
    }
}

// One pixel's scatter straight into the window (global atomics).
__device__ __forceinline__ void adj_t2n4_pixel(const AdjointArgs &a, int64_t x, int64_t y) {
    const int64_t HW = a.H * a.W, idx = y * a.W + x;
    const float g = a.gout[idx];
    if (!scatters(g)) return;
    const int Fg = a.status[ST_FG];
    int64_t o[4][9];
    double w[4][3];
    double den = 1.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float s = clamp_step(a.steps[a.plane[2 * k] * HW + idx], a.max_step);
        const float t = (s - 1.0f) * 0.5f;
        const float Rf = floorf(t);
        const int64_t R = (int64_t)Rf, off = a.off[2 * k];
        const double p = (double)(t - Rf), q = 1.0 - p;
        w[k][0] = q * q;
        w[k][1] = 2.0 * p * q;
        w[k][2] = p * p;
#pragma unroll
        for (int sub = 0; sub < 3; ++sub) {
            o[k][sub] = (2 * R + sub) * off;
            o[k][3 + sub] = (-2 + sub) * off;
            o[k][6 + sub] = (-2 * R - 4 + sub) * off;
        }
        den *= (double)s * (double)s;
    }
    const double fb = __builtin_ldexp((double)g / den, Fg);
    int64_t *Gh = a.Ghat + (y + a.pad_top) * a.Wp + (x + a.pad_left);
    for (int p0 = 0; p0 < 9; ++p0) {
        // X1[a1][a2][a3] = sum_a0 C0(p0, a0) omega(a0, a1, a2, a3)
        int64_t X1[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            const int a1 = q / 9, a2 = (q / 3) % 3, a3 = q % 3;
            const double r = fb * w[1][a1] * w[2][a2] * w[3][a3];
            int64_t v3[3];
            v3[0] = fixed(r * w[0][0]);
            v3[1] = fixed(r * w[0][1]);
            v3[2] = fixed(r * w[0][2]);
            X1[q] = expand3(p0, v3);
        }
        const int64_t b0 = o[0][p0];
#pragma unroll
        for (int p1 = 0; p1 < 9; ++p1) {
            int64_t X2[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int64_t v3[3] = {X1[q], X1[9 + q], X1[18 + q]};
                X2[q] = expand3(p1, v3);
            }
#pragma unroll
            for (int p2 = 0; p2 < 9; ++p2) {
                int64_t X3[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const int64_t v3[3] = {X2[q], X2[3 + q], X2[6 + q]};
                    X3[q] = expand3(p2, v3);
                }
                const int64_t b012 = b0 + o[1][p1] + o[2][p2];
#pragma unroll
                for (int p3 = 0; p3 < 9; ++p3) atomic_add_i64(Gh + b012 + o[3][p3], expand3(p3, X3));
            }
        }
    }
}


__global__ __launch_bounds__(256) void k_adj_scatter_t2n4(AdjointArgs a) {
    int64_t x, y;
    if (!pixel_of_thread(a.H, a.W, x, y)) return;
    adj_t2n4_pixel(a, x, y);
}

// ----------------------------------------------------------------------------
// The same scatter through LDS cluster boxes (directions (1,0), (0,1), (1,1),
// (1,-1), or those of Table 1 in the frame of cluster_box.h).  A 16 x 16 tile visits the 81 cluster combinations; for each,
// every pixel adds its sub-patch weights, summed per distinct point, into the
// combination's box in LDS, and after one barrier the box is added to the
// window with row-contiguous atomics and cleared.  Two LDS boxes alternate,
// so the flush of one combination and the accumulation of the next need a
// single barrier.  The weight of sub-tap q is the sum of omega over the
// operators it feeds: one per T or B direction, aa + bb (doubled) for M1 and
// ab for M0 and M2; combinations with an odd number of M clusters are
// negative, which a single negation of omega between the two parity groups
// takes care of.
// ----------------------------------------------------------------------------
// Weight of sub-tap Q of combination C: the sum of omega over the operators
// it feeds, doubled once per M1 it contains.
template <int C, int Q>
__device__ __forceinline__ uint64_t sub_weight(const uint64_t W[81]) {
    using namespace cbox;
    constexpr int c0 = cl(C, 0), c1 = cl(C, 1), c2 = cl(C, 2), c3 = cl(C, 3);
    constexpr int q0 = Q % 3, q1 = (Q / 3) % 3, q2 = (Q / 9) % 3, q3 = Q / 27;
    constexpr int n0 = (c0 == 1 && q0 == 1) ? 2 : 1, n1 = (c1 == 1 && q1 == 1) ? 2 : 1;
    constexpr int n2 = (c2 == 1 && q2 == 1) ? 2 : 1, n3 = (c3 == 1 && q3 == 1) ? 2 : 1;
    constexpr int sh = (n0 - 1) + (n1 - 1) + (n2 - 1) + (n3 - 1);
    uint64_t u = 0;
#pragma unroll
    for (int j0 = 0; j0 < n0; ++j0)
#pragma unroll
        for (int j1 = 0; j1 < n1; ++j1)
#pragma unroll
            for (int j2 = 0; j2 < n2; ++j2)
#pragma unroll
                for (int j3 = 0; j3 < n3; ++j3) {
                    const int o0 = c0 == 0 ? q0 : c0 == 2 ? 2 - q0 : (q0 == 1 ? 2 * j0 : 1);
                    const int o1 = c1 == 0 ? q1 : c1 == 2 ? 2 - q1 : (q1 == 1 ? 2 * j1 : 1);
                    const int o2 = c2 == 0 ? q2 : c2 == 2 ? 2 - q2 : (q2 == 1 ? 2 * j2 : 1);
                    const int o3 = c3 == 0 ? q3 : c3 == 2 ? 2 - q3 : (q3 == 1 ? 2 * j3 : 1);
                    u += W[jidx(o0, o1, o2, o3)];
                }
    return u << sh;
}

template <int C, int P, int I>
__device__ __forceinline__ uint64_t point_weight(const uint64_t W[81]) {
    constexpr int Q = cbox::kPatch.q[P][I];
    if constexpr (I + 1 < cbox::kPatch.count[P]) return sub_weight<C, Q>(W) + point_weight<C, P, I + 1>(W);
    else return sub_weight<C, Q>(W);
}

// One LDS atomic per distinct patch point, points in row order.
template <int C, int P>
__device__ __forceinline__ void box_adj_points(uint64_t *__restrict__ p, const uint64_t W[81]) {
    if constexpr (cbox::kPatch.count[P] > 0)
        __hip_atomic_fetch_add(p + cbox::point_elem(P), point_weight<C, P, 0>(W), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    if constexpr (P + 1 < 49) box_adj_points<C, P + 1>(p, W);
}

// Frame 1 (the directions of Table 1): the sub-taps at each point X + 13 Y
// of the 13 x 13 patch (at most two share a point), and one LDS atomic per
// point hit, points in row order.
struct F1Patch {
    int count[13 * 13];
    int q[13 * 13][2];
};
__host__ __device__ constexpr F1Patch make_f1_patch() {
    F1Patch t{};
    for (int q = 0; q < 81; ++q) {
        const int q0 = q % 3, q1 = (q / 3) % 3, q2 = (q / 9) % 3, q3 = q / 27;
        const int P = cbox::sub_dx<1>(q0, q1, q2, q3) + 13 * cbox::sub_row<1>(q0, q1, q2, q3);
        t.q[P][t.count[P]++] = q;
    }
    return t;
}
constexpr F1Patch kF1Patch = make_f1_patch();
static_assert(cbox::patch_w<1>() == 13 && cbox::patch_h<1>() == 13, "frame 1 patch");

template <int C, int P>
__device__ __forceinline__ void box_adj_points_f1(uint64_t *__restrict__ p, const uint64_t W[81]) {
    if constexpr (kF1Patch.count[P] > 0) {
        uint64_t v = sub_weight<C, kF1Patch.q[P][0]>(W);
        if constexpr (kF1Patch.count[P] > 1) v += sub_weight<C, kF1Patch.q[P][1]>(W);
        __hip_atomic_fetch_add(p + (P % 13) + cbox::kPitch * (P / 13), v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if constexpr (P + 1 < 13 * 13) box_adj_points_f1<C, P + 1>(p, W);
}

struct AdjTile {
    int x, y;
    int R[4];
    int x_lo, x_hi, y_lo, y_hi;
    int Rlo[4], Rhi[4];
    uint32_t packed;       // cbox::pack_state: all the loop needs of the pixel
};

// Add box b of LDS buffer src to the window and clear it.
__device__ __forceinline__ void box_flush(const AdjointArgs &a, uint64_t *__restrict__ src, const cbox::Box &b) {
    const int64_t r0 = b.oy + a.pad_top, c0 = b.ox + a.pad_left;
    const int n = b.bh * cbox::kPitch;
    for (int i = threadIdx.x; i < n; i += 256) {
        const int r = i / cbox::kPitch, c = i % cbox::kPitch;
        if (c < b.bw) {
            const uint64_t v = src[i];
            if (v != 0) {
                atomic_add_i64(a.Ghat + (r0 + r) * a.Wp + c0 + c, (int64_t)v);
                src[i] = 0;
            }
        }
    }
}

template <int I, int D>
__device__ __forceinline__ void box_adj_all(const AdjointArgs &a, uint64_t *__restrict__ s_box, bool active,
                                            const AdjTile &t, uint64_t W[81]) {
    constexpr int C = cbox::order_at(I);
    const cbox::Box b = cbox::box_of<C, D>(t.x_lo, t.x_hi, t.y_lo, t.y_hi, t.Rlo, t.Rhi, (int)a.pad_left);
    if constexpr (I == cbox::kEven) {
#pragma unroll
        for (int q = 0; q < 81; ++q) W[q] = 0 - W[q];
    }
    // sums of weights are formed again in every combination rather than kept
    // alive across them (which would not fit the registers)
#pragma unroll
    for (int q = 0; q < 81; ++q) asm volatile("" : "+v"(W[q]));
    uint64_t *buf = s_box + (I & 1) * cbox::kElems;
    if (active) {
        uint64_t *p = buf + cbox::packed_base<C, D>(t.packed, t.x_lo, t.y_lo, t.Rlo, b);
        if constexpr (D == 0) box_adj_points<C, 0>(p, W);
        else box_adj_points_f1<C, 0>(p, W);
    }
    __syncthreads();  // box complete; the other buffer was flushed before the previous barrier
    box_flush(a, buf, b);
    if constexpr (I + 1 < cbox::kCombos) box_adj_all<I + 1, D>(a, s_box, active, t, W);
}

// D: the direction frame (cluster_box.h); canon_plane[k] is the step plane of
// the frame's k-th direction.
template <int D>
__global__ __launch_bounds__(256, 2) void k_adj_scatter_t2n4_box(AdjointArgs a) {
    __shared__ uint64_t s_box[2 * cbox::kElems];
    const int64_t tiles_x = (a.W + cbox::kTile - 1) / cbox::kTile, tiles_y = (a.H + cbox::kTile - 1) / cbox::kTile;
    const int64_t item = xcd_item(blockIdx.x, tiles_x * tiles_y);
    if (item >= tiles_x * tiles_y) return;
    const int64_t bx = item % tiles_x, by = item / tiles_x;
    AdjTile t;
    t.x = (int)(bx * cbox::kTile) + (threadIdx.x & 15);
    t.y = (int)(by * cbox::kTile) + (threadIdx.x >> 4);
    const bool inside = t.x < a.W && t.y < a.H;
    const int64_t HW = a.H * a.W, idx = (int64_t)t.y * a.W + t.x;
    const float g = inside ? a.gout[idx] : 0.0f;
    const bool active = inside && scatters(g);
    float ph[4];
    double den = 1.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float s = inside ? clamp_step(a.steps[a.canon_plane[k] * HW + idx], a.max_step) : 1.0f;
        const float tt = (s - 1.0f) * 0.5f;
        const float Rf = floorf(tt);
        t.R[k] = (int)Rf;
        ph[k] = tt - Rf;
        den *= (double)s * (double)s;
    }
    // tile-wide R range over the pixels that scatter
    __shared__ int s_red[4][8];
    {
        int lo[4], hi[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            lo[k] = active ? t.R[k] : 0x7fffffff;
            hi[k] = active ? t.R[k] : -0x7fffffff;
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
            t.Rlo[k] = __builtin_amdgcn_readfirstlane(
                min(min(s_red[0][k], s_red[1][k]), min(s_red[2][k], s_red[3][k])));
            t.Rhi[k] = __builtin_amdgcn_readfirstlane(
                max(max(s_red[0][4 + k], s_red[1][4 + k]), max(s_red[2][4 + k], s_red[3][4 + k])));
        }
    }
    if (t.Rlo[0] > t.Rhi[0]) return;  // nothing in the tile scatters
    t.x_lo = (int)(bx * cbox::kTile);
    t.y_lo = (int)(by * cbox::kTile);
    t.x_hi = (int)min((int64_t)t.x_lo + cbox::kTile - 1, a.W - 1);
    t.y_hi = (int)min((int64_t)t.y_lo + cbox::kTile - 1, a.H - 1);
    if (!cbox::boxes_fit<D>(t.x_lo, t.x_hi, t.y_lo, t.y_hi, t.Rlo, t.Rhi)) {
        if (active) adj_t2n4_pixel(a, t.x, t.y);
        return;
    }
    t.packed = cbox::pack_state(threadIdx.x & 15, threadIdx.x >> 4, t.R, t.Rlo, active);
    // fixed-point weights of the 81 operator combinations
    uint64_t W[81];
    {
        double w[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double pk = (double)ph[k], qk = 1.0 - pk;
            w[k][0] = qk * qk;
            w[k][1] = 2.0 * pk * qk;
            w[k][2] = pk * pk;
        }
        const double fb = active ? __builtin_ldexp((double)g / den, a.status[ST_FG]) : 0.0;
#pragma unroll
        for (int o1 = 0; o1 < 3; ++o1)
#pragma unroll
            for (int o2 = 0; o2 < 3; ++o2)
#pragma unroll
                for (int o3 = 0; o3 < 3; ++o3) {
                    const double r = fb * w[1][o1] * w[2][o2] * w[3][o3];
#pragma unroll
                    for (int o0 = 0; o0 < 3; ++o0) W[cbox::jidx(o0, o1, o2, o3)] = (uint64_t)fixed(r * w[0][o0]);
                }
    }
    for (int i = threadIdx.x; i < 2 * cbox::kElems; i += 256) s_box[i] = 0;
    __syncthreads();
    box_adj_all<0, D>(a, s_box, active, t, W);
}

// Any factor count: per factor the narrow and wide boxes, 2^M box choices e
// with weights prod_j (e_j ? phi_j : 1 - phi_j), each spread over its 2^M taps.
__global__ __launch_bounds__(256) void k_adj_scatter_generic(AdjointArgs a) {
    int64_t x, y;
    if (!pixel_of_thread(a.H, a.W, x, y)) return;
    const int M = a.M;
    const int64_t HW = a.H * a.W, idx = y * a.W + x;
    const float g = a.gout[idx];
    if (!scatters(g)) return;
    const int Fg = a.status[ST_FG];
    int64_t pos[BSF_MAX_FACTORS][4];
    double ph[BSF_MAX_FACTORS];
    double den = 1.0;
    for (int j = 0; j < M; ++j) {
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
    const double fb = __builtin_ldexp((double)g / den, Fg);
    int64_t *Gh = a.Ghat + (y + a.pad_top) * a.Wp + (x + a.pad_left);
    const int n = 1 << M;
    for (int e = 0; e < n; ++e) {
        double w = fb;
        for (int j = 0; j < M; ++j) w *= (e >> j & 1) ? ph[j] : 1.0 - ph[j];
        const int64_t om = fixed(w);
        if (om == 0) continue;
        for (int t = 0; t < n; ++t) {
            int64_t off = 0;
            for (int j = 0; j < M; ++j) off += pos[j][2 * (e >> j & 1) + (t >> j & 1)];
            atomic_add_i64(Gh + off, (__builtin_popcount(t) & 1) ? -om : om);
        }
    }
}

// grad_img = 2^-Fg * (S^T scattered)(x) on the image; grad_steps = g * dout/ds.
__global__ __launch_bounds__(256) void k_adj_finish(const int64_t *__restrict__ Ghat, int64_t Wp, int64_t pad_top,
                                                    int64_t pad_left, int64_t H, int64_t W,
                                                    const int32_t *__restrict__ status, float *__restrict__ grad_img,
                                                    const float *__restrict__ gout,
                                                    const float *__restrict__ dsteps, float *__restrict__ grad_steps,
                                                    int planes) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= W) return;
    const int64_t HW = H * W;
    const int Fg = status[ST_FG];
    const bool poisoned = status[ST_G_NONFINITE] != 0;
    for (int64_t y = blockIdx.y; y < H; y += gridDim.y) {
        const int64_t idx = y * W + x;
        if (grad_img)
            grad_img[idx] = poisoned ? __builtin_nanf("")
                                     : (float)__builtin_ldexp((double)Ghat[(y + pad_top) * Wp + (x + pad_left)], -Fg);
        if (grad_steps) {
            const float g = gout[idx];
            for (int q = 0; q < planes; ++q) grad_steps[q * HW + idx] = g * dsteps[q * HW + idx];
        }
    }
}

#ifndef BSF_ADJOINT_FRAME1_UNIT
}  // namespace

int64_t fill_blocks(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return b < 1 ? 1 : b > 65536 ? 65536 : b;
}

bsf_status run_adjoint_scatter(const Plan &p, const AdjointArgs &a, int32_t *status, void *aux, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_begin, dim3(1), dim3(64), 0, st, status);
    BSF_HIP_CHECK(hipGetLastError());
    int64_t blocks = p.H < 2048 ? p.H : 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_adj_gmax, dim3((unsigned)blocks), dim3(256), 0, st, a.gout, p.H, p.W, status);
    BSF_HIP_CHECK(hipGetLastError());
    dim3 grid((unsigned)((p.W + kTile - 1) / kTile), (unsigned)((p.H + kTile - 1) / kTile));
    // the column-sum bound, built in the window's memory before the scatter
    const int64_t nd = (p.H + 1) * (p.W + 1);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)fill_blocks(nd)), dim3(256), 0, st, a.Ghat, nd);
    BSF_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_adj_colsum_scatter, grid, dim3(256), 0, st, a, reinterpret_cast<uint64_t *>(a.Ghat));
    BSF_HIP_CHECK(hipGetLastError());
    bsf_status r = run_prefix2d(a.Ghat, p.H + 1, p.W + 1, aux, status, st);
    if (r != BSF_OK) return r;
    hipLaunchKernelGGL(k_adj_colsum_max, dim3((unsigned)blocks), dim3(256), 0, st,
                       reinterpret_cast<const uint64_t *>(a.Ghat), p.H, p.W, status);
    BSF_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_adj_choose_Fg, dim3(1), dim3(64), 0, st, status);
    BSF_HIP_CHECK(hipGetLastError());
    const int64_t n = p.Hp * p.Wp;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)fill_blocks(n)), dim3(256), 0, st, a.Ghat, n);
    BSF_HIP_CHECK(hipGetLastError());
    if (p.n_dirs == 4 && p.order == 2 && p.tied && a.canon == 1)
        hipLaunchKernelGGL(k_adj_scatter_t2n4_box<0>, dim3((unsigned)xcd_grid((int64_t)grid.x * grid.y)), dim3(256),
                           0, st, a);
    else if (p.n_dirs == 4 && p.order == 2 && p.tied && a.canon == 2) {
        const bsf_status r = launch_adj_scatter_f1(a, dim3((unsigned)xcd_grid((int64_t)grid.x * grid.y)), st);
        if (r != BSF_OK) return r;
    } else if (p.n_dirs == 4 && p.order == 2 && p.tied)
        hipLaunchKernelGGL(k_adj_scatter_t2n4, grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_adj_scatter_generic, grid, dim3(256), 0, st, a);
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

bsf_status run_adjoint_finish(const Plan &p, const int64_t *Ghat, const int32_t *status, float *grad_img,
                              const float *gout, const float *dsteps, float *grad_steps, hipStream_t st) {
    dim3 grid((unsigned)((p.W + 255) / 256), (unsigned)(p.H < 4096 ? p.H : 4096));
    hipLaunchKernelGGL(k_adj_finish, grid, dim3(256), 0, st, Ghat, p.Wp, p.pad_top, p.pad_left, p.H, p.W, status,
                       grad_img, gout, dsteps, grad_steps, p.planes);
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

}  // namespace bsf

#else  // BSF_ADJOINT_FRAME1_UNIT: the cluster-box scatter of Table 1's directions
}  // namespace

bsf_status launch_adj_scatter_f1(const AdjointArgs &a, dim3 grid, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_scatter_t2n4_box<1>, grid, dim3(256), 0, st, a);
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

}  // namespace bsf
#endif
