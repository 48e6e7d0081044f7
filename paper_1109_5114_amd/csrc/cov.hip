// Steps from a covariance field (Section 1.1, eq. cov and eq. geometry; the
// minimum-kurtosis choice of the scales, Section 1.1 and Section 2.4).
//
// A box spline with one box of s_k lattice steps along each integer direction
// u_k has covariance sum_k A_k u_k u_k^T, A_k = s_k^2 / 12 (a length-s box has
// variance s^2 / 12 along its line).  For four directions the three entries of
// C leave one free parameter: A(t) = A0 + t n with n spanning the null space of
// A -> sum_k A_k u_k u_k^T, A0 a particular solution, t restricted to A(t) >= 0.
// The scales are those of minimum kurtosis: the Frobenius norm of
// sum_k a_k^4 uhat_k uhat_k^T (a_k = s_k |u_k|, uhat_k = u_k / |u_k|), i.e. of
// K(t) = sum_k A_k(t)^2 |u_k|^2 u_k u_k^T up to a constant.  ||K(t)||_F^2 is a
// quartic in t; its minimum over the feasible interval is at an end or at a
// real root of the cubic derivative, solved in closed form and polished by
// Newton steps.  An order-r tied filter splits C evenly over its r copies.
// Steps are floored at one lattice step; a covariance the directions cannot
// reach (too elongated for its orientation, or not positive definite) gets
// the scales that keep min_k A_k largest, and BSF_FLAG_RANGE.
#include <math.h>
#include <string.h>

#include "bsf_common.h"

namespace bsf {
namespace {

__device__ __forceinline__ float clamp_top(float s, float max_step, bool &over) {
    over = over || !(s <= max_step);
    return fminf(s, max_step);
}

// Real roots of a3 t^3 + a2 t^2 + a1 t + a0 (a3 > 0); returns their count.
__device__ int cubic_roots(double a3, double a2, double a1, double a0, double r[3]) {
    const double b = a2 / a3, c = a1 / a3, d = a0 / a3;
    const double p = c - b * b / 3.0, q = 2.0 * b * b * b / 27.0 - b * c / 3.0 + d;
    const double shift = -b / 3.0;
    const double disc = 0.25 * q * q + p * p * p / 27.0;
    int n;
    if (disc > 0.0) {
        const double sq = sqrt(disc);
        r[0] = cbrt(-0.5 * q + sq) + cbrt(-0.5 * q - sq) + shift;
        n = 1;
    } else if (p == 0.0) {
        r[0] = shift;
        n = 1;
    } else {
        const double m = 2.0 * sqrt(-p / 3.0);
        double arg = 3.0 * q / (p * m);
        arg = fmin(1.0, fmax(-1.0, arg));
        const double th = acos(arg) / 3.0;
        r[0] = m * cos(th) + shift;
        r[1] = m * cos(th - 2.0943951023931957) + shift;
        r[2] = m * cos(th - 4.1887902047863905) + shift;
        n = 3;
    }
    // Newton polish on the cubic
    for (int i = 0; i < n; ++i)
        for (int it = 0; it < 2; ++it) {
            const double t = r[i];
            const double f = ((a3 * t + a2) * t + a1) * t + a0, df = (3.0 * a3 * t + 2.0 * a2) * t + a1;
            if (df != 0.0) r[i] = t - f / df;
        }
    return n;
}

struct Quartic {
    double al[3], be[3], ga[3];  // K_e(t) = al t^2 + be t + ga, e = 11, 12, 22
    __device__ double f(double t) const {
        double s = 0.0;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const double k = (al[e] * t + be[e]) * t + ga[e];
            s += (e == 1 ? 2.0 : 1.0) * k * k;
        }
        return s;
    }
};

// Steps of one pixel; returns true when C was out of reach.
__device__ bool steps_of_cov(const CovBank &bk, double c11, double c12, double c22, double s_out[4]) {
    const double tr = c11 + c22;
    if (!(tr > 0.0) || !(tr < 1e300)) {  // NaN, infinite, or not a covariance
#pragma unroll
        for (int k = 0; k < 4; ++k) s_out[k] = 1.0;
        return true;
    }
    const double c[3] = {c11 / tr, c12 / tr, c22 / tr};
    double A0[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) A0[k] = bk.P[k][0] * c[0] + bk.P[k][1] * c[1] + bk.P[k][2] * c[2];
    double lo = -1e300, hi = 1e300;
    bool feasible = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (bk.n[k] > 0.0) lo = fmax(lo, -A0[k] / bk.n[k]);
        else if (bk.n[k] < 0.0) hi = fmin(hi, -A0[k] / bk.n[k]);
        else if (A0[k] < 0.0) feasible = false;
    }
    double t;
    if (feasible && lo <= hi) {
        Quartic q;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            q.al[e] = q.be[e] = q.ga[e] = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                q.al[e] += bk.w[e][k] * bk.n[k] * bk.n[k];
                q.be[e] += 2.0 * bk.w[e][k] * A0[k] * bk.n[k];
                q.ga[e] += bk.w[e][k] * A0[k] * A0[k];
            }
        }
        // f'(t) / 2 = sum_e c_e K_e K_e'
        double a3 = 0.0, a2 = 0.0, a1 = 0.0, a0 = 0.0;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const double ce = e == 1 ? 2.0 : 1.0;
            a3 += ce * 2.0 * q.al[e] * q.al[e];
            a2 += ce * 3.0 * q.al[e] * q.be[e];
            a1 += ce * (q.be[e] * q.be[e] + 2.0 * q.al[e] * q.ga[e]);
            a0 += ce * q.be[e] * q.ga[e];
        }
        t = lo;
        double fb = q.f(lo);
        const double fh = q.f(hi);
        if (fh < fb) {
            t = hi;
            fb = fh;
        }
        if (a3 > 0.0) {
            double r[3];
            const int nr = cubic_roots(a3, a2, a1, a0, r);
            for (int i = 0; i < nr; ++i)
                if (r[i] > lo && r[i] < hi) {
                    const double fr = q.f(r[i]);
                    if (fr < fb) {
                        fb = fr;
                        t = r[i];
                    }
                }
        }
    } else {
        // out of reach: the crossing of two lines A_i(t) = A_j(t) with the
        // largest min_k A_k(t)
        feasible = false;
        double vb = -1e300;
        t = 0.0;
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j) {
                if (bk.n[i] == bk.n[j]) continue;
                const double tc = (A0[j] - A0[i]) / (bk.n[i] - bk.n[j]);
                double v = 1e300;
#pragma unroll
                for (int k = 0; k < 4; ++k) v = fmin(v, A0[k] + tc * bk.n[k]);
                if (v > vb) {
                    vb = v;
                    t = tc;
                }
            }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double A = fmax(A0[k] + t * bk.n[k], 0.0) * tr;
        s_out[k] = fmax(sqrt(12.0 * A), 1.0);
    }
    return !feasible;
}

// Orientation of C in [0, pi) (top eigenvector) and its sector of Alg. 2:
// 0 when an axis of the first box spline (0, 45, 90, 135 degrees) is nearer
// than one of the second (atan 1/2, atan 2 and their mirrors), else 1.
__device__ int bank_of_cov(double c11, double c12, double c22) {
    double phi = 0.5 * atan2(2.0 * c12, c11 - c22);
    if (phi < 0.0) phi += M_PI;
    const double ax1[4] = {0.0, 0.25 * M_PI, 0.5 * M_PI, 0.75 * M_PI};
    const double t2 = atan(0.5), t3 = atan(2.0);
    const double ax2[4] = {t2, t3, M_PI - t3, M_PI - t2};
    double d1 = 1e30, d2 = 1e30;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double d = fabs(phi - ax1[k]);
        d1 = fmin(d1, fmin(d, M_PI - d));
        d = fabs(phi - ax2[k]);
        d2 = fmin(d2, fmin(d, M_PI - d));
    }
    return d2 < d1 ? 1 : 0;
}

// Per pixel: C (three planes) minus sub I, split over the r copies, mapped to
// steps.  With two banks (bk2 non-null), the pixel's sector picks the bank;
// its steps go to that bank's planes and the other bank's planes get 1, and
// sel (nullable) records the bank.
__global__ __launch_bounds__(256) void k_cov_to_steps(CovBank b1, CovBank b2, int two_banks, const float *__restrict__ cov,
                                                      int64_t H, int64_t W, const float *__restrict__ sub_dev, float sub,
                                                      float *__restrict__ steps1, float *__restrict__ steps2,
                                                      uint8_t *__restrict__ sel, int order, int tied, float max_step,
                                                      int32_t *status) {
    const int64_t HW = H * W;
    const float s_sub = sub_dev ? *sub_dev : sub;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < HW; i += (int64_t)gridDim.x * blockDim.x) {
        const double c11 = (double)cov[i] - s_sub, c12 = (double)cov[HW + i], c22 = (double)cov[2 * HW + i] - s_sub;
        int bank = 0;
        if (two_banks) bank = bank_of_cov(c11, c12, c22);
        double s[4];
        const CovBank &bk = bank ? b2 : b1;
        if (steps_of_cov(bk, c11 / order, c12 / order, c22 / order, s)) bad = true;
        float *dst = bank ? steps2 : steps1;
        float *other = bank ? steps1 : steps2;
        const int per = tied ? 1 : order;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float v = clamp_top((float)s[k], max_step, bad);
            for (int q = 0; q < per; ++q) {
                dst[(int64_t)(k * per + q) * HW + i] = v;
                if (two_banks) other[(int64_t)(k * per + q) * HW + i] = 1.0f;
            }
        }
        if (sel) sel[i] = (uint8_t)bank;
    }
    if (__any(bad)) {
        if ((threadIdx.x & 63) == 0) atomicOr((unsigned *)&status[ST_FLAGS], BSF_FLAG_RANGE);
    }
}

}  // namespace

// The null vector and a particular solution of the covariance constraints for
// the plan's four directions (in plan order), and the weights of K.
bsf_status make_cov_bank(const Plan &p, CovBank *b) {
    if (p.n_dirs != 4) return BSF_E_UNSUPPORTED;
    double M[3][4];
    for (int k = 0; k < 4; ++k) {
        const double ux = p.dx[k], uy = p.dy[k], n2 = ux * ux + uy * uy;
        M[0][k] = ux * ux;
        M[1][k] = ux * uy;
        M[2][k] = uy * uy;
        b->w[0][k] = n2 * ux * ux;
        b->w[1][k] = n2 * ux * uy;
        b->w[2][k] = n2 * uy * uy;
    }
    // P = M^T (M M^T)^-1, the minimum-norm particular solution
    double G[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            G[i][j] = 0.0;
            for (int k = 0; k < 4; ++k) G[i][j] += M[i][k] * M[j][k];
        }
    const double det = G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1]) -
                       G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0]) +
                       G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]);
    if (!(fabs(det) > 1e-9)) return BSF_E_INVALID;  // directions do not span the covariances
    double Gi[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
            Gi[i][j] = (G[i1][j1] * G[i2][j2] - G[i1][j2] * G[i2][j1]) / det;
        }
    for (int k = 0; k < 4; ++k)
        for (int j = 0; j < 3; ++j) {
            b->P[k][j] = 0.0;
            for (int i = 0; i < 3; ++i) b->P[k][j] += M[i][k] * Gi[i][j];
        }
    // null vector: the largest column of I - P M
    double best = -1.0;
    for (int j = 0; j < 4; ++j) {
        double v[4], nn = 0.0;
        for (int k = 0; k < 4; ++k) {
            double pm = 0.0;
            for (int i = 0; i < 3; ++i) pm += b->P[k][i] * M[i][j];
            v[k] = (k == j ? 1.0 : 0.0) - pm;
            nn += v[k] * v[k];
        }
        if (nn > best) {
            best = nn;
            for (int k = 0; k < 4; ++k) b->n[k] = v[k] / sqrt(nn);
        }
    }
    return BSF_OK;
}

bsf_status run_cov_to_steps(const Plan &p, const CovBank &b1, const CovBank *b2, const float *cov,
                            const float *sub_dev, float sub, float *steps1, float *steps2, uint8_t *sel,
                            int32_t *status, hipStream_t st) {
    const int64_t HW = p.H * p.W;
    if (HW == 0) return BSF_OK;
    int64_t blocks = (HW + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_cov_to_steps, dim3((unsigned)blocks), dim3(256), 0, st, b1, b2 ? *b2 : b1, b2 ? 1 : 0, cov,
                       p.H, p.W, sub_dev, sub, steps1, steps2, sel, p.order, p.tied, p.max_step, status);
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

}  // namespace bsf
