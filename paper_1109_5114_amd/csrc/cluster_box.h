// Cluster boxes of the tied order-2 filter along four directions u_0..u_3
// (Section 1.1 with the box factors of Table 1 used twice per direction), in
// one of two fixed frames: D = 0 is Section 1.1's set (1,0), (0,1), (1,1),
// (1,-1); D = 1 is the set of Table 1, (2,1), (1,2), (1,-2), (2,-1), that
// Alg. 2 switches to in the sectors Section 1.1's set covers badly.
//
// Along u_k the nine taps of a pixel (Alg. 3 step 3, squared difference
// operator) lie in three clusters of three consecutive lattice points,
//     T = 2R + {0,1,2},   M = -2 + {0,1,2},   B = -2R - 4 + {0,1,2},
// with R = floor((s-1)/2) of the pixel's step.  Picking one cluster per
// direction (a combination; 81 in all) leaves 3^4 taps that sit at
// anchor + sum_k q_k u_k, q in {0,1,2}^4, where anchor = x + sum_k base_k u_k:
// in frame 0 a 7 x 7 patch with 37 distinct points, in frame 1 a 13 x 13 patch
// with 73.  Over a tile of pixels the anchors move with the pixel and with
// 2 (R - R') along u_k, so a combination of a tile reaches one small box of
// the running-sum window.  The gather stages that box in LDS and reads it at
// static offsets; the adjoint accumulates into it and adds it to the window
// once.
//
// The tensor of the 81 exact integer values J[o0][o1][o2][o3] (o = aa, ab,
// bb per direction; the order-2 operators
//     aa = T0 - 2 M1 + B2,   ab = T1 - M0 - M2 + B1,   bb = T2 - 2 M1 + B0)
// is the sum over the combinations of their sub-patch, mapped per direction:
// a T tap q feeds o = q, a B tap q feeds o = 2 - q, M1 feeds aa and bb with
// weight 2 and M0, M2 feed ab; every M tap is negative, so the sign of a whole
// combination is (-1)^(number of M clusters).
#pragma once

#include "bsf_common.h"

namespace bsf {
namespace cbox {

constexpr int kTile = 16;                 // tile side, pixels
constexpr int kPitch = 64;                // LDS box row pitch, elements
constexpr int kRows = 48;                 // LDS box rows
constexpr int kElems = kPitch * kRows;    // 24 KiB of int64
constexpr int kCombos = 81;
constexpr int kEven = 41;                 // combinations with an even number of M clusters

// Cluster of direction k in combination C: 0 = T, 1 = M, 2 = B.
__host__ __device__ constexpr int cl(int C, int k) {
    return k == 0 ? C % 3 : k == 1 ? (C / 3) % 3 : k == 2 ? (C / 9) % 3 : (C / 27) % 3;
}
__host__ __device__ constexpr int n_m(int C) {
    return (cl(C, 0) == 1) + (cl(C, 1) == 1) + (cl(C, 2) == 1) + (cl(C, 3) == 1);
}
// The I-th combination: those with an even number of M clusters first.
__host__ __device__ constexpr int order_at(int I) {
    int seen = 0;
    for (int parity = 0; parity < 2; ++parity)
        for (int C = 0; C < kCombos; ++C)
            if ((n_m(C) & 1) == parity) {
                if (seen == I) return C;
                ++seen;
            }
    return -1;
}

// Per direction, a combination's sub-patch is reduced to "rows" r: a T or B
// cluster keeps its three taps (r = q); an M cluster has two, r = 0 for M1
// (feeding aa and bb, doubled) and r = 1 for M0 + M2 (feeding ab).
__host__ __device__ constexpr int n_rows(int c) { return c == 1 ? 2 : 3; }
__host__ __device__ constexpr int n_sub(int c, int r) { return (c == 1 && r == 1) ? 2 : 1; }
__host__ __device__ constexpr int sub_q(int c, int r, int i) { return c == 1 ? (r == 0 ? 1 : 2 * i) : r; }
__host__ __device__ constexpr int n_out(int c, int r) { return (c == 1 && r == 0) ? 2 : 1; }
__host__ __device__ constexpr int out_o(int c, int r, int j) {
    return c == 0 ? r : c == 2 ? 2 - r : (r == 0 ? 2 * j : 1);
}
__host__ __device__ constexpr int doubled(int c, int r) { return (c == 1 && r == 0) ? 1 : 0; }
__host__ __device__ constexpr int jidx(int o0, int o1, int o2, int o3) { return ((o0 * 3 + o1) * 3 + o2) * 3 + o3; }

// The two frames: u_k = (ux[k], uy[k]).  A pixel's patch spans columns
// X = 0 .. PX - 1 and rows Y = Y0 .. Y0 + PY - 1 around its anchor.
template <int D>
struct Frame;
template <>
struct Frame<0> {
    static constexpr int ux[4] = {1, 0, 1, 1};
    static constexpr int uy[4] = {0, 1, 1, -1};
};
template <>
struct Frame<1> {
    static constexpr int ux[4] = {2, 1, 1, 2};
    static constexpr int uy[4] = {1, 2, -2, -1};
};
template <int D>
__host__ __device__ constexpr int patch_w() {
    return 1 + 2 * (Frame<D>::ux[0] + Frame<D>::ux[1] + Frame<D>::ux[2] + Frame<D>::ux[3]);
}
template <int D>
__host__ __device__ constexpr int patch_h() {
    int h = 1;
    for (int k = 0; k < 4; ++k) h += 2 * (Frame<D>::uy[k] < 0 ? -Frame<D>::uy[k] : Frame<D>::uy[k]);
    return h;
}
template <int D>
__host__ __device__ constexpr int patch_y0() {
    int y = 0;
    for (int k = 0; k < 4; ++k) y += Frame<D>::uy[k] < 0 ? 2 * Frame<D>::uy[k] : 0;
    return y;
}
// Offset of sub-tap q from the anchor, and its patch row Y - Y0.
template <int D>
__host__ __device__ constexpr int sub_dx(int q0, int q1, int q2, int q3) {
    return q0 * Frame<D>::ux[0] + q1 * Frame<D>::ux[1] + q2 * Frame<D>::ux[2] + q3 * Frame<D>::ux[3];
}
template <int D>
__host__ __device__ constexpr int sub_row(int q0, int q1, int q2, int q3) {
    return q0 * Frame<D>::uy[0] + q1 * Frame<D>::uy[1] + q2 * Frame<D>::uy[2] + q3 * Frame<D>::uy[3] - patch_y0<D>();
}

// LDS element offset of sub-tap q from the pixel's base (its patch row Y0).
template <int D = 0>
__host__ __device__ constexpr int sub_elem(int q0, int q1, int q2, int q3) {
    return sub_dx<D>(q0, q1, q2, q3) + kPitch * sub_row<D>(q0, q1, q2, q3);
}

// The sub-taps q (index q0 + 3 q1 + 9 q2 + 27 q3) at each of the 7 x 7 patch
// points P = X + 7 (Y + 2) of frame 0; 37 points are hit, by at most five
// sub-taps.
struct PatchTable {
    int count[49];
    int q[49][5];
};
__host__ __device__ constexpr PatchTable make_patch_table() {
    PatchTable t{};
    for (int q = 0; q < 81; ++q) {
        const int q0 = q % 3, q1 = (q / 3) % 3, q2 = (q / 9) % 3, q3 = q / 27;
        const int P = (q0 + q2 + q3) + 7 * (q1 + q2 - q3 + 2);
        t.q[P][t.count[P]++] = q;
    }
    return t;
}
constexpr PatchTable kPatch = make_patch_table();
__host__ __device__ constexpr int point_elem(int P) { return (P % 7) + kPitch * (P / 7); }

__host__ __device__ __forceinline__ int base_of(int c, int R) { return c == 0 ? 2 * R : c == 1 ? -2 : -2 * R - 4; }

// Box of combination C for a tile whose active pixels span [x_lo, x_hi] x
// [y_lo, y_hi] with R_k in [Rlo_k, Rhi_k]: image coordinates (ox, oy) of box
// element (0, 0), width and height.  The box starts on an even window column
// (widened by one column on the left when needed), so that it can be copied
// in aligned pairs of elements; a pair may then end one column past the box,
// which the window's spare right column keeps inside the window.
struct Box {
    int ox, oy, bw, bh;
};

template <int C, int D = 0>
__host__ __device__ __forceinline__ Box box_of(int x_lo, int x_hi, int y_lo, int y_hi, const int Rlo[4], const int Rhi[4],
                                      int pad_left) {
    using U = Frame<D>;
    int bmin[4], bmax[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = cl(C, k);
        bmin[k] = c == 0 ? 2 * Rlo[k] : c == 1 ? -2 : -2 * Rhi[k] - 4;
        bmax[k] = c == 0 ? 2 * Rhi[k] : c == 1 ? -2 : -2 * Rlo[k] - 4;
    }
    int ax_min, ax_max, ay_min, ay_max;
    if constexpr (D == 0) {
        ax_min = x_lo + bmin[0] + bmin[2] + bmin[3];
        ax_max = x_hi + bmax[0] + bmax[2] + bmax[3];
        ay_min = y_lo + bmin[1] + bmin[2] - bmax[3];
        ay_max = y_hi + bmax[1] + bmax[2] - bmin[3];
    } else {
        ax_min = x_lo, ax_max = x_hi, ay_min = y_lo, ay_max = y_hi;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            ax_min += bmin[k] * U::ux[k];  // ux >= 0 in both frames
            ax_max += bmax[k] * U::ux[k];
            ay_min += (U::uy[k] >= 0 ? bmin[k] : bmax[k]) * U::uy[k];
            ay_max += (U::uy[k] >= 0 ? bmax[k] : bmin[k]) * U::uy[k];
        }
    }
    const int odd = (ax_min + pad_left) & 1;
    return Box{ax_min - odd, ay_min + patch_y0<D>(), ax_max - ax_min + patch_w<D>() + odd,
               ay_max - ay_min + patch_h<D>()};
}

// LDS element of the pixel's patch row Y0, column X = 0.
template <int C, int D = 0>
__host__ __device__ __forceinline__ int pixel_base(int x, int y, const int R[4], const Box &b) {
    using U = Frame<D>;
    int ax = x, ay = y;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int bk = base_of(cl(C, k), R[k]);
        ax += bk * U::ux[k];
        ay += bk * U::uy[k];
    }
    return (ay + patch_y0<D>() - b.oy) * kPitch + (ax - b.ox);
}

// (These index functions are also compiled for the host, where a test walks
// them over random tiles, step ranges and window geometries.)
//
// The pixel's state through a combination loop, in one register: bits 0-9
// hold tx + 64 ty (its position in the 16 x 16 tile), then R_k - Rlo_k in five
// bits per direction (at most 20 whenever the boxes fit).  Inactive pixels
// store zero differences.
__host__ __device__ __forceinline__ uint32_t pack_state(int tx, int ty, const int R[4], const int Rlo[4], bool active) {
    uint32_t st = (uint32_t)(tx + kPitch * ty);
#pragma unroll
    for (int k = 0; k < 4; ++k) st |= (uint32_t)(active ? R[k] - Rlo[k] : 0) << (10 + 5 * k);
    return st;
}

// pixel_base from the packed state: 64 ty + tx + sum_k coef_k b_k with
// coef_k = ux_k + 64 uy_k the LDS offset of u_k ((1, 64, 65, -63) in frame 0,
// (66, 129, -127, -62) in frame 1) and b_k = 2 R_k (T), -2 (M), -2 R_k - 4 (B);
// the tile-uniform part is formed once per combination.
template <int C, int D = 0>
__host__ __device__ __forceinline__ int packed_base(uint32_t st, int x_lo, int y_lo, const int Rlo[4], const Box &b) {
    static_assert(kPitch == 64, "coefficients assume a 64-element pitch");
    using U = Frame<D>;
    int v = (int)(st & 1023u);
    int sc = kPitch * (y_lo + patch_y0<D>() - b.oy) + (x_lo - b.ox);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = cl(C, k);
        const int coef = U::ux[k] + kPitch * U::uy[k];
        const int dR = (int)((st >> (10 + 5 * k)) & 31u);
        if (c == 0) {
            v += 2 * coef * dR;
            sc += 2 * coef * Rlo[k];
        } else if (c == 2) {
            v -= 2 * coef * dR;
            sc += coef * (-2 * Rlo[k] - 4);
        } else {
            sc += -2 * coef;
        }
    }
    return v + sc;
}

// Largest box over the combinations (all clusters T or B, one column of
// alignment) fits an LDS box of the given number of rows.
template <int D = 0>
__host__ __device__ __forceinline__ bool boxes_fit(int x_lo, int x_hi, int y_lo, int y_hi, const int Rlo[4],
                                          const int Rhi[4], int rows = kRows) {
    using U = Frame<D>;
    const int d0 = Rhi[0] - Rlo[0], d1 = Rhi[1] - Rlo[1], d2 = Rhi[2] - Rlo[2], d3 = Rhi[3] - Rlo[3];
    if constexpr (D == 0) {
        const int w = (x_hi - x_lo) + 8 + 2 * (d0 + d2 + d3);
        const int h = (y_hi - y_lo) + 7 + 2 * (d1 + d2 + d3);
        return w <= kPitch && h <= rows;
    }
    const int d[4] = {d0, d1, d2, d3};
    int w = (x_hi - x_lo) + patch_w<D>() + 1, h = (y_hi - y_lo) + patch_h<D>();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        w += 2 * d[k] * U::ux[k];
        h += 2 * d[k] * (U::uy[k] < 0 ? -U::uy[k] : U::uy[k]);
    }
    return w <= kPitch && h <= rows;
}

}  // namespace cbox
}  // namespace bsf
