// Running sums on the window (Section 1.1, first step of BoxFilter; Alg. 3
// step 2: g(p) = f(p) + g(p - u)), r times per direction, in exact int64
// (wrapping modulo 2^64) or plain FP64.
//
// Rows (dy == 0) use one workgroup per row: 1024-element chunks, a thread-local
// prefix over 4 contiguous elements, a wavefront prefix (64-bit lane shuffles)
// and a cross-wave prefix through LDS, with the running carry kept in
// registers.  All other directions use sheared tiles: 64 lanes follow 64
// adjacent lines of direction u for TL steps, so every step reads 64 contiguous
// elements of one row.  A tile's carry comes from the tile before it on the
// same lines, so the scan runs in three phases (tile aggregates, a per-line scan
// of aggregates, the final rescan), none of which waits on another workgroup.
#include <type_traits>

#include "bsf_common.h"

namespace bsf {
namespace {

constexpr int kRowThreads = 256;
constexpr int kRowChunk = kRowThreads * 4;
constexpr int kLineTL = 64;  // steps per line tile

template <typename V>
__device__ __forceinline__ V shfl_up64(V v, int d) {
    return __shfl_up(v, d, 64);
}

// Exclusive prefix of `x` over the 256 threads of the block; also returns the
// block total.  `lds` holds 4 values.
template <typename V>
__device__ __forceinline__ V block_excl_scan(V x, V *lds, V &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    V inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        V t = shfl_up64(inc, d);
        if (lane >= d) inc += t;
    }
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    V w0 = lds[0], w1 = lds[1], w2 = lds[2], w3 = lds[3];
    __syncthreads();
    V before = (w >= 1 ? w0 : V(0)) + (w >= 2 ? w1 : V(0)) + (w >= 3 ? w2 : V(0));
    total = w0 + w1 + w2 + w3;
    return before + inc - x;
}

// Load one window element for pass 1 (from the image, converted) or later
// passes (from the window).
template <typename V, int SRC>
__device__ __forceinline__ V load_src(const V *G, int64_t Wp, const Src &src, int F, int64_t row, int64_t col) {
    if constexpr (SRC == SRC_WINDOW) {
        return G[row * Wp + col];
    } else {
        const int64_t y = row - src.pad_top, x = col - src.pad_left;
        if (y < 0 || x < 0 || y >= src.H || x >= src.W) return V(0);
        if constexpr (SRC == SRC_F32) {
            const float f = static_cast<const float *>(src.img)[y * src.pitch + x];
            if constexpr (std::is_integral_v<V>) {  // integer window: fixed point
                return static_cast<V>(__builtin_rint(__builtin_ldexp(static_cast<double>(f), F)));
            } else {
                return static_cast<V>(f);
            }
        } else if constexpr (SRC == SRC_U8) {
            return static_cast<V>(static_cast<const uint8_t *>(src.img)[y * src.pitch + x]);
        } else {
            return static_cast<V>(static_cast<const uint16_t *>(src.img)[y * src.pitch + x]);
        }
    }
}

template <typename V, int ORDER, int SRC>
__global__ __launch_bounds__(kRowThreads) void k_row_scan(V *__restrict__ G, int64_t Wp, int dir, Src src,
                                                          const int32_t *__restrict__ status) {
    __shared__ V lds[4];
    const int64_t row = blockIdx.x;
    const int F = (SRC == SRC_F32) ? status[ST_F_USED] : 0;
    V carry[ORDER];
#pragma unroll
    for (int o = 0; o < ORDER; ++o) carry[o] = V(0);
    for (int64_t c0 = 0; c0 < Wp; c0 += kRowChunk) {
        V v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t e = c0 + 4 * threadIdx.x + i;
            const int64_t col = dir > 0 ? e : Wp - 1 - e;
            v[i] = (e < Wp) ? load_src<V, SRC>(G, Wp, src, F, row, col) : V(0);
        }
#pragma unroll
        for (int o = 0; o < ORDER; ++o) {
            v[1] += v[0];
            v[2] += v[1];
            v[3] += v[2];
            V total;
            const V excl = block_excl_scan<V>(v[3], lds, total);
            const V add = excl + carry[o];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] += add;
            carry[o] += total;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t e = c0 + 4 * threadIdx.x + i;
            const int64_t col = dir > 0 ? e : Wp - 1 - e;
            if (e < Wp) G[row * Wp + col] = v[i];
        }
    }
}

// ----------------------------------------------------------------------------
// Sheared line tiles for dy != 0.
// ----------------------------------------------------------------------------
struct LineGeom {
    int dx, dy, ay;
    int64_t Hp, Wp;
    int64_t T;         // steps per residue class (rows / |dy|, rounded up)
    int64_t c_lo;      // start column of the first line
    int64_t n_groups;  // groups of 64 lines
    int64_t n_chunks;  // chunks of kLineTL steps
};

__device__ __forceinline__ void line_cell(const LineGeom &g, int64_t q, int64_t c0, int64_t t, int64_t &row,
                                          int64_t &col, bool &inside) {
    row = g.dy > 0 ? q + t * g.ay : g.Hp - 1 - q - t * g.ay;
    col = c0 + g.dx * t;
    inside = row >= 0 && row < g.Hp && col >= 0 && col < g.Wp;
}

// binom(n, m) for m <= 3, as V (exact in integers modulo 2^64).
template <typename V>
__device__ __forceinline__ V binom_small(int64_t n, int m) {
    if (m == 0) return V(1);
    if (m == 1) return V(n);
    if (m == 2) return V((n * (n - 1)) / 2);
    return V((n * (n - 1) * (n - 2)) / 6);
}

template <typename V, int ORDER, int SRC>
__global__ __launch_bounds__(64) void k_line_aggregate(const V *__restrict__ G, LineGeom g, Src src,
                                                       const int32_t *__restrict__ status, V *__restrict__ aux) {
    const int lane = threadIdx.x;
    const int64_t idx = blockIdx.x;
    const int64_t gi = idx % g.n_groups, ch = (idx / g.n_groups) % g.n_chunks, q = idx / (g.n_groups * g.n_chunks);
    const int64_t c0 = g.c_lo + gi * 64 + lane;
    const int64_t t0 = ch * kLineTL, t1 = min(g.T, t0 + kLineTL);
    const int F = (SRC == SRC_F32) ? status[ST_F_USED] : 0;
    V s[ORDER];
#pragma unroll
    for (int o = 0; o < ORDER; ++o) s[o] = V(0);
    for (int64_t t = t0; t < t1; ++t) {
        int64_t row, col;
        bool in;
        line_cell(g, q, c0, t, row, col, in);
        const V v = in ? load_src<V, SRC>(G, g.Wp, src, F, row, col) : V(0);
        s[0] += v;
#pragma unroll
        for (int o = 1; o < ORDER; ++o) s[o] += s[o - 1];
    }
#pragma unroll
    for (int o = 0; o < ORDER; ++o) aux[(idx * ORDER + o) * 64 + lane] = s[o];
}

template <typename V, int ORDER>
__global__ __launch_bounds__(64) void k_line_carry(LineGeom g, V *__restrict__ aux) {
    const int lane = threadIdx.x;
    const int64_t gi = blockIdx.x % g.n_groups, q = blockIdx.x / g.n_groups;
    V state[ORDER];
#pragma unroll
    for (int o = 0; o < ORDER; ++o) state[o] = V(0);
    for (int64_t ch = 0; ch < g.n_chunks; ++ch) {
        const int64_t idx = (q * g.n_chunks + ch) * g.n_groups + gi;
        const int64_t L = min(g.T, (ch + 1) * kLineTL) - ch * kLineTL;
        V agg[ORDER];
#pragma unroll
        for (int o = 0; o < ORDER; ++o) {
            agg[o] = aux[(idx * ORDER + o) * 64 + lane];
            aux[(idx * ORDER + o) * 64 + lane] = state[o];
        }
        // end-of-chunk state: s_k(L-1) = agg_k + sum_{i<=k} binom(L-1+k-i, k-i) C_i
        V next[ORDER];
#pragma unroll
        for (int k = 0; k < ORDER; ++k) {
            V acc = agg[k];
#pragma unroll
            for (int i = 0; i <= k; ++i) acc += binom_small<V>(L - 1 + k - i, k - i) * state[i];
            next[k] = acc;
        }
#pragma unroll
        for (int o = 0; o < ORDER; ++o) state[o] = next[o];
    }
}

template <typename V, int ORDER, int SRC>
__global__ __launch_bounds__(64) void k_line_final(V *__restrict__ G, LineGeom g, Src src,
                                                   const int32_t *__restrict__ status, const V *__restrict__ aux) {
    const int lane = threadIdx.x;
    const int64_t idx = blockIdx.x;
    const int64_t gi = idx % g.n_groups, ch = (idx / g.n_groups) % g.n_chunks, q = idx / (g.n_groups * g.n_chunks);
    const int64_t c0 = g.c_lo + gi * 64 + lane;
    const int64_t t0 = ch * kLineTL, t1 = min(g.T, t0 + kLineTL);
    const int F = (SRC == SRC_F32) ? status[ST_F_USED] : 0;
    V s[ORDER];
#pragma unroll
    for (int o = 0; o < ORDER; ++o) s[o] = aux[(idx * ORDER + o) * 64 + lane];
    for (int64_t t = t0; t < t1; ++t) {
        int64_t row, col;
        bool in;
        line_cell(g, q, c0, t, row, col, in);
        const V v = in ? load_src<V, SRC>(G, g.Wp, src, F, row, col) : V(0);
        s[0] += v;
#pragma unroll
        for (int o = 1; o < ORDER; ++o) s[o] += s[o - 1];
        if (in) G[row * g.Wp + col] = s[ORDER - 1];
    }
}

LineGeom line_geom(int dx, int dy, int64_t Hp, int64_t Wp) {
    LineGeom g;
    g.dx = dx;
    g.dy = dy;
    g.ay = dy > 0 ? dy : -dy;
    g.Hp = Hp;
    g.Wp = Wp;
    g.T = (Hp + g.ay - 1) / g.ay;
    const int64_t span = (int64_t)dx * (g.T - 1);
    g.c_lo = span > 0 ? -span : 0;
    const int64_t c_hi = span < 0 ? Wp - span : Wp;
    g.n_groups = (c_hi - g.c_lo + 63) / 64;
    g.n_chunks = (g.T + kLineTL - 1) / kLineTL;
    return g;
}

size_t line_aux_bytes(int dx, int dy, int64_t Hp, int64_t Wp, int order) {
    LineGeom g = line_geom(dx, dy, Hp, Wp);
    return (size_t)g.ay * g.n_chunks * g.n_groups * 64 * order * 8;
}

template <typename V, int ORDER, int SRC>
bsf_status pass_one(int dx, int dy, int64_t Hp, int64_t Wp, const Src &src, V *G, V *aux, const int32_t *status,
                    hipStream_t st) {
    if (dy == 0) {
        hipLaunchKernelGGL((k_row_scan<V, ORDER, SRC>), dim3((unsigned)Hp), dim3(kRowThreads), 0, st, G, Wp,
                           dx > 0 ? 1 : -1, src, status);
        BSF_HIP_CHECK(hipGetLastError());
        return BSF_OK;
    }
    LineGeom g = line_geom(dx, dy, Hp, Wp);
    const int64_t tiles = g.ay * g.n_chunks * g.n_groups;
    hipLaunchKernelGGL((k_line_aggregate<V, ORDER, SRC>), dim3((unsigned)tiles), dim3(64), 0, st, G, g, src, status,
                       aux);
    BSF_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL((k_line_carry<V, ORDER>), dim3((unsigned)(g.ay * g.n_groups)), dim3(64), 0, st, g, aux);
    BSF_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL((k_line_final<V, ORDER, SRC>), dim3((unsigned)tiles), dim3(64), 0, st, G, g, src, status,
                       aux);
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

template <typename V, int ORDER>
bsf_status pass_dispatch_src(int dx, int dy, int64_t Hp, int64_t Wp, const Src &src, V *G, V *aux,
                             const int32_t *status, hipStream_t st) {
    switch (src.kind) {
    case SRC_WINDOW: return pass_one<V, ORDER, SRC_WINDOW>(dx, dy, Hp, Wp, src, G, aux, status, st);
    case SRC_F32: return pass_one<V, ORDER, SRC_F32>(dx, dy, Hp, Wp, src, G, aux, status, st);
    case SRC_U8: return pass_one<V, ORDER, SRC_U8>(dx, dy, Hp, Wp, src, G, aux, status, st);
    case SRC_U16: return pass_one<V, ORDER, SRC_U16>(dx, dy, Hp, Wp, src, G, aux, status, st);
    }
    return BSF_E_INVALID;
}

template <typename V>
bsf_status pass_dispatch(int order, int dx, int dy, int64_t Hp, int64_t Wp, const Src &src, V *G, V *aux,
                         const int32_t *status, hipStream_t st) {
    switch (order) {
    case 1: return pass_dispatch_src<V, 1>(dx, dy, Hp, Wp, src, G, aux, status, st);
    case 2: return pass_dispatch_src<V, 2>(dx, dy, Hp, Wp, src, G, aux, status, st);
    case 3: return pass_dispatch_src<V, 3>(dx, dy, Hp, Wp, src, G, aux, status, st);
    case 4: return pass_dispatch_src<V, 4>(dx, dy, Hp, Wp, src, G, aux, status, st);
    }
    return BSF_E_UNSUPPORTED;
}

}  // namespace

size_t scan_aux_bytes(const Plan &p) {
    size_t m = 0;
    for (int k = 0; k < p.n_dirs; ++k) {
        if (p.dy[k] == 0) continue;
        size_t b = line_aux_bytes(p.dx[k], p.dy[k], p.Hp, p.Wp, p.order);
        if (b > m) m = b;
    }
    return align_up(m);
}

bsf_status run_preintegrate(const Plan &p, const Src &src, void *G, void *aux, const int32_t *status,
                            hipStream_t st) {
    Src s = src;
    for (int k = 0; k < p.n_dirs; ++k) {
        bsf_status r;
        if (p.arith == BSF_ARITH_FP64)
            r = pass_dispatch<double>(p.order, p.dx[k], p.dy[k], p.Hp, p.Wp, s, (double *)G, (double *)aux, status,
                                      st);
        else
            r = pass_dispatch<int64_t>(p.order, p.dx[k], p.dy[k], p.Hp, p.Wp, s, (int64_t *)G, (int64_t *)aux,
                                       status, st);
        if (r != BSF_OK) return r;
        s.kind = SRC_WINDOW;
    }
    return BSF_OK;
}

bsf_status run_preintegrate_transpose(const Plan &p, void *G, void *aux, hipStream_t st) {
    Src s{};
    s.kind = SRC_WINDOW;
    for (int k = p.n_dirs - 1; k >= 0; --k) {
        bsf_status r = pass_dispatch<int64_t>(p.order, -p.dx[k], -p.dy[k], p.Hp, p.Wp, s, (int64_t *)G,
                                              (int64_t *)aux, nullptr, st);
        if (r != BSF_OK) return r;
    }
    return BSF_OK;
}

}  // namespace bsf
