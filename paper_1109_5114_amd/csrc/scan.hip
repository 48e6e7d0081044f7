// Running sums on the window (Section 1.1, first step of BoxFilter; Alg. 3
// step 2: g(p) = f(p) + g(p - u)), r times per direction, in exact int64
// (wrapping modulo 2^64) or plain FP64.
//
// Rows (dy == 0) use one wavefront per row on a single image and one
// workgroup per row in a batch (1024-element chunks, a thread-local prefix over
// 4 contiguous elements, a wavefront prefix and a cross-wave prefix through
// LDS); the running carry stays in registers.  All other directions use
// sheared tiles: 64 lanes follow 64 adjacent lines of direction u for TL steps,
// so every step reads 64 contiguous elements of one row, 16 steps loaded
// together.  A tile's carry comes from the tile before it on the same lines,
// so the scan runs in three phases (tile aggregates, a per-line scan of
// aggregates, the final rescan), none of which waits on another workgroup: a
// direction has only about (W + H) / 64 groups of lines, so a look-back across
// the tiles of a line would chain one device-coherent round trip per tile.
//
// Every kernel runs either on one image (arguments by value) or on a batch
// (BATCH: a work list over images, each block looking up its image's job).
#include <type_traits>

#include "bsf_common.h"

namespace bsf {
namespace {

constexpr int kRowThreads = 256;
constexpr int kRowChunk = kRowThreads * 4;
constexpr int kUnroll = 16;  // steps of a line tile loaded together

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

// The job of this block and its local work item: a by-value job, or the
// batch's job table searched with the block index.
template <bool BATCH>
__device__ __forceinline__ bool job_of_block(const ScanJob &one, const ScanJob *__restrict__ jobs,
                                             const int64_t *__restrict__ prefix, int B, ScanJob &job,
                                             int64_t &item) {
    if constexpr (BATCH) {
        const int64_t gi = blockIdx.x;
        const int b = find_job(prefix, B, gi);
        job = jobs[b];
        item = gi - prefix[b];
        return item < prefix[b + 1] - prefix[b];
    } else {
        job = one;
        item = blockIdx.x;
        return true;
    }
}

template <typename V, int ORDER, int SRC, bool BATCH>
__global__ __launch_bounds__(kRowThreads) void k_row_scan(ScanJob one, const ScanJob *__restrict__ jobs,
                                                          const int64_t *__restrict__ prefix, int B) {
    __shared__ V lds[4];
    ScanJob job;
    int64_t row;
    if (!job_of_block<BATCH>(one, jobs, prefix, B, job, row)) return;
    V *__restrict__ G = static_cast<V *>(job.G);
    const int64_t Wp = job.Wp;
    const int dir = job.dir;
    const int F = (SRC == SRC_F32) ? job.status[ST_F_USED] : 0;
    V carry[ORDER];
#pragma unroll
    for (int o = 0; o < ORDER; ++o) carry[o] = V(0);
    for (int64_t c0 = 0; c0 < Wp; c0 += kRowChunk) {
        V v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t e = c0 + 4 * threadIdx.x + i;
            const int64_t col = dir > 0 ? e : Wp - 1 - e;
            v[i] = (e < Wp) ? load_src<V, SRC>(G, Wp, job.src, F, row, col) : V(0);
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

template <typename V, int ORDER, int SRC, bool BATCH>
__global__ __launch_bounds__(64) void k_line_aggregate(ScanJob one, const ScanJob *__restrict__ jobs,
                                                       const int64_t *__restrict__ prefix, int B) {
    ScanJob job;
    int64_t idx;
    if (!job_of_block<BATCH>(one, jobs, prefix, B, job, idx)) return;
    const LineGeom &g = job.g;
    const V *__restrict__ G = static_cast<const V *>(job.G);
    V *__restrict__ aux = static_cast<V *>(job.aux);
    const int lane = threadIdx.x;
    const int64_t gi = idx % g.n_groups, ch = (idx / g.n_groups) % g.n_chunks, q = idx / (g.n_groups * g.n_chunks);
    const int64_t c0 = g.c_lo + gi * 64 + lane;
    const int64_t t0 = ch * g.tl, t1 = min(g.T, t0 + g.tl);
    const int F = (SRC == SRC_F32) ? job.status[ST_F_USED] : 0;
    V s[ORDER];
#pragma unroll
    for (int o = 0; o < ORDER; ++o) s[o] = V(0);
    // kUnroll loads in flight per lane, then their sums
    for (int64_t tb = t0; tb < t1; tb += kUnroll) {
        V v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            int64_t row, col;
            bool in;
            line_cell(g, q, c0, tb + u, row, col, in);
            v[u] = (in && tb + u < t1) ? load_src<V, SRC>(G, g.Wp, job.src, F, row, col) : V(0);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (tb + u < t1) {
                s[0] += v[u];
#pragma unroll
                for (int o = 1; o < ORDER; ++o) s[o] += s[o - 1];
            }
        }
    }
#pragma unroll
    for (int o = 0; o < ORDER; ++o) aux[(idx * ORDER + o) * 64 + lane] = s[o];
}

template <typename V, int ORDER, bool BATCH>
__global__ __launch_bounds__(64) void k_line_carry(ScanJob one, const ScanJob *__restrict__ jobs,
                                                   const int64_t *__restrict__ prefix, int B) {
    ScanJob job;
    int64_t grp;
    if (!job_of_block<BATCH>(one, jobs, prefix, B, job, grp)) return;
    const LineGeom &g = job.g;
    V *__restrict__ aux = static_cast<V *>(job.aux);
    const int lane = threadIdx.x;
    const int64_t gi = grp % g.n_groups, q = grp / g.n_groups;
    V state[ORDER];
#pragma unroll
    for (int o = 0; o < ORDER; ++o) state[o] = V(0);
    for (int64_t ch = 0; ch < g.n_chunks; ++ch) {
        const int64_t idx = (q * g.n_chunks + ch) * g.n_groups + gi;
        const int64_t L = min(g.T, (ch + 1) * g.tl) - ch * g.tl;
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

template <typename V, int ORDER, int SRC, bool BATCH>
__global__ __launch_bounds__(64) void k_line_final(ScanJob one, const ScanJob *__restrict__ jobs,
                                                   const int64_t *__restrict__ prefix, int B) {
    ScanJob job;
    int64_t idx;
    if (!job_of_block<BATCH>(one, jobs, prefix, B, job, idx)) return;
    const LineGeom &g = job.g;
    V *__restrict__ G = static_cast<V *>(job.G);
    const V *__restrict__ aux = static_cast<const V *>(job.aux);
    const int lane = threadIdx.x;
    const int64_t gi = idx % g.n_groups, ch = (idx / g.n_groups) % g.n_chunks, q = idx / (g.n_groups * g.n_chunks);
    const int64_t c0 = g.c_lo + gi * 64 + lane;
    const int64_t t0 = ch * g.tl, t1 = min(g.T, t0 + g.tl);
    const int F = (SRC == SRC_F32) ? job.status[ST_F_USED] : 0;
    V s[ORDER];
#pragma unroll
    for (int o = 0; o < ORDER; ++o) s[o] = aux[(idx * ORDER + o) * 64 + lane];
    for (int64_t tb = t0; tb < t1; tb += kUnroll) {
        V v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            int64_t row, col;
            bool in;
            line_cell(g, q, c0, tb + u, row, col, in);
            v[u] = (in && tb + u < t1) ? load_src<V, SRC>(G, g.Wp, job.src, F, row, col) : V(0);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            int64_t row, col;
            bool in;
            line_cell(g, q, c0, tb + u, row, col, in);
            if (tb + u < t1) {
                s[0] += v[u];
#pragma unroll
                for (int o = 1; o < ORDER; ++o) s[o] += s[o - 1];
                if (in) G[row * g.Wp + col] = s[ORDER - 1];
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Single-image row passes: one wavefront per row, segments of 128 elements
// with lane l holding elements 2l and 2l + 1; per order level the pair is
// summed, a wavefront prefix of the pair sums gives each lane its offset, and
// the carry moves to the next segment in registers.  Four segments are
// scanned together (their prefixes do not depend on the carry) and the next
// four are loaded before they are.
// ----------------------------------------------------------------------------
template <typename V>
__device__ __forceinline__ V wave_incl_scan(V x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const V t = shfl_up64(x, d);
        if (lane >= d) x += t;
    }
    return x;
}

template <typename V, int ORDER, int SRC>
__global__ __launch_bounds__(256) void k_row_scan_wave(ScanJob job) {
    constexpr int kSeg = 4;  // segments per step: their wavefront prefixes are independent
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= job.Hp) return;  // the whole wavefront
    V *__restrict__ G = static_cast<V *>(job.G);
    const int64_t Wp = job.Wp;
    const int dir = job.dir;
    const int F = (SRC == SRC_F32) ? job.status[ST_F_USED] : 0;
    auto col_of = [&](int64_t e) { return dir > 0 ? e : Wp - 1 - e; };
    auto load_step = [&](int64_t step, V x[2 * kSeg]) {
#pragma unroll
        for (int k = 0; k < kSeg; ++k) {
            const int64_t e0 = (step * kSeg + k) * 128 + 2 * lane;
            x[2 * k] = e0 < Wp ? load_src<V, SRC>(G, Wp, job.src, F, row, col_of(e0)) : V(0);
            x[2 * k + 1] = e0 + 1 < Wp ? load_src<V, SRC>(G, Wp, job.src, F, row, col_of(e0 + 1)) : V(0);
        }
    };
    V carry[ORDER];
#pragma unroll
    for (int o = 0; o < ORDER; ++o) carry[o] = V(0);
    const int64_t nstep = (Wp + 128 * kSeg - 1) / (128 * kSeg);
    V a[2 * kSeg], b[2 * kSeg];
    load_step(0, a);
    for (int64_t step = 0; step < nstep; ++step) {
        if (step + 1 < nstep) load_step(step + 1, b);
#pragma unroll
        for (int o = 0; o < ORDER; ++o) {
            V incl[kSeg];
#pragma unroll
            for (int k = 0; k < kSeg; ++k) {
                a[2 * k + 1] += a[2 * k];
                incl[k] = wave_incl_scan<V>(a[2 * k + 1]);
            }
#pragma unroll
            for (int k = 0; k < kSeg; ++k) {
                const V add = incl[k] - a[2 * k + 1] + carry[o];
                a[2 * k] += add;
                a[2 * k + 1] += add;
                carry[o] += __shfl(incl[k], 63, 64);
            }
        }
#pragma unroll
        for (int k = 0; k < kSeg; ++k) {
            const int64_t e0 = (step * kSeg + k) * 128 + 2 * lane;
            if (e0 < Wp) G[row * Wp + col_of(e0)] = a[2 * k];
            if (e0 + 1 < Wp) G[row * Wp + col_of(e0 + 1)] = a[2 * k + 1];
        }
#pragma unroll
        for (int k = 0; k < 2 * kSeg; ++k) a[k] = b[k];
    }
}

template <typename V, int ORDER, int SRC>
bsf_status pass_single_sweep(int dx, int dy, const ScanJob &job, void *aux, hipStream_t st) {
    (void)dx;
    (void)aux;
    hipLaunchKernelGGL((k_row_scan_wave<V, ORDER, SRC>), dim3((unsigned)((job.Hp + 3) / 4)), dim3(256), 0, st, job);
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

template <typename V, int ORDER>
bsf_status sweep_dispatch_src(int src_kind, int dx, int dy, const ScanJob &job, void *aux, hipStream_t st) {
    switch (src_kind) {
    case SRC_WINDOW: return pass_single_sweep<V, ORDER, SRC_WINDOW>(dx, dy, job, aux, st);
    case SRC_F32: return pass_single_sweep<V, ORDER, SRC_F32>(dx, dy, job, aux, st);
    case SRC_U8: return pass_single_sweep<V, ORDER, SRC_U8>(dx, dy, job, aux, st);
    case SRC_U16: return pass_single_sweep<V, ORDER, SRC_U16>(dx, dy, job, aux, st);
    }
    return BSF_E_INVALID;
}

template <typename V>
bsf_status sweep_dispatch(int order, int src_kind, int dx, int dy, const ScanJob &job, void *aux, hipStream_t st) {
    switch (order) {
    case 1: return sweep_dispatch_src<V, 1>(src_kind, dx, dy, job, aux, st);
    case 2: return sweep_dispatch_src<V, 2>(src_kind, dx, dy, job, aux, st);
    case 3: return sweep_dispatch_src<V, 3>(src_kind, dx, dy, job, aux, st);
    case 4: return sweep_dispatch_src<V, 4>(src_kind, dx, dy, job, aux, st);
    }
    return BSF_E_UNSUPPORTED;
}

// Launch one pass: a by-value job (jobs == nullptr) or a batch.
template <typename V, int ORDER, int SRC>
bsf_status pass_one(int dy, const ScanJob &one, const ScanJob *jobs, const int64_t *prefix_items,
                    int64_t total_items, const int64_t *prefix_groups, int64_t total_groups, int B,
                    hipStream_t st) {
    const bool batch = jobs != nullptr;
    if (total_items <= 0) return BSF_OK;
    if (dy == 0) {
        if (batch)
            hipLaunchKernelGGL((k_row_scan<V, ORDER, SRC, true>), dim3((unsigned)total_items), dim3(kRowThreads), 0,
                               st, one, jobs, prefix_items, B);
        else
            hipLaunchKernelGGL((k_row_scan<V, ORDER, SRC, false>), dim3((unsigned)total_items), dim3(kRowThreads),
                               0, st, one, jobs, prefix_items, B);
        BSF_HIP_CHECK(hipGetLastError());
        return BSF_OK;
    }
    if (batch) {
        hipLaunchKernelGGL((k_line_aggregate<V, ORDER, SRC, true>), dim3((unsigned)total_items), dim3(64), 0, st,
                           one, jobs, prefix_items, B);
        hipLaunchKernelGGL((k_line_carry<V, ORDER, true>), dim3((unsigned)total_groups), dim3(64), 0, st, one, jobs,
                           prefix_groups, B);
        hipLaunchKernelGGL((k_line_final<V, ORDER, SRC, true>), dim3((unsigned)total_items), dim3(64), 0, st, one,
                           jobs, prefix_items, B);
    } else {
        hipLaunchKernelGGL((k_line_aggregate<V, ORDER, SRC, false>), dim3((unsigned)total_items), dim3(64), 0, st,
                           one, jobs, prefix_items, B);
        hipLaunchKernelGGL((k_line_carry<V, ORDER, false>), dim3((unsigned)total_groups), dim3(64), 0, st, one,
                           jobs, prefix_groups, B);
        hipLaunchKernelGGL((k_line_final<V, ORDER, SRC, false>), dim3((unsigned)total_items), dim3(64), 0, st, one,
                           jobs, prefix_items, B);
    }
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

template <typename V, int ORDER>
bsf_status pass_dispatch_src(int src_kind, int dy, const ScanJob &one, const ScanJob *jobs, const int64_t *pi,
                             int64_t ti, const int64_t *pg, int64_t tg, int B, hipStream_t st) {
    switch (src_kind) {
    case SRC_WINDOW: return pass_one<V, ORDER, SRC_WINDOW>(dy, one, jobs, pi, ti, pg, tg, B, st);
    case SRC_F32: return pass_one<V, ORDER, SRC_F32>(dy, one, jobs, pi, ti, pg, tg, B, st);
    case SRC_U8: return pass_one<V, ORDER, SRC_U8>(dy, one, jobs, pi, ti, pg, tg, B, st);
    case SRC_U16: return pass_one<V, ORDER, SRC_U16>(dy, one, jobs, pi, ti, pg, tg, B, st);
    }
    return BSF_E_INVALID;
}

template <typename V>
bsf_status pass_dispatch(int order, int src_kind, int dy, const ScanJob &one, const ScanJob *jobs, const int64_t *pi,
                         int64_t ti, const int64_t *pg, int64_t tg, int B, hipStream_t st) {
    switch (order) {
    case 1: return pass_dispatch_src<V, 1>(src_kind, dy, one, jobs, pi, ti, pg, tg, B, st);
    case 2: return pass_dispatch_src<V, 2>(src_kind, dy, one, jobs, pi, ti, pg, tg, B, st);
    case 3: return pass_dispatch_src<V, 3>(src_kind, dy, one, jobs, pi, ti, pg, tg, B, st);
    case 4: return pass_dispatch_src<V, 4>(src_kind, dy, one, jobs, pi, ti, pg, tg, B, st);
    }
    return BSF_E_UNSUPPORTED;
}

size_t line_aux_bytes(int dx, int dy, int64_t Hp, int64_t Wp, int order) {
    LineGeom g = line_geom(dx, dy, Hp, Wp, tuning().line_tl);
    return (size_t)g.ay * g.n_chunks * g.n_groups * 64 * order * 8;
}

// One pass of one image through the single-image kernels.
bsf_status pass_single(int arith, int order, int dx, int dy, int64_t Hp, int64_t Wp, const Src &src, void *G,
                       void *aux, const int32_t *status, hipStream_t st) {
    ScanJob job{};
    job.G = G;
    job.aux = aux;
    job.status = status;
    job.src = src;
    job.Hp = Hp;
    job.Wp = Wp;
    job.dir = dx > 0 ? 1 : -1;
    if (dy == 0) {
        if (arith == BSF_ARITH_FP64) return sweep_dispatch<double>(order, src.kind, dx, dy, job, aux, st);
        return sweep_dispatch<int64_t>(order, src.kind, dx, dy, job, aux, st);
    }
    job.g = line_geom(dx, dy, Hp, Wp, tuning().line_tl);
    const int64_t items = job.g.ay * job.g.n_chunks * job.g.n_groups, groups = job.g.ay * job.g.n_groups;
    if (arith == BSF_ARITH_FP64)
        return pass_dispatch<double>(order, src.kind, dy, job, nullptr, nullptr, items, nullptr, groups, 1, st);
    return pass_dispatch<int64_t>(order, src.kind, dy, job, nullptr, nullptr, items, nullptr, groups, 1, st);
}

}  // namespace

LineGeom line_geom(int dx, int dy, int64_t Hp, int64_t Wp, int tl) {
    LineGeom g;
    g.dx = dx;
    g.dy = dy;
    g.ay = dy > 0 ? dy : -dy;
    g.tl = tl;
    g.Hp = Hp;
    g.Wp = Wp;
    g.T = (Hp + g.ay - 1) / g.ay;
    const int64_t span = (int64_t)dx * (g.T - 1);
    g.c_lo = span > 0 ? -span : 0;
    const int64_t c_hi = span < 0 ? Wp - span : Wp;
    g.n_groups = (c_hi - g.c_lo + 63) / 64;
    g.n_chunks = (g.T + tl - 1) / tl;
    return g;
}

size_t scan_aux_bytes(const Plan &p) {
    // the column pass of run_prefix2d over at most the window's size
    size_t m = line_aux_bytes(0, 1, p.Hp, p.Wp, 1);
    for (int k = 0; k < p.n_dirs; ++k) {
        // both the forward pass (dx, dy) and the transposed one (-dx, -dy)
        if (p.dy[k] == 0) continue;
        size_t b = line_aux_bytes(p.dx[k], p.dy[k], p.Hp, p.Wp, p.order);
        size_t bt = line_aux_bytes(-p.dx[k], -p.dy[k], p.Hp, p.Wp, p.order);
        if (b > m) m = b;
        if (bt > m) m = bt;
    }
    return align_up(m);
}

bsf_status run_preintegrate(const Plan &p, const Src &src, void *G, void *aux, const int32_t *status,
                            hipStream_t st) {
    Src s = src;
    for (int k = 0; k < p.n_dirs; ++k) {
        bsf_status r = pass_single(p.arith, p.order, p.dx[k], p.dy[k], p.Hp, p.Wp, s, G, aux, status, st);
        if (r != BSF_OK) return r;
        s.kind = SRC_WINDOW;
    }
    return BSF_OK;
}

bsf_status run_preintegrate_transpose(const Plan &p, void *G, void *aux, const int32_t *status, hipStream_t st) {
    Src s{};
    s.kind = SRC_WINDOW;
    for (int k = p.n_dirs - 1; k >= 0; --k) {
        bsf_status r =
            pass_single(BSF_ARITH_EXACT, p.order, -p.dx[k], -p.dy[k], p.Hp, p.Wp, s, G, aux, status, st);
        if (r != BSF_OK) return r;
    }
    return BSF_OK;
}

bsf_status run_prefix2d(int64_t *D, int64_t rows, int64_t cols, void *aux, const int32_t *status, hipStream_t st) {
    Src s{};
    s.kind = SRC_WINDOW;
    bsf_status r = pass_single(BSF_ARITH_EXACT, 1, 1, 0, rows, cols, s, D, aux, status, st);
    if (r != BSF_OK) return r;
    return pass_single(BSF_ARITH_EXACT, 1, 0, 1, rows, cols, s, D, aux, status, st);
}

bsf_status run_pass_batch(int arith, int order, int src_kind, int dx, int dy, const ScanJob *jobs,
                          const int64_t *prefix_items, int64_t total_items, const int64_t *prefix_groups,
                          int64_t total_groups, int B, hipStream_t st) {
    (void)dx;
    ScanJob none{};
    if (arith == BSF_ARITH_FP64)
        return pass_dispatch<double>(order, src_kind, dy, none, jobs, prefix_items, total_items, prefix_groups,
                                     total_groups, B, st);
    return pass_dispatch<int64_t>(order, src_kind, dy, none, jobs, prefix_items, total_items, prefix_groups,
                                  total_groups, B, st);
}

}  // namespace bsf
