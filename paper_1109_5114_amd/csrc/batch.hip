// Batched forward over images of uneven sizes: the filter of Section 1.1
// (BoxFilter's two steps, Alg. 3) applied to every image of a batch, with each
// stage of the path one launch over the whole batch.
//
// The launch tables (one record per image for the bound check, each running-sum
// pass and the gather, and prefix sums of the per-image work counts) are built
// on the host and copied into the workspace by small kernels that carry the
// bytes in their arguments, so the whole call is stream-ordered kernel work and
// can be recorded into a HIP graph as it stands.  Each image keeps the
// single-image workspace layout (status block, window, scan carries), so a
// batch gives exactly the results of one call per image.
#include <string.h>

#include <list>
#include <mutex>
#include <vector>

#include "bsf_common.h"

namespace bsf {
namespace {

constexpr int kMaxBatch = 65536;
constexpr int kUploadWords = 256;  // 2 KiB of table per upload launch
constexpr size_t kGraphCacheSize = 16;

struct UploadChunk {
    uint64_t w[kUploadWords];
};

__global__ __launch_bounds__(kUploadWords) void k_upload(uint64_t *dst, int n, UploadChunk c) {
    const int i = threadIdx.x;
    if (i < n) dst[i] = c.w[i];
}

// Every image's status block starts each call cleared.
__global__ void k_batch_begin(int32_t *const *__restrict__ status) {
    if (threadIdx.x < ST_WORDS) status[blockIdx.x][threadIdx.x] = 0;
}

// Batch status: flags OR-ed (sticky), the smallest F and the largest bound.
__global__ __launch_bounds__(256) void k_batch_end(int32_t *const *__restrict__ status, int B,
                                                   int32_t *__restrict__ batch) {
    __shared__ int s_flags[4], s_F[4], s_bound[4];
    int flags = 0, F = 1 << 30, bound = -(1 << 30);
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        const int32_t *s = status[b];
        flags |= s[ST_FLAGS];
        F = min(F, s[ST_F_USED]);
        bound = max(bound, s[ST_LOG2_BOUND]);
    }
    for (int d = 32; d >= 1; d >>= 1) {
        flags |= __shfl_xor(flags, d, 64);
        F = min(F, __shfl_xor(F, d, 64));
        bound = max(bound, __shfl_xor(bound, d, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_flags[w] = flags;
        s_F[w] = F;
        s_bound[w] = bound;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            flags |= s_flags[k];
            F = min(F, s_F[k]);
            bound = max(bound, s_bound[k]);
        }
        batch[ST_FLAGS] |= flags;
        batch[ST_F_USED] = B > 0 ? F : 0;
        batch[ST_LOG2_BOUND] = B > 0 ? bound : 0;
    }
}

size_t align16(size_t v) { return (v + 15) / 16 * 16; }

// Everything a batched call needs, derived on the host from (cfg, descs, ws).
struct BatchPlan {
    int B = 0;
    std::vector<Plan> plans;
    std::vector<size_t> image_off;  // workspace offset of each image's region
    // byte offsets inside the table region
    size_t t_status, t_bound, t_prefix_rows, t_gather, t_prefix_tiles;
    size_t t_scan[BSF_MAX_DIRS], t_prefix_items[BSF_MAX_DIRS], t_prefix_groups[BSF_MAX_DIRS];
    size_t tables_bytes = 0;
    size_t total_bytes = 0;
    int first = -1;  // first non-empty image
};

bool nonempty(const bsf_image_desc &d) { return d.H > 0 && d.W > 0; }

bsf_status plan_batch(const bsf_config *cfg, int32_t B, const bsf_image_desc *descs, BatchPlan &bp) {
    if (!cfg || B < 0 || B > kMaxBatch || (B > 0 && !descs)) return BSF_E_INVALID;
    bp.B = B;
    bp.plans.resize(B);
    bp.image_off.resize(B);
    for (int b = 0; b < B; ++b) {
        const bsf_image_desc &d = descs[b];
        bsf_status r = make_plan(cfg, d.H, d.W, &bp.plans[b]);
        if (r != BSF_OK) return r;
        if (nonempty(d)) {
            if (!d.img || !d.steps || !d.out || d.pitch < d.W) return BSF_E_INVALID;
            if (bp.first < 0) bp.first = b;
        }
    }
    if (bp.plans.empty()) {
        Plan p;
        bsf_status r = make_plan(cfg, 0, 0, &p);
        if (r != BSF_OK) return r;
    }
    const int n_dirs = cfg->n_dirs;
    const size_t pre = (size_t)(B + 1) * sizeof(int64_t);
    size_t t = 0;
    bp.t_status = t;
    t = align16(t + (size_t)B * sizeof(int32_t *));
    bp.t_bound = t;
    t = align16(t + (size_t)B * bound_job_bytes());
    bp.t_prefix_rows = t;
    t = align16(t + pre);
    for (int k = 0; k < n_dirs; ++k) {
        bp.t_scan[k] = t;
        t = align16(t + (size_t)B * sizeof(ScanJob));
        bp.t_prefix_items[k] = t;
        t = align16(t + pre);
        bp.t_prefix_groups[k] = t;
        t = align16(t + pre);
    }
    bp.t_gather = t;
    t = align16(t + (size_t)B * sizeof(GatherArgs));
    bp.t_prefix_tiles = t;
    t = align16(t + pre);
    bp.tables_bytes = align_up(t);
    size_t off = kStatusBytes + bp.tables_bytes;
    for (int b = 0; b < B; ++b) {
        bp.image_off[b] = off;
        off += align_up(ws_bytes_for(bp.plans[b], true));
    }
    bp.total_bytes = off;
    return BSF_OK;
}

// Host image of the table region, and the totals of each work list.
struct Tables {
    std::vector<uint64_t> host;
    int64_t rows = 0, tiles = 0;
    int64_t items[BSF_MAX_DIRS] = {}, groups[BSF_MAX_DIRS] = {};
    bool uniform_gather = true;
};

template <typename T>
void put(std::vector<uint64_t> &h, size_t off, size_t idx, const T &v) {
    memcpy(reinterpret_cast<char *>(h.data()) + off + idx * sizeof(T), &v, sizeof(T));
}

void build_tables(const bsf_config *cfg, const bsf_image_desc *descs, const BatchPlan &bp, char *ws, Tables &tb) {
    const int B = bp.B;
    tb.host.assign(bp.tables_bytes / 8, 0);
    std::vector<uint64_t> &h = tb.host;
    const int tl = tuning().line_tl;
    std::vector<char> job(bound_job_bytes());
    int variant0 = -1;
    put<int64_t>(h, bp.t_prefix_rows, 0, 0);
    put<int64_t>(h, bp.t_prefix_tiles, 0, 0);
    for (int k = 0; k < cfg->n_dirs; ++k) {
        put<int64_t>(h, bp.t_prefix_items[k], 0, 0);
        put<int64_t>(h, bp.t_prefix_groups[k], 0, 0);
    }
    for (int b = 0; b < B; ++b) {
        const bsf_image_desc &d = descs[b];
        const Plan &p = bp.plans[b];
        const bool live = nonempty(d);
        char *region = ws + bp.image_off[b];
        int32_t *status = reinterpret_cast<int32_t *>(region);
        void *G = region + kStatusBytes;
        void *aux = region + kStatusBytes + align_up(p.g_bytes);
        put<int32_t *>(h, bp.t_status, b, status);
        make_bound_job(d.steps, d.img, live ? d.H : 0, live ? d.W : 0, d.pitch, status, job.data());
        memcpy(reinterpret_cast<char *>(h.data()) + bp.t_bound + (size_t)b * job.size(), job.data(), job.size());
        tb.rows += live ? d.H : 0;
        put<int64_t>(h, bp.t_prefix_rows, b + 1, tb.rows);
        for (int k = 0; k < cfg->n_dirs; ++k) {
            ScanJob j;
            memset(&j, 0, sizeof(j));
            j.G = G;
            j.aux = aux;
            j.status = status;
            j.src = Src{d.img, k == 0 ? SRC_F32 : SRC_WINDOW, d.H, d.W, d.pitch, p.pad_top, p.pad_left};
            j.Hp = p.Hp;
            j.Wp = p.Wp;
            j.dir = p.dx[k] > 0 ? 1 : -1;
            int64_t items = 0, groups = 0;
            if (live) {
                if (p.dy[k] == 0) {
                    items = p.Hp;
                } else {
                    j.g = line_geom(p.dx[k], p.dy[k], p.Hp, p.Wp, tl);
                    items = j.g.ay * j.g.n_chunks * j.g.n_groups;
                    groups = j.g.ay * j.g.n_groups;
                }
            }
            put<ScanJob>(h, bp.t_scan[k], b, j);
            tb.items[k] += items;
            tb.groups[k] += groups;
            put<int64_t>(h, bp.t_prefix_items[k], b + 1, tb.items[k]);
            put<int64_t>(h, bp.t_prefix_groups[k], b + 1, tb.groups[k]);
        }
        GatherArgs a = gather_args(p, G, d.steps, d.out, nullptr, nullptr, nullptr, status);
        if (a.canon == 2) a.canon = 0;  // no batched cluster-box kernel in the frame of Table 1
        put<GatherArgs>(h, bp.t_gather, b, a);
        if (live) {
            tb.tiles += gather_tiles(p, a);
            const int v = gather_variant(p, a);
            if (variant0 < 0) variant0 = v;
            else if (v != variant0) tb.uniform_gather = false;
        }
        put<int64_t>(h, bp.t_prefix_tiles, b + 1, tb.tiles);
    }
}

bsf_status upload(const std::vector<uint64_t> &h, void *dst, hipStream_t st) {
    uint64_t *d = static_cast<uint64_t *>(dst);
    UploadChunk c;
    for (size_t i = 0; i < h.size(); i += kUploadWords) {
        const int n = (int)((h.size() - i) < (size_t)kUploadWords ? (h.size() - i) : (size_t)kUploadWords);
        memset(&c, 0, sizeof(c));
        memcpy(c.w, h.data() + i, n * sizeof(uint64_t));
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(kUploadWords), 0, st, d + i, n, c);
        BSF_HIP_CHECK(hipGetLastError());
    }
    return BSF_OK;
}

bool fits_grid(int64_t n) { return n < (int64_t(1) << 31); }

// Enqueue the whole batched forward on st.
bsf_status enqueue(const bsf_config *cfg, const bsf_image_desc *descs, const BatchPlan &bp, void *ws,
                   hipStream_t st) {
    const int B = bp.B;
    char *wsb = static_cast<char *>(ws);
    if (B == 0) return BSF_OK;
    Tables tb;
    build_tables(cfg, descs, bp, wsb, tb);
    if (!fits_grid(tb.rows) || !fits_grid(tb.tiles)) return BSF_E_UNSUPPORTED;
    for (int k = 0; k < cfg->n_dirs; ++k)
        if (!fits_grid(tb.items[k]) || !fits_grid(tb.groups[k])) return BSF_E_UNSUPPORTED;
    char *tab = wsb + kStatusBytes;
    bsf_status r = upload(tb.host, tab, st);
    if (r != BSF_OK) return r;
    int32_t *const *status_tab = reinterpret_cast<int32_t *const *>(tab + bp.t_status);
    hipLaunchKernelGGL(k_batch_begin, dim3((unsigned)B), dim3(64), 0, st, status_tab);
    BSF_HIP_CHECK(hipGetLastError());
    if (bp.first >= 0) {
        const Plan &p0 = bp.plans[bp.first];
        r = run_bound_batch(p0, SRC_F32, cfg->frac_bits, tab + bp.t_bound,
                            reinterpret_cast<const int64_t *>(tab + bp.t_prefix_rows), B, tb.rows, st);
        if (r != BSF_OK) return r;
        for (int k = 0; k < cfg->n_dirs; ++k) {
            r = run_pass_batch(p0.arith, p0.order, k == 0 ? SRC_F32 : SRC_WINDOW, p0.dx[k], p0.dy[k],
                               reinterpret_cast<const ScanJob *>(tab + bp.t_scan[k]),
                               reinterpret_cast<const int64_t *>(tab + bp.t_prefix_items[k]), tb.items[k],
                               reinterpret_cast<const int64_t *>(tab + bp.t_prefix_groups[k]), tb.groups[k], B, st);
            if (r != BSF_OK) return r;
        }
        if (tb.uniform_gather) {
            const bsf_image_desc &d0 = descs[bp.first];
            char *region = wsb + bp.image_off[bp.first];
            const GatherArgs a0 = gather_args(p0, region + kStatusBytes, d0.steps, d0.out, nullptr, nullptr, nullptr,
                                              reinterpret_cast<int32_t *>(region));
            r = run_gather_batch(p0, a0, reinterpret_cast<const GatherArgs *>(tab + bp.t_gather),
                                 reinterpret_cast<const int64_t *>(tab + bp.t_prefix_tiles), B, tb.tiles, st);
            if (r != BSF_OK) return r;
        } else {
            // images whose windows need different gather kernels: one launch each
            for (int b = 0; b < B; ++b) {
                if (!nonempty(descs[b])) continue;
                char *region = wsb + bp.image_off[b];
                const GatherArgs a = gather_args(bp.plans[b], region + kStatusBytes, descs[b].steps, descs[b].out,
                                                 nullptr, nullptr, nullptr, reinterpret_cast<int32_t *>(region));
                r = run_gather(bp.plans[b], a, st);
                if (r != BSF_OK) return r;
            }
        }
    }
    hipLaunchKernelGGL(k_batch_end, dim3(1), dim3(256), 0, st, status_tab, B, reinterpret_cast<int32_t *>(wsb));
    BSF_HIP_CHECK(hipGetLastError());
    return BSF_OK;
}

// ----------------------------------------------------------------------------
// Graph cache: one executable graph per (device, cfg, descs, ws, ws_bytes,
// tuning).  Kernel arguments, including the uploaded tables, are fixed at
// capture, so a key match replays exactly the same work.
// ----------------------------------------------------------------------------
struct GraphEntry {
    std::vector<char> key;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

std::mutex g_graph_mu;
std::list<GraphEntry> g_graphs;

std::vector<char> graph_key(const bsf_config *cfg, int32_t B, const bsf_image_desc *descs, void *ws,
                            size_t ws_bytes) {
    int dev = -1;
    (void)hipGetDevice(&dev);
    const Tuning t = tuning();
    std::vector<char> k(sizeof(int) + sizeof(bsf_config) + sizeof(int32_t) + (size_t)B * sizeof(bsf_image_desc) +
                        sizeof(void *) + sizeof(size_t) + sizeof(Tuning));
    char *p = k.data();
    auto add = [&p](const void *src, size_t n) {
        memcpy(p, src, n);
        p += n;
    };
    add(&dev, sizeof(dev));
    add(cfg, sizeof(bsf_config));
    add(&B, sizeof(B));
    if (B > 0) add(descs, (size_t)B * sizeof(bsf_image_desc));
    add(&ws, sizeof(ws));
    add(&ws_bytes, sizeof(ws_bytes));
    add(&t, sizeof(t));
    return k;
}

bsf_status run_graph(const bsf_config *cfg, int32_t B, const bsf_image_desc *descs, const BatchPlan *bp, void *ws,
                     size_t ws_bytes, hipStream_t st, bool *hit) {
    std::vector<char> key = graph_key(cfg, B, descs, ws, ws_bytes);
    std::lock_guard<std::mutex> lock(g_graph_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it) {
        if (it->key == key) {
            g_graphs.splice(g_graphs.begin(), g_graphs, it);
            *hit = true;
            BSF_HIP_CHECK(hipGraphLaunch(g_graphs.front().exec, st));
            return BSF_OK;
        }
    }
    *hit = false;
    if (!bp) return BSF_OK;  // caller plans, then calls again with the plan
    BSF_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    bsf_status r = enqueue(cfg, descs, *bp, ws, st);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (r != BSF_OK || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return r != BSF_OK ? r : BSF_E_DEVICE;
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return BSF_E_DEVICE;
    }
    if (g_graphs.size() >= kGraphCacheSize) {
        // a replay of the evicted graph may still be running
        BSF_HIP_CHECK(hipDeviceSynchronize());
        GraphEntry &old = g_graphs.back();
        (void)hipGraphExecDestroy(old.exec);
        (void)hipGraphDestroy(old.graph);
        g_graphs.pop_back();
    }
    g_graphs.push_front(GraphEntry{std::move(key), graph, exec});
    BSF_HIP_CHECK(hipGraphLaunch(exec, st));
    return BSF_OK;
}

}  // namespace
}  // namespace bsf

using namespace bsf;

extern "C" {

size_t bsf_batched_workspace_bytes(const bsf_config *cfg, int32_t B, const bsf_image_desc *descs) {
    BatchPlan bp;
    if (plan_batch(cfg, B, descs, bp) != BSF_OK) return 0;
    return bp.total_bytes;
}

bsf_status bsf_filter_batched(const bsf_config *cfg, int32_t B, const bsf_image_desc *descs, void *ws,
                              size_t ws_bytes, void *stream, int32_t use_graph) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    bool graph = use_graph != 0 && st != nullptr;
    if (graph) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        BSF_HIP_CHECK(hipStreamIsCapturing(st, &cs));
        if (cs != hipStreamCaptureStatusNone) graph = false;  // part of the caller's own capture
    }
    if (!ws) return BSF_E_INVALID;
    if (graph && cfg && B >= 0 && B <= kMaxBatch && (B == 0 || descs)) {
        // a cached graph was captured from a call that passed every check below
        bool hit = false;
        bsf_status r = run_graph(cfg, B, descs, nullptr, ws, ws_bytes, st, &hit);
        if (r != BSF_OK || hit) return r;
    }
    BatchPlan bp;
    bsf_status r = plan_batch(cfg, B, descs, bp);
    if (r != BSF_OK) return r;
    if (ws_bytes < bp.total_bytes) return BSF_E_WORKSPACE;
    if (graph) {
        bool hit = false;
        return run_graph(cfg, B, descs, &bp, ws, ws_bytes, st, &hit);
    }
    return enqueue(cfg, descs, bp, ws, st);
}

}  // extern "C"
