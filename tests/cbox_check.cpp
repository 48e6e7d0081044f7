// Host check of the cluster-box index functions (paper_1109_5114_amd/csrc/
// cluster_box.h) used by the tied order-2 gather and adjoint kernels.
//
// For random tiles, per-pixel step ranges and window geometries it checks that
//   - the nine taps of each direction's squared difference operator
//     D^2 = ((1 - phi)(T_R - T_{-R-1}) + phi (T_{R+1} - T_{-R-2}))^2 are exactly
//     the three clusters base_of(c, R) + {0, 1, 2};
//   - whenever boxes_fit() accepts a tile, every combination's box starts on an
//     even window column, fits the LDS box (64 columns, the given rows), lies in
//     the window with the spare column its pair copies may touch, and holds
//     every sub-tap of every pixel of the tile at the element its LDS offset
//     (pixel_base, and packed_base from the packed state) points to: the box
//     element is the window element of that tap;
//   - the packed state keeps the tile position and R_k - Rlo_k exactly.
// Both direction frames are checked (frame 0: (1,0), (0,1), (1,1), (1,-1);
// frame 1: (2,1), (1,2), (1,-2), (2,-1)).
// Input (stdin): lines "frame H W R_max pad_top pad_left win_h win_w tile_w
// tile_h rows cases seed"; prints "ok <fitting tiles> <taps checked>" or the first
// failure, and exits non-zero on failure.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <utility>

#include "../paper_1109_5114_amd/csrc/cluster_box.h"

using namespace bsf;

namespace {

struct Geom {
    long H, W;
    int R_max;
    long pad_top, pad_left, win_h, win_w;
    int tile_w, tile_h, rows;
};

long g_taps = 0;

bool fail(const char *what, long a, long b) {
    std::printf("FAIL %s (%ld vs %ld)\n", what, a, b);
    return false;
}

const int kU[2][4][2] = {{{1, 0}, {0, 1}, {1, 1}, {1, -1}}, {{2, 1}, {1, 2}, {1, -2}, {2, -1}}};

bool check_clusters(int R) {
    std::multiset<int> d2, cl;
    const int ends[4] = {R, -R - 1, R + 1, -R - 2};
    // D^2 reads the sums of one end of each D factor: narrow-narrow, ...
    const int pairs[][2] = {{0, 0}, {0, 1}, {1, 0}, {1, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3},
                            {2, 0}, {2, 1}, {3, 0}, {3, 1}, {2, 2}, {2, 3}, {3, 2}, {3, 3}};
    for (auto &p : pairs) d2.insert(ends[p[0]] + ends[p[1]]);
    std::set<int> want(d2.begin(), d2.end());
    std::set<int> got;
    for (int c = 0; c < 3; ++c)
        for (int q = 0; q < 3; ++q) got.insert(cbox::base_of(c, R) + q);
    if (want != got) return fail("clusters of D^2", (long)want.size(), (long)got.size());
    return true;
}

template <int D, int C>
bool check_combo(const Geom &g, int x_lo, int x_hi, int y_lo, int y_hi, const int Rlo[4], const int Rhi[4],
                 const int (*R)[4], const bool *active) {
    const cbox::Box b = cbox::box_of<C, D>(x_lo, x_hi, y_lo, y_hi, Rlo, Rhi, (int)g.pad_left);
    if ((b.ox + g.pad_left) % 2 != 0) return fail("box start column parity", b.ox + g.pad_left, 0);
    if (b.bw > cbox::kPitch) return fail("box width", b.bw, cbox::kPitch);
    if (b.bh > g.rows) return fail("box rows", b.bh, g.rows);
    if (b.ox + g.pad_left < 0 || b.oy + g.pad_top < 0) return fail("box before the window", b.ox, b.oy);
    if (b.ox + g.pad_left + ((b.bw + 1) / 2) * 2 > g.win_w) return fail("box pairs past the window", b.ox, b.bw);
    if (b.oy + g.pad_top + b.bh > g.win_h) return fail("box below the window", b.oy, b.bh);
    for (int ty = 0; ty <= y_hi - y_lo; ++ty)
        for (int tx = 0; tx <= x_hi - x_lo; ++tx) {
            const int i = ty * g.tile_w + tx;
            if (!active[i]) continue;
            const int x = x_lo + tx, y = y_lo + ty;
            const uint32_t st = cbox::pack_state(tx, ty, R[i], Rlo, true);
            if ((int)(st & 1023u) != tx + cbox::kPitch * ty) return fail("packed position", st & 1023u, tx);
            for (int k = 0; k < 4; ++k)
                if ((int)((st >> (10 + 5 * k)) & 31u) != R[i][k] - Rlo[k])
                    return fail("packed R", (st >> (10 + 5 * k)) & 31u, R[i][k] - Rlo[k]);
            const int base = cbox::pixel_base<C, D>(x, y, R[i], b);
            const int pbase = cbox::packed_base<C, D>(st, x_lo, y_lo, Rlo, b);
            if (base != pbase) return fail("packed_base", pbase, base);
            for (int q = 0; q < 81; ++q) {
                const int q0 = q % 3, q1 = (q / 3) % 3, q2 = (q / 9) % 3, q3 = q / 27;
                const int e = base + cbox::sub_elem<D>(q0, q1, q2, q3);
                if (e < 0) return fail("negative LDS element", e, 0);
                const int row = e / cbox::kPitch, col = e % cbox::kPitch;
                if (row >= b.bh || col >= b.bw) return fail("tap outside its box", row, col);
                const int qs[4] = {q0, q1, q2, q3};
                long tx_img = x, ty_img = y;
                for (int k = 0; k < 4; ++k) {
                    const int m = cbox::base_of(cbox::cl(C, k), R[i][k]) + qs[k];
                    tx_img += (long)m * kU[D][k][0];
                    ty_img += (long)m * kU[D][k][1];
                }
                if (b.ox + col != tx_img || b.oy + row != ty_img) return fail("box element is not the tap", tx_img, ty_img);
                ++g_taps;
            }
        }
    return true;
}

template <int D, int... Cs>
bool check_all(std::integer_sequence<int, Cs...>, const Geom &g, int x_lo, int x_hi, int y_lo, int y_hi,
               const int Rlo[4], const int Rhi[4], const int (*R)[4], const bool *active) {
    return (check_combo<D, Cs>(g, x_lo, x_hi, y_lo, y_hi, Rlo, Rhi, R, active) && ...);
}

}  // namespace

int main() {
    Geom g;
    int cases;
    unsigned seed;
    long fitting = 0;
    for (int R = 0; R < 200; ++R)
        if (!check_clusters(R)) return 1;
    int frame;
    while (std::scanf("%d %ld %ld %d %ld %ld %ld %ld %d %d %d %d %u", &frame, &g.H, &g.W, &g.R_max, &g.pad_top,
                      &g.pad_left, &g.win_h, &g.win_w, &g.tile_w, &g.tile_h, &g.rows, &cases, &seed) == 13) {
        if (frame != 0 && frame != 1) return fail("frame", frame, 0), 1;
        std::mt19937 rng(seed);
        const long tiles_x = (g.W + g.tile_w - 1) / g.tile_w, tiles_y = (g.H + g.tile_h - 1) / g.tile_h;
        static int R[256][4];
        static bool active[256];
        for (int n = 0; n < cases; ++n) {
            // corner and edge tiles often, interior ones otherwise
            long bx = rng() % tiles_x, by = rng() % tiles_y;
            if (rng() % 4 == 0) bx = (rng() % 2) ? 0 : tiles_x - 1;
            if (rng() % 4 == 0) by = (rng() % 2) ? 0 : tiles_y - 1;
            const int x_lo = (int)(bx * g.tile_w), y_lo = (int)(by * g.tile_h);
            const int x_hi = (int)std::min<long>(x_lo + g.tile_w - 1, g.W - 1);
            const int y_hi = (int)std::min<long>(y_lo + g.tile_h - 1, g.H - 1);
            int Rlo[4], Rhi[4];
            for (int k = 0; k < 4; ++k) {
                const int spread = (rng() % 2) ? (int)(rng() % 13) : (int)(rng() % 3);
                Rlo[k] = (int)(rng() % (g.R_max + 1));
                Rhi[k] = std::min(Rlo[k] + spread, g.R_max);
            }
            // pixels take R in the range; the range ends are attained
            for (int i = 0; i < g.tile_w * g.tile_h; ++i) {
                active[i] = rng() % 8 != 0;
                for (int k = 0; k < 4; ++k) R[i][k] = Rlo[k] + (int)(rng() % (Rhi[k] - Rlo[k] + 1));
            }
            for (int k = 0; k < 4; ++k) {
                R[0][k] = Rlo[k];
                R[(x_hi - x_lo) + (y_hi - y_lo) * g.tile_w][k] = Rhi[k];
            }
            active[0] = true;
            active[(x_hi - x_lo) + (y_hi - y_lo) * g.tile_w] = true;
            const bool fits = frame == 0 ? cbox::boxes_fit<0>(x_lo, x_hi, y_lo, y_hi, Rlo, Rhi, g.rows)
                                         : cbox::boxes_fit<1>(x_lo, x_hi, y_lo, y_hi, Rlo, Rhi, g.rows);
            if (!fits) continue;
            ++fitting;
            const bool ok =
                frame == 0 ? check_all<0>(std::make_integer_sequence<int, cbox::kCombos>{}, g, x_lo, x_hi, y_lo, y_hi,
                                          Rlo, Rhi, R, active)
                           : check_all<1>(std::make_integer_sequence<int, cbox::kCombos>{}, g, x_lo, x_hi, y_lo, y_hi,
                                          Rlo, Rhi, R, active);
            if (!ok) {
                std::printf("frame %d case H=%ld W=%ld Rmax=%d tile %dx%d rows %d at (%d,%d) Rlo %d %d %d %d Rhi %d %d %d %d\n",
                            frame, g.H, g.W, g.R_max, g.tile_w, g.tile_h, g.rows, x_lo, y_lo, Rlo[0], Rlo[1], Rlo[2],
                            Rlo[3], Rhi[0], Rhi[1], Rhi[2], Rhi[3]);
                return 1;
            }
        }
    }
    std::printf("ok %ld %ld\n", fitting, g_taps);
    return 0;
}
