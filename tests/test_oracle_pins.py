"""Pins of the CPU oracle against what the paper and the mathematics fix:
brute-force enumeration, closed forms (mass, mean, covariance, Fourier
transform), textbook special cases, the paper's printed values and its
propositions.  None of these re-run the oracle's own formulas."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import workloads as WL
from tests import brute

DIRS4 = [(1, 0), (0, 1), (1, 1), (1, -1)]


def var_discrete(s):
    """Variance of the normalised factor weights: the mixture
    (1-lam) box_{|i|<=r} + lam box_{|i|<=r+1} of two odd boxes (closed form)."""
    r = math.floor((s - 1) / 2)
    lam = (s - 2 * r - 1) / 2
    return ((1 - lam) * r * (r + 1) * (2 * r + 1) / 3 + lam * (r + 1) * (r + 2) * (2 * r + 3) / 3) / s


def dirichlet(q, th):
    """D_q(th) = sum_{|i|<=q} exp(-i i th) = sin((2q+1) th/2) / sin(th/2)."""
    if abs(math.sin(th / 2)) < 1e-300:
        return 2 * q + 1
    return math.sin((2 * q + 1) * th / 2) / math.sin(th / 2)


# ---------------------------------------------------------------- factor weights

@pytest.mark.parametrize("s", [1.0, 1.5, 2.0, 2.25, 3.0, 4.7, 7.0, 10.125, 33.3])
def test_factor_weights_mass_symmetry_and_cells(s):
    i, w = O.weights_real(s)
    assert abs(w.sum() - s) < 1e-12                     # a box of length s has mass s
    np.testing.assert_array_equal(w, w[::-1])           # symmetric
    for ii, wi in zip(i, w):                            # exact unit-cell overlaps
        assert wi == float(brute.box_cell_weight(int(ii), Fraction(s)))


@pytest.mark.parametrize("s", [1, 3, 5, 9, 15])
def test_factor_weights_odd_integer_is_plain_box(s):
    i, w = O.weights_real(float(s))
    np.testing.assert_array_equal(w, (np.abs(i) <= (s - 1) // 2).astype(float))
    ii, wi = O.weights_int(s)
    np.testing.assert_array_equal(wi, (np.abs(ii) <= (s - 1) // 2).astype(np.int64))


@pytest.mark.parametrize("s", [1, 2, 3, 4, 6, 7, 10, 31])
def test_factor_weights_int_half_open_box(s):
    """Box_a is 1/a on (-a/2, a/2]: as a convolution kernel the sample at
    offset i is taken when -a/2 < -i <= a/2; an even length gets its extra
    sample on the -u side."""
    i, w = O.weights_int(s)
    want = [ii for ii in i if -s / 2 < -ii <= s / 2]
    assert list(i[w == 1]) == want
    assert w.sum() == s
    if s % 2 == 0:
        assert i[w == 1].min() == -(s // 2) and i[w == 1].max() == s // 2 - 1


@pytest.mark.parametrize("s", [1.25, 2.0, 2.5, 3.9, 8.2])
def test_factor_weight_derivative_is_half_at_both_ends(s):
    i, dw = O.dweights_real(s)
    assert abs(dw.sum() - 1.0) < 1e-15                  # d/ds (mass s) = 1
    h = 1e-7
    _, wp = O.weights_real(s + h)
    _, w0 = O.weights_real(s)
    n = min(len(wp), len(w0))
    c0, cp = len(w0) // 2, len(wp) // 2
    k = min(c0, cp)
    fd = (wp[cp - k:cp + k + 1] - w0[c0 - k:c0 + k + 1]) / h
    np.testing.assert_allclose(fd, dw[c0 - k:c0 + k + 1], atol=1e-6)


# ---------------------------------------------------------------- kernels by brute force

@pytest.mark.parametrize("fdirs,steps", [
    ([(1, 0), (0, 1)], [2.5, 1.75]),
    ([(1, 0), (0, 1), (1, 1), (1, -1)], [3.3, 2.6, 2.2, 1.7]),
    ([(1, 0), (1, 0), (1, 1), (1, 1)], [2.5, 2.5, 1.5, 1.5]),
    ([(2, 1), (1, 2), (1, -2), (2, -1)], [1.5, 2.25, 1.0, 3.0]),
    ([(1, 0), (0, 1), (1, 1), (1, -1), (1, 0)], [1.5, 1.25, 2.0, 1.0, 2.75]),
])
def test_kernel_real_matches_enumeration(fdirs, steps):
    x0, y0, K = O.kernel_real(fdirs, steps)
    bd = brute.kernel_by_enumeration_real(fdirs, [Fraction(s) for s in steps])
    for (px, py), v in bd.items():
        assert abs(K[py - y0, px - x0] - float(v)) < 1e-14
    assert abs(K.sum() - sum(float(v) for v in bd.values())) < 1e-13


@pytest.mark.parametrize("fdirs,steps", [
    ([(1, 0), (0, 1)], [2, 3]),
    ([(1, 0), (0, 1), (1, 1), (1, -1)], [4, 3, 2, 5]),
    ([(1, 0), (1, 0), (0, 1), (0, 1)], [2, 4, 3, 1]),
])
def test_kernel_int_matches_enumeration(fdirs, steps):
    x0, y0, K = O.kernel_int(fdirs, steps)
    bd = brute.kernel_by_enumeration_int(fdirs, steps)
    dense = np.zeros_like(K)
    for (px, py), v in bd.items():
        dense[py - y0, px - x0] = v
    np.testing.assert_array_equal(K, dense)


# ---------------------------------------------------------------- closed forms

def moments(K, x0, y0):
    h, w = K.shape
    xs = (x0 + np.arange(w))[None, :].astype(float)
    ys = (y0 + np.arange(h))[:, None].astype(float)
    m = K.sum()
    mx, my = (K * xs).sum() / m, (K * ys).sum() / m
    cxx = (K * (xs - mx) ** 2).sum() / m
    cyy = (K * (ys - my) ** 2).sum() / m
    cxy = (K * (xs - mx) * (ys - my)).sum() / m
    return m, mx, my, np.array([[cxx, cxy], [cxy, cyy]])


@pytest.mark.parametrize("seed", range(6))
def test_kernel_real_mass_mean_covariance(seed):
    """Mass 1, centred, covariance sum_j v(s_j) u_j u_j^T: the factor variances
    add under convolution (Prop. 1) and v is the discrete variance of the
    two-box mixture."""
    rng = np.random.default_rng(seed)
    fdirs = DIRS4 * (1 + seed % 2)
    steps = rng.uniform(1.0, 9.0, size=len(fdirs))
    x0, y0, K = O.kernel_real(fdirs, steps)
    m, mx, my, C = moments(K, x0, y0)
    assert abs(m - 1.0) < 1e-12
    assert abs(mx) < 1e-11 and abs(my) < 1e-11
    want = sum(var_discrete(s) * np.outer(u, u) for s, u in zip(steps, fdirs))
    np.testing.assert_allclose(C, want, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(K, K[::-1, ::-1], atol=1e-15)   # even kernel


@pytest.mark.parametrize("seed", range(4))
def test_kernel_int_mean_covariance(seed):
    """Integer steps: counts sum to prod s; factor mean 0 (odd) or -1/2 (even);
    factor variance (s^2 - 1)/12 (discrete uniform)."""
    rng = np.random.default_rng(100 + seed)
    steps = [int(v) for v in rng.integers(1, 9, size=4)]
    x0, y0, K = O.kernel_int(DIRS4, steps)
    m, mx, my, C = moments(K.astype(float), x0, y0)
    assert K.sum() == np.prod(steps)
    mu = sum((0.0 if s % 2 else -0.5) * np.array(u) for s, u in zip(steps, DIRS4))
    assert abs(mx - mu[0]) < 1e-12 and abs(my - mu[1]) < 1e-12
    want = sum((s * s - 1) / 12 * np.outer(u, u) for s, u in zip(steps, DIRS4))
    np.testing.assert_allclose(C, want, atol=1e-11)


@pytest.mark.parametrize("seed", range(4))
def test_kernel_real_fourier_product_form(seed):
    """DTFT of the kernel = prod_j [(1-lam_j) D_{r_j} + lam_j D_{r_j+1}](w.u_j) / s_j."""
    rng = np.random.default_rng(200 + seed)
    fdirs = DIRS4 * 2 if seed % 2 else DIRS4
    steps = rng.uniform(1.0, 7.0, size=len(fdirs))
    x0, y0, K = O.kernel_real(fdirs, steps)
    for wx, wy in rng.uniform(-math.pi, math.pi, size=(8, 2)):
        got = brute.dtft(K, x0, y0, wx, wy)
        want = 1.0
        for s, (dx, dy) in zip(steps, fdirs):
            r = math.floor((s - 1) / 2)
            lam = (s - 2 * r - 1) / 2
            th = wx * dx + wy * dy
            want *= ((1 - lam) * dirichlet(r, th) + lam * dirichlet(r + 1, th)) / s
        assert abs(got - want) < 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_kernel_int_fourier_product_form(seed):
    """DTFT of the integer kernel = prod_j exp(-i mu_j w.u_j) sin(s w.u/2)/sin(w.u/2)."""
    rng = np.random.default_rng(300 + seed)
    steps = [int(v) for v in rng.integers(1, 8, size=4)]
    x0, y0, K = O.kernel_int(DIRS4, steps)
    for wx, wy in rng.uniform(-math.pi, math.pi, size=(6, 2)):
        got = brute.dtft(K.astype(float), x0, y0, wx, wy)
        want = 1.0 + 0j
        for s, (dx, dy) in zip(steps, DIRS4):
            th = wx * dx + wy * dy
            mu = 0.0 if s % 2 else -0.5
            want *= np.exp(-1j * mu * th) * math.sin(s * th / 2) / math.sin(th / 2)
        assert abs(got - want) < 1e-9 * max(1.0, abs(want))


def test_kernel_covariance_tends_to_paper_formula():
    """eq. cov: the four-direction box spline with physical scales a_k has
    covariance (1/24)[[2a1^2+a2^2+a4^2, a2^2-a4^2], [., 2a3^2+a2^2+a4^2]]
    (a1 on the x axis, a2 on the diagonal, a3 on the y axis, a4 on the
    anti-diagonal).  With a lattice step count s along u, a = s|u|; the
    discrete kernel differs from the continuous one by O(1) per factor."""
    s = dict(x=40.0, d=28.5, y=33.0, a=21.25)
    fdirs = [(1, 0), (1, 1), (0, 1), (-1, 1)]
    steps = [s["x"], s["d"], s["y"], s["a"]]
    x0, y0, K = O.kernel_real(fdirs, steps)
    _, _, _, C = moments(K, x0, y0)
    a1, a2, a3, a4 = s["x"], s["d"] * math.sqrt(2), s["y"], s["a"] * math.sqrt(2)
    paper = np.array([[2 * a1 ** 2 + a2 ** 2 + a4 ** 2, a2 ** 2 - a4 ** 2],
                      [a2 ** 2 - a4 ** 2, 2 * a3 ** 2 + a2 ** 2 + a4 ** 2]]) / 24
    # each factor's discrete variance is within 1/12 of s^2/12 (|u|^2 <= 2)
    assert np.abs(C - paper).max() <= 4 * 2 / 12 + 1e-9
    assert np.abs(C - paper).max() / np.abs(paper).max() < 2e-3
    # eq. geometry: size = trace = sum a^2 / 12
    assert abs(np.trace(paper) - (a1 ** 2 + a2 ** 2 + a3 ** 2 + a4 ** 2) / 12) < 1e-9


def test_isotropic_rule():
    """Equal scales a = sqrt(6) sigma give covariance sigma^2 I (Section 1.1)."""
    sig = 3.7
    a = math.sqrt(6) * sig
    paper = np.array([[2 * a * a + a * a + a * a, 0], [0, 2 * a * a + 2 * a * a]]) / 24
    np.testing.assert_allclose(paper, sig * sig * np.eye(2))


def test_fourier_large_step_limit_is_sinc_product():
    """Large-step limit: the factor transform D(w.u)/s tends to sinc(s w.u/2),
    the building block of the product in Theorem 1 (eq. conv)."""
    steps = [60.0, 60.0, 42.0, 42.0]
    x0, y0, K = O.kernel_real(DIRS4, steps)
    for wx, wy in [(0.01, 0.0), (0.02, -0.015), (0.0, 0.03)]:
        got = brute.dtft(K, x0, y0, wx, wy).real
        want = np.prod([np.sinc(s * (wx * dx + wy * dy) / 2 / math.pi)
                        for s, (dx, dy) in zip(steps, DIRS4)])
        assert abs(got - want) < 2e-3


# ---------------------------------------------------------------- the filter

def small_case(seed, H=23, W=29, mode="real", order=1, lo=1.0, hi=5.0, tied=True):
    rng = np.random.default_rng(seed)
    img = rng.random((H, W), dtype=np.float32)
    planes = 4 if tied else 4 * order
    steps = rng.uniform(lo, hi, size=(planes, H, W)).astype(np.float32)
    if mode == "int":
        steps = np.rint(steps).astype(np.float32)
    return img, steps


def test_filter_impulse_response_is_kernel():
    """Fig. 6 idea: filtering an impulse returns the kernel (reflected)."""
    H = W = 41
    img = np.zeros((H, W), np.float32)
    img[20, 20] = 1.0
    s = [3.5, 2.25, 2.75, 1.5]
    steps = np.stack([np.full((H, W), v, np.float32) for v in s])
    out = O.filter(img, DIRS4, 1, True, O.REAL, steps)
    x0, y0, K = O.kernel_real(DIRS4, s)
    h, w = K.shape
    for b in range(h):
        for a in range(w):
            # out(x) = sum_p K(p) f(x + p): impulse at c gives out(c - p) = K(p)
            assert abs(out[20 - (y0 + b), 20 - (x0 + a)] - K[b, a]) < 1e-15


def test_filter_constant_image_interior_and_linearity():
    img, steps = small_case(1, H=40, W=44, hi=4.0)
    ones = np.ones_like(img)
    out1 = O.filter(ones, DIRS4, 1, True, O.REAL, steps)
    reach = 2 + 2 + 2 + 3          # |offset| <= sum_j (R_j+1)|u_j|_inf with s <= 4
    inner = out1[reach:-reach, reach:-reach]
    np.testing.assert_allclose(inner, 1.0, atol=1e-14)
    a = O.filter(img, DIRS4, 1, True, O.REAL, steps)
    g = np.random.default_rng(5).random(img.shape, dtype=np.float32)
    b = O.filter(g, DIRS4, 1, True, O.REAL, steps)
    c = O.filter((img + 2 * g).astype(np.float32), DIRS4, 1, True, O.REAL, steps)
    # img + 2g is rounded to float32, so compare against that exact input
    lin = a + 2 * b
    assert np.abs(c - lin).max() < 1e-6


def test_filter_axis_only_is_bilinear_summed_area_box():
    """Axis directions only, continuous steps: the mean of the nearest-
    neighbour image over the rectangle [x - sx/2, x + sx/2] x [y - sy/2, y + sy/2],
    i.e. Crow's summed-area table read with bilinear interpolation."""
    rng = np.random.default_rng(9)
    H, W = 30, 34
    img = rng.random((H, W), dtype=np.float32)
    sx = rng.uniform(1.0, 8.0, size=(H, W)).astype(np.float32)
    sy = rng.uniform(1.0, 8.0, size=(H, W)).astype(np.float32)
    out = O.filter(img, [(1, 0), (0, 1)], 1, True, O.REAL, np.stack([sx, sy]))
    # summed-area table of the piecewise-constant image with cells [i-1/2,i+1/2)
    sat = np.zeros((H + 1, W + 1))
    sat[1:, 1:] = np.cumsum(np.cumsum(img.astype(np.float64), 0), 1)

    def I(xc, yc):
        # integral over (-inf, xc] x (-inf, yc] of the cell image; cell i spans [i-1/2, i+1/2)
        u, v = np.clip(xc + 0.5, 0, W), np.clip(yc + 0.5, 0, H)
        i0, j0 = int(min(math.floor(u), W - 1)), int(min(math.floor(v), H - 1))
        fu, fv = u - i0, v - j0
        return ((1 - fu) * (1 - fv) * sat[j0, i0] + fu * (1 - fv) * sat[j0, i0 + 1]
                + (1 - fu) * fv * sat[j0 + 1, i0] + fu * fv * sat[j0 + 1, i0 + 1])

    for y in range(H):
        for x in range(W):
            a, b = float(sx[y, x]) / 2, float(sy[y, x]) / 2
            want = (I(x + a, y + b) - I(x - a, y + b) - I(x + a, y - b) + I(x - a, y - b)) / (4 * a * b)
            assert abs(out[y, x] - want) < 1e-12


def test_filter_int_axis_only_is_summed_area_box():
    """Integer steps on the axes: the textbook summed-area-table box sum."""
    rng = np.random.default_rng(10)
    H, W = 27, 31
    img = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    sx = rng.integers(1, 9, size=(H, W)).astype(np.float32)
    sy = rng.integers(1, 9, size=(H, W)).astype(np.float32)
    out, num, den = O.filter(img, [(1, 0), (0, 1)], 1, True, O.INT, np.stack([sx, sy]), want_int=True)
    sat = np.zeros((H + 1, W + 1), dtype=np.int64)
    sat[1:, 1:] = np.cumsum(np.cumsum(img.astype(np.int64), 0), 1)

    def S(xi, yi):   # sum over cols < xi, rows < yi (clipped)
        return sat[min(max(yi, 0), H), min(max(xi, 0), W)]

    for y in range(H):
        for x in range(W):
            a, b = int(sx[y, x]), int(sy[y, x])
            ca, cb = (a - 1) // 2, (b - 1) // 2
            x1, x0 = x + ca + 1, x + ca - a + 1
            y1, y0 = y + cb + 1, y + cb - b + 1
            want = S(x1, y1) - S(x0, y1) - S(x1, y0) + S(x0, y0)
            assert num[y, x] == want and den[y, x] == a * b


def test_prop2_two_pass_equals_one_pass():
    """Prop. 2: a convolution with constant steps b followed by the
    space-variant filter with steps a(x) equals one space-variant filter whose
    kernel is the convolution of both, i.e. the untied order-2 filter with
    factors (a, b) per direction, away from the border."""
    rng = np.random.default_rng(11)
    H, W = 48, 52
    img = rng.random((H, W), dtype=np.float32)
    a = rng.uniform(1.0, 4.0, size=(4, H, W)).astype(np.float32)
    bconst = [2.5, 1.5, 1.75, 2.0]
    b = np.stack([np.full((H, W), v, np.float32) for v in bconst])
    # two passes in FP64: the oracle takes float32 images, so run the first
    # pass and feed its FP64 result through the kernel sum by hand
    first = O.filter(img, DIRS4, 1, True, O.REAL, b)
    reach = 14
    untied = np.empty((8, H, W), np.float32)
    for k in range(4):
        untied[2 * k] = a[k]
        untied[2 * k + 1] = b[k]
    one = O.filter(img, DIRS4, 2, False, O.REAL, untied)
    for y in range(reach, H - reach):
        for x in range(reach, W - reach):
            s = [float(a[k, y, x]) for k in range(4)]
            x0, y0, K = O.kernel_real(DIRS4, s)
            h, w = K.shape
            two = (K * first[y + y0:y + y0 + h, x + x0:x + x0 + w]).sum()
            assert abs(two - one[y, x]) < 1e-13


# ---------------------------------------------------------------- pre-integration

def test_preintegrate_matches_definition_when_lines_leave_through_zeros():
    """Directions whose backward lines leave the window through the zero part
    of the plane: the windowed recursions equal G(p) = sum_k f(p - sum k_j u_j)."""
    rng = np.random.default_rng(12)
    f = rng.integers(0, 9, size=(4, 5)).astype(np.uint8)
    for fdirs, order in [([(1, 0), (0, 1), (1, 1)], 1), ([(1, 0), (0, 1)], 2), ([(1, 1), (2, 1)], 1)]:
        pads = (3, 3, 3, 4)
        G = O.preintegrate(f, fdirs, order, 0, pads)
        window = (-pads[0], 4 + pads[1], -pads[2], 5 + pads[3])
        want = brute.preintegrate_by_definition(f, [d for d in fdirs for _ in range(order)], window)
        for (y, x), v in want.items():
            assert int(G[y + pads[0], x + pads[2]]) == v % (1 << 64)


def _taps_int(G, pads, fdirs, svec, x, y):
    """Table 1 pattern: sum over eps in {0,1}^M of (-1)^|eps| G at
    x + sum_j (c_j - eps_j s_j) u_j, c_j = floor((s_j - 1)/2); mod 2^64 then signed."""
    acc = 0
    for eps in itertools.product((0, 1), repeat=len(fdirs)):
        px, py = x, y
        for e, s, (dx, dy) in zip(eps, svec, fdirs):
            m = (s - 1) // 2 - e * s
            px += m * dx
            py += m * dy
        assert 0 <= py + pads[0] < G.shape[0] and 0 <= px + pads[2] < G.shape[1]
        acc += (-1) ** sum(eps) * int(G[py + pads[0], px + pads[2]])
    acc %= 1 << 64
    return acc - (1 << 64) if acc >= 1 << 63 else acc


@pytest.mark.parametrize("order", [1, 2])
def test_running_sums_and_signed_taps_reproduce_filter_int(order):
    """The BoxFilter identity (Section 1.1; Table 1 signs (-1)^popcount): the
    2^M signed taps of the pre-integrated image give the integer filter's
    numerator exactly, including the anti-diagonal pass whose window
    truncation the taps cancel."""
    rng = np.random.default_rng(13 + order)
    H, W = 13, 17
    img = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    steps = rng.integers(1, 5, size=(4, H, W)).astype(np.float32)
    smax = 4
    reach = 3 * order * (smax + 1)      # |sum_j m_j u_j| with |m_j| <= s_j per factor
    pads = (reach, reach, reach, reach)
    G = O.preintegrate(img, DIRS4, order, 0, pads)
    out, num, den = O.filter(img, DIRS4, order, True, O.INT, steps, want_int=True)
    fdirs = [d for d in DIRS4 for _ in range(order)]
    for y in range(H):
        for x in range(W):
            svec = [int(steps[j // order, y, x]) for j in range(4 * order)]
            assert _taps_int(G, pads, fdirs, svec, x, y) == num[y, x]


@pytest.mark.parametrize("dirs", [
    ((2, 1), (1, 2), (1, -2), (2, -1)),     # the directions of Alg. 3 / Table 1
    ((1, -2), (2, -1), (2, 1), (1, 2)),     # both upward directions first
    ((1, -1), (1, 0), (0, 1), (1, 1)),      # the anti-diagonal first
])
@pytest.mark.parametrize("order", [1, 2])
def test_signed_taps_cancel_truncation_of_any_pass(dirs, order):
    """Lines of every running sum start at zero where they enter the window;
    what that leaves out is cancelled by the signed taps whichever passes point
    upward and in whatever order they run, so the taps reproduce the integer
    filter exactly for any direction set (the reading under which the library
    accepts any canonical directions)."""
    rng = np.random.default_rng(17 + order)
    H, W = 11, 13
    img = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    steps = rng.integers(1, 5, size=(4, H, W)).astype(np.float32)
    reach = 2 * 4 * order * (4 + 1)
    pads = (reach, reach, reach, reach)
    G = O.preintegrate(img, dirs, order, 0, pads)
    out, num, den = O.filter(img, dirs, order, True, O.INT, steps, want_int=True)
    fdirs = [d for d in dirs for _ in range(order)]
    for y in range(H):
        for x in range(W):
            svec = [int(steps[j // order, y, x]) for j in range(4 * order)]
            assert _taps_int(G, pads, fdirs, svec, x, y) == num[y, x]


def _table1():
    """Rows of tests/golden/table1_fd_mesh.txt: (cx[4], cy[4], sign)."""
    import os
    rows = []
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_fd_mesh.txt")
    for line in open(path):
        line = line.split("#")[0].split()
        if not line:
            continue
        v = [int(t) for t in line[1:9]]
        rows.append((v[:4], v[4:], +1 if line[9] == "+" else -1))
    return rows


def test_table1_mesh_and_shifts_reproduce_the_filter():
    """Table 1 (finite-difference mesh of beta'_a in Alg. 3) with the shifts of
    eq. (shifts): the 16 printed taps, read at x - tau on running sums that
    accumulate from the +u side along the four directions of beta' (the
    directions are those of the single-scale rows 1, 2, 4 and 8), give the
    oracle's integer filter for odd scales a' (tau is then a lattice point).
    This pins the oracle's directions, step units (a' = a / sqrt 5), centring
    and signs against the printed table."""
    rows = _table1()
    assert len(rows) == 16
    dirs = []
    for k, i in enumerate((1, 2, 4, 8)):
        cx, cy, _ = rows[i]
        dirs.append((cx[k], cy[k]))
    assert dirs == [(2, 1), (1, 2), (-1, 2), (-2, 1)]
    # row i carries the scales of the binary digits of i, sign (-1)^(digits)
    for i, (cx, cy, sg) in enumerate(rows):
        used = [k for k in range(4) if cx[k] or cy[k]]
        assert used == [k for k in range(4) if i >> k & 1]
        assert sg == (-1) ** len(used)
    rng = np.random.default_rng(21)
    H, W = 11, 14
    img = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    steps = (2 * rng.integers(0, 3, size=(4, H, W)) + 1).astype(np.float32)   # a' in {1, 3, 5}
    pad = 24
    G = O.preintegrate(img, [(-dx, -dy) for dx, dy in dirs], 1, 0, (pad, pad, pad, pad))
    _, num, den = O.filter(img, dirs, 1, True, O.INT, steps, want_int=True)
    for y in range(H):
        for x in range(W):
            a = [int(steps[k, y, x]) for k in range(4)]
            t1 = (2 * a[0] + a[1] - a[2] - 2 * a[3]) // 2
            t2 = (a[0] + 2 * a[1] + 2 * a[2] + a[3] - 6) // 2
            acc = 0
            for cx, cy, sg in rows:
                px = x - t1 + sum(c * v for c, v in zip(cx, a))
                py = y - t2 + sum(c * v for c, v in zip(cy, a))
                acc += sg * int(G[py + pad, px + pad])
            acc %= 1 << 64
            acc = acc - (1 << 64) if acc >= 1 << 63 else acc
            assert acc == num[y, x], (y, x, a)
            assert den[y, x] == np.prod(a)


def test_running_sums_and_interpolated_taps_reproduce_filter_real():
    """Continuous steps: reading the running sum linearly between lattice
    points along each u_j (the one-direction restriction of eq.
    interpolation) gives the unit-cell-integrated box filter.  Per factor the
    tap pair is (1-phi)[T_R - T_{-R-1}] + phi[T_{R+1} - T_{-R-2}] with
    R = floor((s-1)/2), phi = (s-1)/2 - R; the bracketed integer differences are
    combined exactly before the phase weights are applied."""
    rng = np.random.default_rng(15)
    H, W = 11, 13
    img = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    steps = rng.uniform(1.0, 4.5, size=(4, H, W)).astype(np.float32)
    pads = (16, 16, 16, 16)
    G = O.preintegrate(img, DIRS4, 1, 0, pads)
    ref = O.filter(img, DIRS4, 1, True, O.REAL, steps)
    for y in range(H):
        for x in range(W):
            s = [float(steps[k, y, x]) for k in range(4)]
            R = [math.floor((v - 1) / 2) for v in s]
            ph = [(v - 1) / 2 - r for v, r in zip(s, R)]
            tot = 0.0
            for e in itertools.product((0, 1), repeat=4):
                J = 0
                for t in itertools.product((0, 1), repeat=4):
                    px, py = x, y
                    for k in range(4):
                        m = (R[k] + e[k]) if t[k] == 0 else (-R[k] - 1 - e[k])
                        px += m * DIRS4[k][0]
                        py += m * DIRS4[k][1]
                    J += (-1) ** sum(t) * int(G[py + pads[0], px + pads[2]])
                J %= 1 << 64
                J = J - (1 << 64) if J >= 1 << 63 else J
                wgt = np.prod([ph[k] if e[k] else 1 - ph[k] for k in range(4)])
                tot += wgt * J
            assert abs(tot / np.prod(s) - ref[y, x]) < 1e-12


# ---------------------------------------------------------------- adjoint

@pytest.mark.parametrize("order,tied", [(1, True), (2, True), (2, False)])
def test_adjoint_dot_product(order, tied):
    img, steps = small_case(20 + order, H=21, W=24, order=order, hi=4.0, tied=tied)
    g = np.random.default_rng(30).standard_normal(img.shape).astype(np.float32)
    out = O.filter(img, DIRS4, order, tied, O.REAL, steps)
    gi, _ = O.grad_real(img, DIRS4, order, tied, steps, g, want_steps=False)
    lhs = float((out * g.astype(np.float64)).sum())
    rhs = float((img.astype(np.float64) * gi).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("order", [1, 2])
def test_grad_steps_central_differences(order):
    """Central differences, h = 1e-3, FP64; entries whose step is within 2h of
    an odd integer (a kink of the phase) are masked."""
    img, steps = small_case(40 + order, H=12, W=14, order=order, lo=1.2, hi=4.0)
    g = np.random.default_rng(41).standard_normal(img.shape).astype(np.float32)
    _, gs = O.grad_real(img, DIRS4, order, True, steps, g, want_img=False)
    h = 1e-3
    rng = np.random.default_rng(42)
    checked = 0
    for _ in range(40):
        q = int(rng.integers(0, 4))
        y, x = int(rng.integers(0, 12)), int(rng.integers(0, 14))
        s0 = float(steps[q, y, x])
        if abs((s0 - 1) / 2 - round((s0 - 1) / 2)) * 2 < 2 * h + 1e-6:
            continue
        vals = []
        for sgn in (1, -1):
            st = steps.astype(np.float64).copy()
            st[q, y, x] = s0 + sgn * h
            # steps are float32 inputs; evaluate the perturbed pixel's kernel in FP64
            s = [st[k, y, x] for k in range(4)]
            fdirs = [d for d in DIRS4 for _ in range(order)]
            x0, y0, K = O.kernel_real(fdirs, [v for v in s for _ in range(order)])
            hh, ww = K.shape
            pad = np.zeros((12 + 2 * 40, 14 + 2 * 40))
            pad[40:52, 40:54] = img
            vals.append((K * pad[40 + y + y0:40 + y + y0 + hh, 40 + x + x0:40 + x + x0 + ww]).sum())
        fd = g[y, x] * (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gs[q, y, x]) <= 1e-4 * max(1.0, abs(fd))
        checked += 1
    assert checked >= 20


# ---------------------------------------------------------------- paper values used by the inputs

def test_elongation_bound_matches_table_previous_row():
    """eq. boundE against the 'previous bound' row of the elongation-bound
    table (Section 3); the 30 degree entry (6.1 printed, 6.46 by the formula)
    is taken from the formula."""
    row = {5: 13.6, 13.3: 6.8, 20: 5.9, 22.5: 5.8, 25: 5.9, 26.6: 6.0, 40: 13.6}
    for deg, v in row.items():
        assert abs(float(WL.elongation_bound(math.radians(deg))) - v) < 0.06
    assert math.isinf(float(WL.elongation_bound(0.0)))
    assert abs(float(WL.elongation_bound(math.radians(22.5))) - (3 + 2 * math.sqrt(2))) < 1e-9


def test_steps_from_cov_reproduce_covariance():
    rng = np.random.default_rng(50)
    th = rng.uniform(0, math.pi, 200)
    rho = np.minimum(rng.uniform(1, 6, 200), 0.9 * WL.elongation_bound(th))
    sig = rng.uniform(6, 24, 200)
    C11, C12, C22 = WL.cov_field(th, rho, sig)
    s = WL.steps_from_cov(C11, C12, C22)
    ok = np.all(np.stack(s) > 1.0, axis=0)
    A = [v * v / 12 for v in s]
    np.testing.assert_allclose((A[0] + A[2] + A[3])[ok], C11[ok], rtol=1e-9)
    np.testing.assert_allclose((A[1] + A[2] + A[3])[ok], C22[ok], rtol=1e-9)
    np.testing.assert_allclose((A[2] - A[3])[ok], C12[ok], rtol=1e-9, atol=1e-9)
