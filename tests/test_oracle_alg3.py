"""Pins of the oracle's Alg. 3 (the box-spline filter of Table 1 read through
eq. interpolation) against facts that do not come from the oracle itself.

- beta_b, the unit box spline of eq. interpolation, is checked against the area
  of overlap of two parallelograms computed here by polygon clipping
  (Sutherland-Hodgman, a different algorithm from the oracle's), against the
  partition of unity, its symmetry and support, and against the covariance
  (1/12) sum_k u_k u_k^T that the paper's covariance formula for the box
  spline of Alg. 3 gives at a = (sqrt5, sqrt5, sqrt5, sqrt5).
- Alg. 3 itself (running sums, 16 taps at the shifts of eq. shifts, the
  interpolation of eq. interpolation, w = 1 / prod a) must reproduce the image
  convolved with the centred box spline of the pixel's own scales, evaluated
  here by clipping: sum_p f(p) beta_a(x - p).  That is what the method is
  built to compute without the O(a^2) sum, so a dropped tap, a wrong sign, a
  wrong shift or a wrong interpolation weight fails it.
- The paper's covariance of the box spline of Alg. 3 (in terms of its scales)
  pins which scale goes with which direction in Table 1.
"""
import numpy as np
import pytest

import oracle as O

PAPER = O.BANK2_PAPER


def _clip(subject, clipper):
    """Sutherland-Hodgman: subject polygon clipped by a convex counter-clockwise clipper."""
    out = list(subject)
    n = len(clipper)
    for i in range(n):
        a, b = np.asarray(clipper[i]), np.asarray(clipper[(i + 1) % n])
        inp, out = out, []
        if not inp:
            break

        def side(p):
            return (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])

        for j in range(len(inp)):
            p, q = np.asarray(inp[j]), np.asarray(inp[(j + 1) % len(inp)])
            sp, sq = side(p), side(q)
            if sp >= 0:
                out.append(p)
            if (sp >= 0) != (sq >= 0):
                t = sp / (sp - sq)
                out.append(p + t * (q - p))
    return out


def _area(poly):
    if len(poly) < 3:
        return 0.0
    a = 0.0
    for j in range(len(poly)):
        p, q = poly[j], poly[(j + 1) % len(poly)]
        a += p[0] * q[1] - q[0] * p[1]
    return 0.5 * abs(a)


def _para(u, v, lu, lv, c):
    u, v = np.asarray(u, float) * lu, np.asarray(v, float) * lv
    pts = [c - u / 2 - v / 2, c + u / 2 - v / 2, c + u / 2 + v / 2, c - u / 2 + v / 2]
    if u[0] * v[1] - u[1] * v[0] < 0:
        pts = pts[::-1]
    return pts


def box_spline(dirs, lengths, x, y):
    """The box spline of boxes of the given lengths (lattice steps) along the
    four directions, unit mass: the overlap of the parallelograms of the first
    and the last two boxes, divided by both their areas."""
    u = [np.asarray(d, float) for d in dirs]
    P = _para(u[0], u[1], lengths[0], lengths[1], np.zeros(2))
    Q = _para(u[2], u[3], lengths[2], lengths[3], np.array([x, y], float))
    aP = abs(u[0][0] * u[1][1] - u[0][1] * u[1][0]) * lengths[0] * lengths[1]
    aQ = abs(u[2][0] * u[3][1] - u[2][1] * u[3][0]) * lengths[2] * lengths[3]
    return _area(_clip(P, Q)) / (aP * aQ)


@pytest.mark.parametrize("dirs", [PAPER, O.BANK1, ((1, 0), (0, 1), (1, 2), (2, 1))])
def test_unit_box_spline_is_the_overlap_area(dirs):
    rng = np.random.default_rng(11)
    ext = 0.5 * sum(abs(d[0]) for d in dirs) + 0.5, 0.5 * sum(abs(d[1]) for d in dirs) + 0.5
    for _ in range(400):
        x, y = (rng.random(2) * 2 - 1) * ext
        want = box_spline(dirs, (1, 1, 1, 1), x, y)
        assert O.unit_box_spline(dirs, x, y) == pytest.approx(want, abs=1e-13)


@pytest.mark.parametrize("dirs", [PAPER, O.BANK1])
def test_unit_box_spline_partition_symmetry_support(dirs):
    rng = np.random.default_rng(12)
    for _ in range(50):
        q = rng.random(2)
        tot = sum(O.unit_box_spline(dirs, q[0] - mx, q[1] - my) for mx in range(-5, 6) for my in range(-5, 6))
        assert tot == pytest.approx(1.0, abs=1e-13)
        x, y = (rng.random(2) * 2 - 1) * 3.5
        assert O.unit_box_spline(dirs, x, y) == pytest.approx(O.unit_box_spline(dirs, -x, -y), abs=1e-14)
    ex = 0.5 * sum(abs(d[0]) for d in dirs)
    ey = 0.5 * sum(abs(d[1]) for d in dirs)
    for x, y in [(ex + 1e-9, 0), (0, ey + 1e-9), (-ex - 0.1, 0.3), (0.2, -ey - 0.05)]:
        assert O.unit_box_spline(dirs, x, y) == 0.0


def test_unit_box_spline_covariance_is_the_papers():
    # the covariance of the box spline of Alg. 3 with all scales sqrt5 (one
    # lattice step along each direction): (1/60) [[4+1+1+4, 2(1+1-1-1)], [., 1+4+4+1]] * 5
    h = 0.02
    xs = np.arange(-3 + h / 2, 3, h)
    m0 = 0.0
    m2 = np.zeros((2, 2))
    for x in xs:
        for y in xs:
            b = O.unit_box_spline(PAPER, x, y)
            if b:
                m0 += b
                v = np.array([x, y])
                m2 += b * np.outer(v, v)
    m0 *= h * h
    m2 *= h * h
    a2 = np.full(4, 5.0)
    want = np.array([[4 * a2[0] + a2[1] + a2[2] + 4 * a2[3], 2 * (a2[0] + a2[1] - a2[2] - a2[3])],
                     [2 * (a2[0] + a2[1] - a2[2] - a2[3]), a2[0] + 4 * a2[1] + 4 * a2[2] + a2[3]]]) / 60
    assert m0 == pytest.approx(1.0, abs=1e-4)
    np.testing.assert_allclose(m2, want, atol=2e-4)


def test_scaled_box_spline_covariance_matches_table1_reading():
    """The paper's covariance of the box spline of Alg. 3 as a function of
    its scales a_1..a_4 holds with a_k = sqrt5 s_k along Table 1's directions
    (2,1), (1,2), (-1,2), (-2,1) in that order."""
    s = np.array([1.3, 2.1, 1.7, 2.6])
    a2 = 5 * s ** 2
    want = np.array([[4 * a2[0] + a2[1] + a2[2] + 4 * a2[3], 2 * (a2[0] + a2[1] - a2[2] - a2[3])],
                     [2 * (a2[0] + a2[1] - a2[2] - a2[3]), a2[0] + 4 * a2[1] + 4 * a2[2] + a2[3]]]) / 60
    h = 0.05
    R = 0.5 * float(np.dot(s, [2, 1, 1, 2])) + 0.01
    xs = np.arange(-R + h / 2, R, h)
    m0, m2 = 0.0, np.zeros((2, 2))
    for x in xs:
        for y in xs:
            b = box_spline(PAPER, s, x, y)
            if b:
                m0 += b
                v = np.array([x, y])
                m2 += b * np.outer(v, v)
    m0 *= h * h
    m2 *= h * h
    assert m0 == pytest.approx(1.0, abs=2e-3)
    np.testing.assert_allclose(m2, want, rtol=5e-3, atol=5e-3)


def _direct(img, dirs, steps, x, y):
    H, W = img.shape
    tot = 0.0
    s = [float(steps[k, y, x]) for k in range(4)]
    rx = 0.5 * sum(abs(d[0]) * sk for d, sk in zip(dirs, s)) + 1
    ry = 0.5 * sum(abs(d[1]) * sk for d, sk in zip(dirs, s)) + 1
    for py in range(max(0, int(y - ry)), min(H, int(y + ry) + 1)):
        for px in range(max(0, int(x - rx)), min(W, int(x + rx) + 1)):
            b = box_spline(dirs, s, x - px, y - py)
            if b:
                tot += float(img[py, px]) * b
    return tot


@pytest.mark.parametrize("kind", ["real", "integer", "half", "one"])
def test_alg3_is_the_image_convolved_with_the_pixels_box_spline(kind):
    rng = np.random.default_rng({"real": 1, "integer": 2, "half": 3, "one": 4}[kind])
    H, W = 9, 11
    img = rng.random((H, W)).astype(np.float32)
    if kind == "real":
        steps = 1 + 2.5 * rng.random((4, H, W))
    elif kind == "integer":
        steps = rng.integers(1, 4, (4, H, W)).astype(float)
    elif kind == "half":
        steps = rng.integers(2, 7, (4, H, W)) / 2.0
    else:
        steps = np.ones((4, H, W))
    steps = steps.astype(np.float32)
    out = O.alg3(img, PAPER, steps)
    pts = [(x, y) for y in range(H) for x in range(W)]
    idx = rng.choice(len(pts), 40, replace=False)
    for i in idx:
        x, y = pts[i]
        assert out[y, x] == pytest.approx(_direct(img, PAPER, steps, x, y), abs=1e-12), (x, y)


def test_alg3_other_directions_and_signs():
    """Any four directions in a half-plane; the signs of the directions do not
    change the result (the filter is the centred box spline)."""
    rng = np.random.default_rng(5)
    H, W = 8, 9
    img = rng.random((H, W)).astype(np.float32)
    steps = (1 + 2 * rng.random((4, H, W))).astype(np.float32)
    for dirs in (O.BANK1, ((1, 0), (0, 1), (1, 2), (2, 1)), O.BANK2):
        out = O.alg3(img, dirs, steps)
        for x, y in [(0, 0), (4, 3), (8, 7), (2, 6)]:
            assert out[y, x] == pytest.approx(_direct(img, dirs, steps, x, y), abs=1e-12)
    np.testing.assert_allclose(O.alg3(img, O.BANK2, steps), O.alg3(img, PAPER, steps), atol=1e-12)


def test_alg3_pixels_subset_and_errors():
    rng = np.random.default_rng(6)
    img = rng.random((7, 6)).astype(np.float32)
    steps = (1 + rng.random((4, 7, 6))).astype(np.float32)
    full = O.alg3(img, PAPER, steps)
    pix = np.array([0, 5, 17, 41])
    np.testing.assert_array_equal(O.alg3(img, PAPER, steps, pix=pix), full.reshape(-1)[pix])
    bad = steps.copy()
    bad[2, 3, 3] = 0.5
    with pytest.raises(ValueError):
        O.alg3(img, PAPER, bad)
