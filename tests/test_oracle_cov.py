"""Pins of the oracle's covariance -> steps mapping (eq. cov, eq. geometry,
eq. boundE, condition2, the minimum-kurtosis choice of Section 2.4) and of the
sector rule of Alg. 2, against what the paper prints: the covariance matrices
of both four-direction box splines in terms of their scales, the isotropic
scale sqrt(6) sigma, the kurtosis matrix of the second box spline, the
closed-form elongation bound and Table 3's row for the first box spline."""
import numpy as np
import pytest

import oracle as O

B1, B2 = O.BANK1, O.BANK2


def cov_of(rho, phi, lam1):
    R = np.array([[np.cos(phi), -np.sin(phi)], [np.sin(phi), np.cos(phi)]])
    C = R @ np.diag([lam1, lam1 / rho]) @ R.T
    return C[0, 0], C[0, 1], C[1, 1]


def paper_cov_bank1(a):
    """Covariance of the box spline of Section 1.1 from its scales a_1..a_4
    along 0, 45, 90, 135 degrees (the printed (1/24) matrix)."""
    a1, a2, a3, a4 = np.asarray(a) ** 2
    return np.array([[2 * a1 + a2 + a4, a2 - a4], [a2 - a4, 2 * a3 + a2 + a4]]) / 24.0


def paper_cov_bank2(a):
    """Covariance of the box spline of Alg. 3 from its scales along 26.6, 63.4,
    116.6, 153.4 degrees (the printed (1/60) matrix)."""
    a1, a2, a3, a4 = np.asarray(a) ** 2
    return np.array([[4 * a1 + a2 + a3 + 4 * a4, 2 * (a1 + a2 - a3 - a4)],
                     [2 * (a1 + a2 - a3 - a4), a1 + 4 * a2 + 4 * a3 + a4]]) / 60.0


def paper_kurtosis_bank2(a):
    """Kurtosis matrix of the box spline of Alg. 3, up to the constant kappa/5
    (Section 2.4)."""
    a1, a2, a3, a4 = np.asarray(a) ** 4
    return np.array([[4 * a1 + a2 + a3 + 4 * a4, 2 * (a1 + a2 - a3 - a4)],
                     [2 * (a1 + a2 - a3 - a4), a1 + 4 * a2 + 4 * a3 + a4]])


def physical(steps, bank):
    """Scales in pixel lengths, in the paper's angle order: steps along the
    lattice vectors times their lengths.  Bank 1 lattice order (1,0), (0,1),
    (1,1), (1,-1) is paper order a1 (0), a3 (90), a2 (45), a4 (135)."""
    s = np.asarray(steps, dtype=float)
    if bank == 1:
        return np.array([s[0], s[2] * np.sqrt(2), s[1], s[3] * np.sqrt(2)])
    return s * np.sqrt(5.0)


def random_feasible_cov(rng, dirs):
    """A covariance inside the cone of the directions: sum_k A_k u_k u_k^T."""
    A = rng.uniform(3.0, 60.0, size=4)
    C = sum(Ak * np.outer(u, u) for Ak, u in zip(A, np.asarray(dirs, dtype=float)))
    return C[0, 0], C[0, 1], C[1, 1]


@pytest.mark.parametrize("bank", [1, 2])
def test_printed_covariance_is_reproduced(bank):
    rng = np.random.default_rng(100 + bank)
    dirs = B1 if bank == 1 else B2
    paper = paper_cov_bank1 if bank == 1 else paper_cov_bank2
    tested = 0
    for _ in range(400):
        c = random_feasible_cov(rng, dirs)
        s, bad = O.cov_to_steps(dirs, 1, *c)
        assert not bad and (s >= 1.0).all()
        if (s == 1.0).any():
            # the minimum sits where a direction's scale vanishes, floored to one step
            continue
        tested += 1
        np.testing.assert_allclose(paper(physical(s, bank)), [[c[0], c[1]], [c[1], c[2]]], rtol=1e-10, atol=1e-9)
    assert tested > 100


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("bank", [1, 2])
def test_isotropic_scales_are_sqrt6_sigma(bank, order):
    """C = sigma^2 I gives equal scales a = sqrt(6) sigma per copy (the paper's
    isotropic rule; r tied copies each carry sigma^2 / r)."""
    for sigma in (0.7, 2.0, 9.5):
        s, bad = O.cov_to_steps(B1 if bank == 1 else B2, order, sigma ** 2, 0.0, sigma ** 2)
        a = physical(s, bank)
        want = max(np.sqrt(6.0 / order) * sigma, 1.0)
        assert not bad
        np.testing.assert_allclose(a, np.maximum(want, physical(np.ones(4), bank)), rtol=1e-7)


def test_bank2_minimum_kurtosis_under_the_printed_matrix():
    """The chosen scales minimise the Frobenius norm of the printed kurtosis
    matrix among the scales with the same covariance: moving along the one
    free direction of a^2 (+1, -1, +1, -1 in the paper's order) only raises it."""
    rng = np.random.default_rng(7)
    for _ in range(100):
        c = random_feasible_cov(rng, B2)
        s, bad = O.cov_to_steps(B2, 1, *c)
        if (s == 1.0).any():
            continue   # a scale at its floor: not an interior minimum
        a2 = physical(s, 2) ** 2
        k0 = np.linalg.norm(paper_kurtosis_bank2(np.sqrt(a2)))
        for d in (1e-3, 1e-2, 1e-1):
            for sgn in (1, -1):
                b2 = a2 + sgn * d * np.array([1.0, -1.0, 1.0, -1.0])
                if (b2 <= 0).any():
                    continue
                np.testing.assert_allclose(paper_cov_bank2(np.sqrt(b2)), paper_cov_bank2(np.sqrt(a2)), atol=1e-9)
                assert np.linalg.norm(paper_kurtosis_bank2(np.sqrt(b2))) >= k0 * (1 - 1e-12)


def max_feasible_elongation(dirs, phi):
    lo, hi = 1.0, 1e5
    if not O.cov_to_steps(dirs, 1, *cov_of(hi, phi, 100.0))[1]:
        return np.inf
    for _ in range(80):
        m = np.sqrt(lo * hi)
        if O.cov_to_steps(dirs, 1, *cov_of(m, phi, 100.0))[1]:
            hi = m
        else:
            lo = m
    return lo


def test_bank1_elongation_bound_is_eq_boundE():
    """The largest elongation the first box spline reaches at orientation phi
    (where the scales stop being real) is eq. boundE, and Table 3's first row
    (13.6, 6.8, 5.9, 5.8, 5.9, 6.0, 13.6 at 5, 13.3, 20, 22.5, 25, 26.6, 40
    degrees; its 30-degree entry, 6.1, disagrees with eq. boundE's 6.46)."""
    for deg, printed in ((5, 13.6), (13.3, 6.8), (20, 5.9), (22.5, 5.8), (25, 5.9), (26.6, 6.0), (40, 13.6)):
        phi = np.deg2rad(deg)
        e = O.elongation_bound(phi)
        np.testing.assert_allclose(max_feasible_elongation(B1, phi), e, rtol=1e-6)
        assert abs(e - printed) < 0.06, (deg, e, printed)
    assert np.isinf(O.elongation_bound(0.0)) and O.elongation_bound(np.deg2rad(22.5)) == pytest.approx(
        3 + 2 * np.sqrt(2))


def test_orientation_and_geometry():
    """eq. geometry: size = trace / ... elongation = ratio of eigenvalues and
    orientation = angle of the top eigenvector, for the reproduced C."""
    rng = np.random.default_rng(9)
    for _ in range(50):
        rho, phi, lam = rng.uniform(1, 5), rng.uniform(0, np.pi), rng.uniform(1, 50)
        c = cov_of(rho, phi, lam)
        assert O.orientation(*c) == pytest.approx(phi % np.pi, abs=1e-9)


def test_condition2_keeps_the_residual_reachable():
    """condition2: below its bound C - sigma^2 I stays inside the first box
    spline's reach, above it (for anisotropic C near the bound) it leaves it."""
    rng = np.random.default_rng(11)
    for _ in range(100):
        phi = rng.uniform(0.05, np.pi / 4 - 0.05)
        e = O.elongation_bound(phi)
        c = cov_of(rng.uniform(1.2, 0.95 * e), phi, rng.uniform(5, 200))
        b = O.condition2_bound(*c)
        assert b > 0
        _, bad = O.cov_to_steps(B1, 1, c[0] - 0.999 * b, c[1], c[2] - 0.999 * b)
        assert not bad
        _, bad = O.cov_to_steps(B1, 1, c[0] - 1.001 * b, c[1], c[2] - 1.001 * b)
        assert bad
    # isotropic: the bound is the smallest eigenvalue (condition1)
    assert O.condition2_bound(4.0, 0.0, 4.0) == pytest.approx(4.0)


def test_sector_rule_switches_midway():
    """Alg. 2: an orientation takes the box spline whose axis is nearer; the
    switch points are midway between neighbouring axes (13.3 degrees between 0
    and 26.6, as Table 3's minimum)."""
    axes1 = [0.0, 45.0, 90.0, 135.0]
    axes2 = [np.degrees(np.arctan(0.5)), np.degrees(np.arctan(2.0)), 180 - np.degrees(np.arctan(2.0)),
             180 - np.degrees(np.arctan(0.5))]
    for a in axes1:
        assert O.bank_of(np.deg2rad(a)) == 0
    for a in axes2:
        assert O.bank_of(np.deg2rad(a)) == 1
    all_axes = sorted([(a, 0) for a in axes1] + [(a, 1) for a in axes2] + [(180.0, 0)])
    for (a, ka), (b, kb) in zip(all_axes, all_axes[1:]):
        mid = 0.5 * (a + b)
        assert O.bank_of(np.deg2rad(mid - 1e-6)) == ka
        assert O.bank_of(np.deg2rad(mid + 1e-6)) == kb
    assert abs(0.5 * np.degrees(np.arctan(0.5)) - 13.3) < 0.05


def test_unreachable_covariance_is_flagged():
    phi = np.deg2rad(22.5)
    c = cov_of(8.0, phi, 50.0)           # elongation 8 > e(22.5 deg) = 5.83
    s, bad = O.cov_to_steps(B1, 1, *c)
    assert bad and (s >= 1.0).all()
    s, bad = O.cov_to_steps(B2, 1, *c)   # 4 degrees from an axis of the second box spline
    assert not bad
