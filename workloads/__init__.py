"""Seeded synthetic inputs for the space-variant box-spline filter.

This module holds input recipes only: images, per-pixel step fields and
upstream gradients.  It contains none of the filter's arithmetic (no running
sums, no finite differences), so the GPU path and the CPU oracle can both read
its outputs without sharing any of the method.

The paper measures on analytic Gaussians and impulse images and ships no
dataset, so every workload is synthetic.  Workload i draws from
``numpy.random.default_rng(11095114 + i)`` in the order written in its
function.  Steps are lattice steps along each direction; continuous step
fields come from a smooth covariance field mapped to the four-direction box
spline by the covariance formula (eq. cov) and the minimum-kurtosis choice the
paper borrows from its predecessor (Section 1.1), with the elongation capped
below the bound e(phi) of eq. boundE.
"""
import math

import numpy as np

SEED0 = 11095114
DIRS4 = ((1, 0), (0, 1), (1, 1), (1, -1))


def smooth(rng, H, W, lo, hi, terms=8, kmax=4):
    """Sum of `terms` low-frequency cosines cos(2*pi*(kx*x/W + ky*y/H) + ph),
    kx, ky integers in [-kmax, kmax] not both zero, ph ~ U[0, 2*pi); rescaled
    affinely so that its min and max are lo and hi.  float64 [H][W]."""
    ks = []
    while len(ks) < terms:
        kx, ky = (int(v) for v in rng.integers(-kmax, kmax + 1, size=2))
        if kx == 0 and ky == 0:
            continue
        ks.append((kx, ky, float(rng.uniform(0.0, 2.0 * math.pi))))
    x = np.arange(W, dtype=np.float64)[None, :] / W
    y = np.arange(H, dtype=np.float64)[:, None] / H
    acc = np.zeros((H, W))
    for kx, ky, ph in ks:
        # cos(a + b) = cos a cos b - sin a sin b keeps this separable and cheap
        a = 2.0 * math.pi * kx * x + ph
        b = 2.0 * math.pi * ky * y
        acc += np.cos(a) * np.cos(b) - np.sin(a) * np.sin(b)
    mn, mx = acc.min(), acc.max()
    return lo + (acc - mn) * (hi - lo) / (mx - mn)


def elongation_bound(phi):
    """e(phi) of eq. boundE: the largest eigenvalue ratio the four-direction
    box spline reaches at orientation phi (inf on the axes and diagonals)."""
    phi = np.asarray(phi, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.abs(np.tan(phi) - 1.0 / np.tan(phi)) / 2.0
        r = np.sqrt(1.0 + t * t)
        e = (1.0 + t + r) / (1.0 + t - r)
    return np.where(np.isfinite(e), e, np.inf)


def cov_field(theta, rho, sigma):
    """C = R_theta diag(sigma^2, sigma^2/rho) R_theta^T, returned as (C11, C12, C22)."""
    l1 = sigma * sigma
    l2 = l1 / rho
    c, s = np.cos(theta), np.sin(theta)
    return l1 * c * c + l2 * s * s, (l1 - l2) * s * c, l1 * s * s + l2 * c * c


def steps_from_cov(C11, C12, C22):
    """Grid steps (s1..s4) along (1,0), (0,1), (1,1), (1,-1) of the box spline
    whose covariance sum_k (s_k^2/12) u_k u_k^T equals C (eq. cov with the
    scale counted in lattice steps), choosing among the one-parameter family of
    solutions the one of least kurtosis: with A_k = s_k^2/12 and the free
    parameter t = A3 + A4, minimise the Frobenius norm of
    sum_k A_k^2 |u_k|^2 u_k u_k^T over t in [|C12|, min(C11, C22)].  That norm
    is convex in t.  Its derivative (over 4) is the cubic
        h(t) = 8 t^3 - 6 S t^2 + 4 (C11^2 + C22^2 + 2 C12^2) t
               - (C11^3 + C22^3 + C12^2 S),   S = C11 + C22,
    strictly increasing on the whole line (its depressed form has
    p = ((5 C11^2 - 6 C11 C22 + 5 C22^2)/16 + C12^2) > 0), so it has one real
    root, found by Cardano's formula, polished by two Newton steps and clamped
    to the feasible interval.  Steps are floored at 1.  Vectorised."""
    C11 = np.asarray(C11, dtype=np.float64)
    C12 = np.asarray(C12, dtype=np.float64)
    C22 = np.asarray(C22, dtype=np.float64)
    lo = np.abs(C12)
    hi = np.maximum(np.minimum(C11, C22), lo)
    c2 = C12 * C12
    S = C11 + C22
    a2, a1, a0 = -6.0 * S / 8.0, 4.0 * (C11 * C11 + C22 * C22 + 2.0 * c2) / 8.0, \
        -(C11 ** 3 + C22 ** 3 + c2 * S) / 8.0
    p = a1 - a2 * a2 / 3.0
    q = 2.0 * a2 ** 3 / 27.0 - a2 * a1 / 3.0 + a0
    disc = np.sqrt(np.maximum(q * q / 4.0 + p ** 3 / 27.0, 0.0))
    t = np.cbrt(-q / 2.0 + disc) + np.cbrt(-q / 2.0 - disc) - a2 / 3.0
    for _ in range(2):
        h = 8.0 * t ** 3 - 6.0 * S * t * t + 8.0 * a1 * t + 8.0 * a0
        dh = 24.0 * t * t - 12.0 * S * t + 8.0 * a1
        t = t - h / dh
    t = np.clip(t, lo, hi)
    A = [np.maximum(C11 - t, 0.0), np.maximum(C22 - t, 0.0),
         np.maximum((t + C12) / 2.0, 0.0), np.maximum((t - C12) / 2.0, 0.0)]
    return [np.maximum(np.sqrt(12.0 * Ak), 1.0) for Ak in A]


def _uniform_image(rng, H, W):
    return rng.random((H, W), dtype=np.float32)


# --------------------------------------------------------------------------
# The five workloads.  Each returns a dict: img, steps [planes][H][W] float32,
# dirs, order, tied, mode ("int" | "real"), plus workload-specific extras.
# --------------------------------------------------------------------------

def workload1(H=256, W=256, seed=SEED0 + 0):
    """FP32 uniform[0,1) image; four directions at order 1; integer steps in
    [1, 15] from smooth fields (one field per direction)."""
    rng = np.random.default_rng(seed)
    img = _uniform_image(rng, H, W)
    steps = np.stack([np.rint(smooth(rng, H, W, 1.0, 15.0)) for _ in range(4)]).astype(np.float32)
    return dict(name="integer-steps order-1 %dx%d fp32" % (H, W), img=img, steps=steps,
                dirs=DIRS4, order=1, tied=True, mode="int", max_step=15.0)


def workload2(H=4096, W=4096, seed=SEED0 + 1):
    """FP32 uniform[0,1) image with 5% salt-and-pepper; four directions, each
    pre-integrated twice (order 2, steps tied per direction); per-pixel
    elliptical covariance from smooth fields: orientation in [0, pi),
    elongation (eigenvalue ratio) in [1, 6] capped at 0.9 e(theta), sigma (the
    larger eigenvalue's square root) in [2, 24] px.  Each of the two box
    splines carries half the covariance (Prop. 1)."""
    rng = np.random.default_rng(seed)
    img = _uniform_image(rng, H, W)
    mask = rng.random((H, W)) < 0.05
    salt = (rng.random((H, W)) < 0.5).astype(np.float32)
    img = np.where(mask, salt, img).astype(np.float32)
    theta = smooth(rng, H, W, 0.0, math.pi)
    rho = smooth(rng, H, W, 1.0, 6.0)
    sigma = smooth(rng, H, W, 2.0, 24.0)
    rho = np.minimum(rho, 0.9 * elongation_bound(theta))
    rho = np.maximum(rho, 1.0)
    C11, C12, C22 = cov_field(theta, rho, sigma)
    steps = np.stack(steps_from_cov(C11 / 2, C12 / 2, C22 / 2)).astype(np.float32)
    return dict(name="order-2 tied %dx%d fp32 covariance field" % (H, W), img=img, steps=steps,
                dirs=DIRS4, order=2, tied=True, mode="real",
                max_step=float(np.ceil(steps.max())))


def workload3(H=2048, W=2048, seed=SEED0 + 2):
    """uint8 image of piecewise-constant blocks (sides 4..64 px, random
    levels) plus uniform integer noise in [-16, 16], clipped; four directions at
    order 1; integer steps in [1, 31]."""
    rng = np.random.default_rng(seed)
    widths, heights = [], []
    while sum(widths) < W:
        widths.append(int(rng.integers(4, 65)))
    while sum(heights) < H:
        heights.append(int(rng.integers(4, 65)))
    levels = rng.integers(0, 256, size=(len(heights), len(widths)))
    xs = np.repeat(np.arange(len(widths)), widths)[:W]
    ys = np.repeat(np.arange(len(heights)), heights)[:H]
    base = levels[ys[:, None], xs[None, :]]
    noise = rng.integers(-16, 17, size=(H, W))
    img = np.clip(base + noise, 0, 255).astype(np.uint8)
    steps = np.stack([np.rint(smooth(rng, H, W, 1.0, 31.0)) for _ in range(4)]).astype(np.float32)
    return dict(name="integer-steps order-1 %dx%d uint8" % (H, W), img=img, steps=steps,
                dirs=DIRS4, order=1, tied=True, mode="int", max_step=31.0)


def workload4(B=64, lo=128, hi=2048, seed=SEED0 + 3):
    """B FP32 uniform images of random non-square sides in [lo, hi]; isotropic
    order-2 box splines with sigma in [1, 16] from a smooth field: each copy
    carries sigma^2/2 I, so a = sqrt(3) sigma, i.e. sqrt(3) sigma steps on the
    axes and sqrt(1.5) sigma steps on the diagonals."""
    rng = np.random.default_rng(seed)
    items = []
    for _ in range(B):
        H, W = (int(v) for v in rng.integers(lo, hi + 1, size=2))
        img = _uniform_image(rng, H, W)
        sig = smooth(rng, H, W, 1.0, 16.0)
        sa = np.maximum(math.sqrt(3.0) * sig, 1.0)
        sd = np.maximum(math.sqrt(1.5) * sig, 1.0)
        steps = np.stack([sa, sa, sd, sd]).astype(np.float32)
        items.append(dict(img=img, steps=steps))
    max_step = float(np.ceil(max(it["steps"].max() for it in items)))
    return dict(name="batched %d images %d..%d order-2 tied" % (B, lo, hi), items=items,
                dirs=DIRS4, order=2, tied=True, mode="real", max_step=max_step)


def workload5(B=16, H=1024, W=1024, seed=SEED0 + 4):
    """B FP32 uniform images; order-2 tied steps, each direction's plane an
    independent smooth field in [1.5, 20]; standard-normal upstream gradient;
    the finite-difference check uses rows and columns [480, 544) of image 0."""
    rng = np.random.default_rng(seed)
    imgs = rng.random((B, H, W), dtype=np.float32)
    steps = np.stack([np.stack([smooth(rng, H, W, 1.5, 20.0) for _ in range(4)])
                      for _ in range(B)]).astype(np.float32)
    gout = rng.standard_normal((B, H, W), dtype=np.float32)
    return dict(name="forward+adjoint %dx %dx%d order-2 tied" % (B, H, W), imgs=imgs,
                steps=steps, gout=gout, dirs=DIRS4, order=2, tied=True, mode="real",
                max_step=20.0, fd_crop=(480, 544, 480, 544))


# The directions of Alg. 3 / Table 1, in the library's canonical sign
# ((-1,2) and (-2,1) turned to (1,-2) and (2,-1)).
DIRS_TABLE1 = ((2, 1), (1, 2), (1, -2), (2, -1))


def workload_alg3(H=4096, W=4096, seed=SEED0 + 5):
    """The image of workload2 (FP32 uniform[0,1) with 5% salt-and-pepper) and a
    per-pixel elliptical covariance from smooth fields for the box spline of
    Table 1: orientation in [0, pi), elongation in [1, 6], sigma in [2, 12] px.
    Returns img and cov [3][H][W] float32 (C11, C12, C22); the steps are the
    minimum-kurtosis scales of that box spline for cov."""
    rng = np.random.default_rng(seed)
    img = _uniform_image(rng, H, W)
    mask = rng.random((H, W)) < 0.05
    salt = (rng.random((H, W)) < 0.5).astype(np.float32)
    img = np.where(mask, salt, img).astype(np.float32)
    theta = smooth(rng, H, W, 0.0, math.pi)
    rho = smooth(rng, H, W, 1.0, 6.0)
    sigma = smooth(rng, H, W, 2.0, 12.0)
    cov = np.stack(cov_field(theta, rho, sigma)).astype(np.float32)
    return dict(name="Alg. 3 %dx%d fp32 covariance field" % (H, W), img=img, cov=cov,
                dirs=DIRS_TABLE1, order=1, tied=True, mode="real", max_step=21.0)
