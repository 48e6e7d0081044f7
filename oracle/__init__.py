"""CPU oracle for the space-variant box-spline filter -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (``paper_1109_5114_amd``)
never imports it, and it never imports the product path.

The arithmetic lives in ``bsf_oracle.c`` (plain C, FP64 and exact integers),
written from the definitions of Chaudhury & Sanyal (arXiv:1109.5114):
Box_a and the box spline as a convolution of line boxes (Section 1.1,
eq. boxSpline), the running-sum recursion (Alg. 3 step 2) and the
space-variant filtering integral (Section 2.1).  This module only marshals
numpy arrays to it.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

U8, U16, F32, F64 = 1, 2, 3, 4
INT, REAL = 0, 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        l, i, d = ctypes.c_long, ctypes.c_int, ctypes.c_double
        L.bsfo_weights_real.argtypes = [d, P, i]
        L.bsfo_dweights_real.argtypes = [d, P, i]
        L.bsfo_weights_int.argtypes = [l, P, i]
        L.bsfo_kernel_real.argtypes = [i, P, P, P, P, P, P, P, P, l]
        L.bsfo_kernel_int.argtypes = [i, P, P, P, P, P, P, P, P, l]
        L.bsfo_filter.argtypes = [P, i, l, l, l, i, P, i, i, i, P, l, P, P, P, P, i]
        L.bsfo_grad_real.argtypes = [P, l, l, l, i, P, i, i, P, P, P, l, l, l, l, l, P, P, i]
        L.bsfo_preintegrate.argtypes = [P, i, l, l, l, i, P, i, i, l, l, l, l, P]
        L.bsfo_num_threads.argtypes = []
        L.bsfo_cov_to_steps.argtypes = [P, i, d, d, d, P]
        L.bsfo_cov_to_steps_field.argtypes = [P, i, l, P, d, P, P]
        L.bsfo_orientation.argtypes = [d, d, d]
        L.bsfo_orientation.restype = d
        L.bsfo_elongation_bound.argtypes = [d]
        L.bsfo_elongation_bound.restype = d
        L.bsfo_condition2_bound.argtypes = [d, d, d]
        L.bsfo_condition2_bound.restype = d
        L.bsfo_bank_of.argtypes = [d]
        L.bsfo_unit_box_spline.argtypes = [P, d, d]
        L.bsfo_unit_box_spline.restype = d
        L.bsfo_alg3.argtypes = [P, l, l, P, P, l, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _dtype_code(img):
    if img.dtype == np.uint8:
        return U8
    if img.dtype == np.uint16:
        return U16
    if img.dtype == np.float32:
        return F32
    if img.dtype == np.float64:
        return F64
    raise TypeError("oracle images are uint8, uint16, float32 or float64")


def num_threads():
    return lib().bsfo_num_threads()


def weights_real(s):
    """1-D factor weights w_s(i), i = -h..h, for a continuous step s."""
    buf = np.zeros(4096)
    h = lib().bsfo_weights_real(float(s), _p(buf), 4096)
    return np.arange(-h, h + 1), buf[: 2 * h + 1].copy()


def dweights_real(s):
    buf = np.zeros(4096)
    h = lib().bsfo_dweights_real(float(s), _p(buf), 4096)
    return np.arange(-h, h + 1), buf[: 2 * h + 1].copy()


def weights_int(s):
    buf = np.zeros(4096, dtype=np.int64)
    h = lib().bsfo_weights_int(int(s), _p(buf), 4096)
    return np.arange(-h, h + 1), buf[: 2 * h + 1].copy()


def _factor_dirs(fdirs):
    fd = np.ascontiguousarray(np.asarray(fdirs, dtype=np.int32).reshape(-1, 2))
    return np.ascontiguousarray(fd[:, 0]), np.ascontiguousarray(fd[:, 1])


def kernel_real(fdirs, steps):
    """Normalised kernel of one pixel: factor j has direction fdirs[j] and
    continuous step steps[j].  Returns (x0, y0, K) with K[b, a] the weight of
    the offset (x0 + a, y0 + b)."""
    dx, dy = _factor_dirs(fdirs)
    s = np.ascontiguousarray(np.asarray(steps, dtype=np.float64))
    M = len(s)
    ext = np.zeros(4, dtype=np.int64)
    L = lib()
    rc = L.bsfo_kernel_real(M, _p(dx), _p(dy), _p(s), _p(ext[0:]), ext[1:].ctypes.data,
                            ext[2:].ctypes.data, ext[3:].ctypes.data, None, 0)
    if rc:
        raise ValueError(rc)
    x0, y0, w, h = (int(v) for v in ext)
    K = np.zeros((h, w))
    rc = L.bsfo_kernel_real(M, _p(dx), _p(dy), _p(s), _p(ext[0:]), ext[1:].ctypes.data,
                            ext[2:].ctypes.data, ext[3:].ctypes.data, _p(K), K.size)
    if rc:
        raise ValueError(rc)
    return x0, y0, K


def kernel_int(fdirs, steps):
    """Unnormalised integer-step kernel (sample counts) of one pixel."""
    dx, dy = _factor_dirs(fdirs)
    s = np.ascontiguousarray(np.asarray(steps, dtype=np.int64))
    M = len(s)
    ext = np.zeros(4, dtype=np.int64)
    L = lib()
    rc = L.bsfo_kernel_int(M, _p(dx), _p(dy), _p(s), _p(ext[0:]), ext[1:].ctypes.data,
                           ext[2:].ctypes.data, ext[3:].ctypes.data, None, 0)
    if rc:
        raise ValueError(rc)
    x0, y0, w, h = (int(v) for v in ext)
    K = np.zeros((h, w), dtype=np.int64)
    rc = L.bsfo_kernel_int(M, _p(dx), _p(dy), _p(s), _p(ext[0:]), ext[1:].ctypes.data,
                           ext[2:].ctypes.data, ext[3:].ctypes.data, _p(K), K.size)
    if rc:
        raise ValueError(rc)
    return x0, y0, K


def filter(img, dirs, order, tied, mode, steps, pix=None, threads=0, want_int=False):
    """Space-variant box-spline filter, FP64 (and exact num/den for integer
    images in integer-step mode when want_int).  img [H][W]; steps
    [planes][H][W] float32; pix: optional flat pixel indices.  Returns out, or
    (out, num, den)."""
    img = np.ascontiguousarray(img)
    H, W = img.shape
    dirs = np.ascontiguousarray(np.asarray(dirs, dtype=np.int32).reshape(-1))
    steps = np.ascontiguousarray(steps, dtype=np.float32)
    planes = (len(dirs) // 2) if tied else (len(dirs) // 2) * order
    assert steps.shape == (planes, H, W), steps.shape
    if pix is not None:
        pix = np.ascontiguousarray(np.asarray(pix, dtype=np.int64).reshape(-1))
        count = len(pix)
    else:
        count = H * W
    out = np.zeros(count)
    num = np.zeros(count, dtype=np.int64) if want_int else None
    den = np.zeros(count, dtype=np.int64) if want_int else None
    rc = lib().bsfo_filter(_p(img), _dtype_code(img), H, W, W, len(dirs) // 2, _p(dirs),
                           order, int(bool(tied)), mode, _p(steps),
                           count if pix is not None else 0, _p(pix), _p(out), _p(num), _p(den),
                           int(threads))
    if rc == -2:
        raise ValueError("invalid step (below 1, or non-integer in integer mode)")
    if rc:
        raise ValueError(rc)
    if pix is None:
        out = out.reshape(H, W)
        if want_int:
            num, den = num.reshape(H, W), den.reshape(H, W)
    return (out, num, den) if want_int else out


def grad_real(img, dirs, order, tied, steps, gout, window=None, pix=None, want_img=True,
              want_steps=True, threads=0):
    """FP64 gradients of sum(gout * out) for continuous steps.

    grad_img [H][W]: contributions of the output pixels inside window
    (x0, x1, y0, y1) (default: all).  grad_steps: [planes][H][W], or
    [n][planes] when pix is given."""
    img = np.ascontiguousarray(img, dtype=np.float32)
    H, W = img.shape
    dirs = np.ascontiguousarray(np.asarray(dirs, dtype=np.int32).reshape(-1))
    n_dirs = len(dirs) // 2
    steps = np.ascontiguousarray(steps, dtype=np.float32)
    gout = np.ascontiguousarray(gout, dtype=np.float32)
    planes = n_dirs if tied else n_dirs * order
    gi = np.zeros((H, W)) if want_img else None
    if window is None:
        window = (0, W, 0, H)
    x0, x1, y0, y1 = window
    if pix is not None:
        pix = np.ascontiguousarray(np.asarray(pix, dtype=np.int64).reshape(-1))
        count = len(pix)
    else:
        count = H * W
    gs = np.zeros((count, planes)) if want_steps else None
    rc = lib().bsfo_grad_real(_p(img), H, W, W, n_dirs, _p(dirs), order, int(bool(tied)),
                              _p(steps), _p(gout), _p(gi), x0, x1, y0, y1,
                              count if pix is not None else 0, _p(pix), _p(gs), int(threads))
    if rc:
        raise ValueError(rc)
    if want_steps and pix is None:
        gs = gs.T.reshape(planes, H, W).copy()
    return gi, gs


def preintegrate(img, dirs, order, F, pads):
    """Running sums on the window; pads = (top, bottom, left, right).  Returns
    uint64 G [H + top + bottom][W + left + right]."""
    img = np.ascontiguousarray(img)
    H, W = img.shape
    dirs = np.ascontiguousarray(np.asarray(dirs, dtype=np.int32).reshape(-1))
    pt, pb, pl, pr = pads
    G = np.zeros((H + pt + pb, W + pl + pr), dtype=np.uint64)
    rc = lib().bsfo_preintegrate(_p(img), _dtype_code(img), H, W, W, len(dirs) // 2, _p(dirs),
                                 order, int(F), pt, pb, pl, pr, _p(G))
    if rc:
        raise ValueError(rc)
    return G


# ----------------------------------------------------------------------------- covariance -> steps

BANK1 = ((1, 0), (0, 1), (1, 1), (1, -1))      # the four directions of Section 1.1
BANK2 = ((2, 1), (1, 2), (1, -2), (2, -1))     # those of Alg. 3 / Table 1, canonical sign


def cov_to_steps(dirs, order, c11, c12, c22):
    """Minimum-kurtosis steps (one per direction) of the box spline along four
    integer directions with covariance C; returns (steps[4], infeasible)."""
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.int32).reshape(-1))
    out = np.zeros(4)
    r = lib().bsfo_cov_to_steps(_p(d), int(order), float(c11), float(c12), float(c22), _p(out))
    if r < 0:
        raise ValueError("degenerate directions")
    return out, bool(r)


def cov_to_steps_field(dirs, order, cov, sub=0.0):
    """cov [3][H][W] float32 (C11, C12, C22) -> steps [4][H][W] float64 and
    the per-pixel infeasibility flags [H][W]."""
    cov = np.ascontiguousarray(cov, dtype=np.float32)
    _, H, W = cov.shape
    n = H * W
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.int32).reshape(-1))
    steps = np.zeros((4, n))
    flags = np.zeros(n, dtype=np.int32)
    if lib().bsfo_cov_to_steps_field(_p(d), int(order), n, _p(cov), float(sub), _p(steps), _p(flags)):
        raise ValueError("degenerate directions")
    return steps.reshape(4, H, W), flags.reshape(H, W)


def orientation(c11, c12, c22):
    return lib().bsfo_orientation(float(c11), float(c12), float(c22))


def elongation_bound(phi):
    return lib().bsfo_elongation_bound(float(phi))


def condition2_bound(c11, c12, c22):
    return lib().bsfo_condition2_bound(float(c11), float(c12), float(c22))


def bank_of(phi):
    return lib().bsfo_bank_of(float(phi))


def alg1(img, cov, order=1, sigma2=None, steps2=None):
    """Alg. 1 written out with the oracle's pieces: sigma^2 = half the smallest
    condition2 bound (unless given), the isotropic pass with scales
    sqrt(6) sigma (sqrt(6 sigma^2 / r) lattice steps on the axes, sqrt(3 sigma^2 / r)
    on the diagonals, floored at 1), then every pixel's minimum-kurtosis steps
    for C - sigma^2 I (unless steps2 is given) on the first pass's FP64 output.
    Returns (out, sigma2, steps1, steps2)."""
    img = np.ascontiguousarray(img, dtype=np.float32)
    H, W = img.shape
    cov = np.ascontiguousarray(cov, dtype=np.float32)
    if sigma2 is None:
        b = np.array([condition2_bound(cov[0].flat[i], cov[1].flat[i], cov[2].flat[i]) for i in range(H * W)])
        b = np.where(np.isfinite(b), np.maximum(b, 0.0), 0.0)
        sigma2 = 0.5 * b.min()
    axis = max(np.sqrt(6.0 * sigma2 / order), 1.0)
    diag = max(np.sqrt(3.0 * sigma2 / order), 1.0)
    steps1 = np.empty((4, H, W), dtype=np.float32)
    for k, (dx, dy) in enumerate(BANK1):
        steps1[k] = diag if dx and dy else axis
    mid = filter(img, BANK1, order, True, REAL, steps1)
    if steps2 is None:
        steps2, _ = cov_to_steps_field(BANK1, order, cov, sub=sigma2)
    out = filter(np.ascontiguousarray(mid), BANK1, order, True, REAL, np.asarray(steps2, dtype=np.float32))
    return out, sigma2, steps1, steps2


def alg2_banks(cov):
    """The sector of Alg. 2 at every pixel: 0 for the box spline of Section
    1.1, 1 for the one of Alg. 3."""
    cov = np.asarray(cov, dtype=np.float32)
    _, H, W = cov.shape
    return np.array([bank_of(orientation(float(cov[0].flat[i]), float(cov[1].flat[i]), float(cov[2].flat[i])))
                     for i in range(H * W)], dtype=np.uint8).reshape(H, W)


def alg2(img, cov, order=2, steps=None):
    """Alg. 2 written out: each pixel filtered by the box spline of its
    sector with its minimum-kurtosis steps (or with steps = (steps_bank1,
    steps_bank2) when given).  Returns (out, banks)."""
    img = np.ascontiguousarray(img)
    H, W = img.shape
    banks = alg2_banks(cov)
    if steps is None:
        steps = (cov_to_steps_field(BANK1, order, cov)[0], cov_to_steps_field(BANK2, order, cov)[0])
    out = np.zeros(H * W)
    for bank, dirs, st in ((0, BANK1, steps[0]), (1, BANK2, steps[1])):
        pix = np.flatnonzero(banks.reshape(-1) == bank)
        if len(pix):
            st = np.where(np.isfinite(st), np.maximum(st, 1.0), 1.0).astype(np.float32)
            out[pix] = filter(img, dirs, order, True, REAL, st, pix=pix)
    return out.reshape(H, W), banks


# ----------------------------------------------------------------------------- Alg. 3

BANK2_PAPER = ((2, 1), (1, 2), (-1, 2), (-2, 1))  # Table 1's a_1 .. a_4, as the paper orients them


def _upper(dirs):
    """Each direction turned into the upper half-plane (dy > 0, or dy == 0 and
    dx > 0): the filter is the centred box spline, whatever the signs."""
    out = []
    for dx, dy in dirs:
        if dy < 0 or (dy == 0 and dx < 0):
            dx, dy = -dx, -dy
        out.append((int(dx), int(dy)))
    return out


def unit_box_spline(dirs, x, y):
    """beta_b of eq. interpolation: the box spline of one lattice step along
    each of the four directions, unit mass, at (x, y)."""
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.int32).reshape(-1))
    return lib().bsfo_unit_box_spline(_p(d), float(x), float(y))


def alg3(img, dirs, steps, pix=None):
    """Alg. 3 (running sums, eq. interpolation, Table 1 taps, eq. shifts) on a
    float image [H][W] with steps [4][H][W] (lattice steps along each
    direction, >= 1).  Returns float64 [H][W] (or the values at pix)."""
    img = np.ascontiguousarray(img, dtype=np.float32)
    H, W = img.shape
    st = np.ascontiguousarray(steps, dtype=np.float32)
    d = np.ascontiguousarray(np.asarray(_upper(dirs), dtype=np.int32).reshape(-1))
    if pix is None:
        out = np.zeros(H * W)
        r = lib().bsfo_alg3(_p(img), H, W, _p(d), _p(st), 0, None, _p(out))
        out = out.reshape(H, W)
    else:
        pix = np.ascontiguousarray(pix, dtype=np.int64)
        out = np.zeros(len(pix))
        r = lib().bsfo_alg3(_p(img), H, W, _p(d), _p(st), len(pix), _p(pix), _p(out))
    if r == -1:
        raise ValueError("directions")
    if r == -2:
        raise ValueError("a step below 1")
    if r < 0:
        raise MemoryError("alg3")
    return out
