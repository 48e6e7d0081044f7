"""GPU parity of Alg. 3 (running sums, the 16 taps of Table 1 read through
eq. interpolation, in FP64) against the oracle's Alg. 3.

Tolerance.  The oracle accumulates the running sums of the whole zero-extended
image in long double; the GPU takes them in FP64 inside each tile's rectangle,
where they stay below (rectangle points) x (representations of an offset) x
max|f|, about 1e7 max|f| for the largest rectangles here, so every sum and
every interpolated tap carries an absolute rounding error near
2^-53 x 1e7 x (a few hundred operations), about 1e-7 of a unit in the worst
case and far less in practice; the 16 taps and 1 / prod s do not enlarge it.
The tests allow 1e-9 max|f| (measured errors are below 1e-11) on the FP64
output and one FP32 rounding more on the FP32 output."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1109_5114_amd as bsf
import workloads as WL
from tests.gpu_util import note

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
TABLE1 = WL.DIRS_TABLE1
TOL = 1e-9


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def run(cfg, img, steps):
    H, W = img.shape
    ws = bsf.Workspace(bsf.lib().bsf_alg3_workspace_bytes(bsf.ctypes.byref(cfg.c()), H, W), DEV)
    o64 = torch.empty((H, W), dtype=torch.float64, device=DEV)
    o32 = torch.empty((H, W), dtype=torch.float32, device=DEV)
    bsf.filter_alg3(cfg, to_dev(img), to_dev(steps), out=o32, out_f64=o64, ws=ws)
    flags, _, _ = ws.status()
    return o32.cpu().numpy(), o64.cpu().numpy(), flags


def check(out32, out64, ref, scale):
    err = np.abs(out64 - ref)
    assert err.max() <= TOL * scale, (err.max(), np.unravel_index(np.argmax(err), err.shape))
    np.testing.assert_array_equal(out32, out64.astype(np.float32))


@pytest.mark.parametrize("dirs", [TABLE1, O.BANK1, ((1, 0), (0, 1), (1, 2), (2, 1))])
def test_alg3_matches_oracle(dirs):
    note("alg3 dirs", dirs)
    rng = np.random.default_rng(700 + len(str(dirs)))
    H, W = 45, 70                         # 3 x 5 tiles, ragged on both sides
    img = rng.random((H, W), dtype=np.float32)
    steps = np.stack([WL.smooth(rng, H, W, 1.0, 5.0) for _ in range(4)]).astype(np.float32)
    steps[:, 10:14, 20:30] = np.round(steps[:, 10:14, 20:30])      # integer steps
    steps[:, 30:33, 5:9] = 1.0                                        # the unit box spline itself
    cfg = bsf.Config(dirs=dirs, order=1, max_step=6.0)
    o32, o64, flags = run(cfg, img, steps)
    ref = O.alg3(img, dirs, steps)
    check(o32, o64, ref, 1.0)
    assert flags == 0


def test_alg3_integer_image():
    note("alg3 u8")
    rng = np.random.default_rng(710)
    H, W = 33, 41
    img = rng.integers(0, 256, (H, W)).astype(np.uint8)
    steps = (1 + 3 * rng.random((4, H, W))).astype(np.float32)
    cfg = bsf.Config(dirs=TABLE1, order=1, max_step=4.0)
    o32, o64, flags = run(cfg, img, steps)
    ref = O.alg3(img.astype(np.float32), TABLE1, steps)
    check(o32, o64, ref, 255.0)
    assert flags == 0


def test_alg3_sub_tiles():
    """Steps near max_step = 20: a tile whose rectangle does not fit the LDS
    buffer works in 8 x 8, 4 x 4, 2 x 2 or 1 x 1 pieces."""
    note("alg3 sub-tiles")
    rng = np.random.default_rng(720)
    H, W = 48, 48
    img = rng.random((H, W), dtype=np.float32)
    steps = (1 + rng.random((4, H, W))).astype(np.float32)
    steps[:, 0:16, 16:32] = (18.0 + 0.8 * rng.random((4, 16, 16))).astype(np.float32)   # 8 x 8 pieces
    steps[:, 32:48, 32:48] = (18.9 + 0.4 * rng.random((4, 16, 16))).astype(np.float32)  # 4 x 4 or 2 x 2
    steps[:, 16:32, 0:16] = (19.6 + 0.4 * rng.random((4, 16, 16))).astype(np.float32)   # 1 x 1
    cfg = bsf.Config(dirs=TABLE1, order=1, max_step=20.0)
    o32, o64, flags = run(cfg, img, steps)
    ys, xs = np.mgrid[0:H, 0:W]
    pix = np.concatenate([np.flatnonzero(((ys < 16) & (xs >= 16) & (xs < 32)).ravel())[::5],
                          np.flatnonzero(((ys >= 32) & (xs >= 32)).ravel())[::7],
                          np.flatnonzero(((ys >= 16) & (ys < 32) & (xs < 16)).ravel())[::9],
                          np.arange(0, H * W, 97)])
    ref = O.alg3(img, TABLE1, steps, pix=pix)
    err = np.abs(o64.reshape(-1)[pix] - ref)
    assert err.max() <= TOL, err.max()
    assert flags == 0


def test_alg3_range_and_nonfinite():
    note("alg3 range")
    rng = np.random.default_rng(730)
    H, W = 20, 24
    img = rng.random((H, W), dtype=np.float32)
    steps = (1 + 2 * rng.random((4, H, W))).astype(np.float32)
    steps[1, 3, 4] = 0.5
    steps[2, 7, 9] = np.nan
    steps[0, 15, 20] = 4.5
    cfg = bsf.Config(dirs=TABLE1, order=1, max_step=4.0)
    o32, o64, flags = run(cfg, img, steps)
    assert flags == bsf.FLAG_RANGE
    bad = np.zeros((H, W), bool)
    bad[3, 4] = bad[7, 9] = bad[15, 20] = True
    assert np.isnan(o64[bad]).all() and np.isnan(o32[bad]).all()
    good = np.flatnonzero(~bad.reshape(-1))
    ref = O.alg3(img, TABLE1, steps, pix=good)
    assert np.abs(o64.reshape(-1)[good] - ref).max() <= TOL
    img2 = img.copy()
    img2[10, 10] = np.inf
    ok = np.ones((4, H, W), np.float32)
    _, o64b, flags = run(cfg, img2, ok)
    assert flags == bsf.FLAG_NONFINITE
    assert not np.isfinite(o64b[10, 10])


def test_alg3_rejects():
    note("alg3 rejects")
    H, W = 8, 8
    for cfg in (bsf.Config(dirs=TABLE1, order=2, max_step=4.0),
                bsf.Config(dirs=TABLE1[:3], order=1, max_step=4.0),
                bsf.Config(dirs=TABLE1, order=1, max_step=40.0)):
        assert bsf.lib().bsf_alg3_workspace_bytes(bsf.ctypes.byref(cfg.c()), H, W) == 0
        with pytest.raises(bsf.BsfError):
            bsf.filter_alg3(cfg, torch.zeros((H, W), device=DEV), torch.ones((cfg.planes, H, W), device=DEV))


def test_alg3_full_size_sampled():
    """The 4096 x 4096 covariance-field workload, steps from bsf_cov_to_steps for
    the box spline of Table 1; sampled pixels against the oracle on crops that
    hold each pixel's footprint (outside it the filter reads nothing)."""
    d = WL.workload_alg3()
    H, W = d["img"].shape
    note("alg3 full size", H, W)
    cfg = bsf.Config(dirs=TABLE1, order=1, max_step=d["max_step"])
    steps = bsf.cov_to_steps(cfg, to_dev(d["cov"])).cpu().numpy()
    o32, o64, flags = run(cfg, d["img"], steps)
    assert flags == 0
    assert np.isfinite(o64).all()
    rng = np.random.default_rng(740)
    pts = [(0, 0), (W - 1, H - 1), (0, H - 1), (W - 1, 0)] + [tuple(p) for p in rng.integers(0, [W, H], (60, 2))]
    for x, y in pts:
        s = steps[:, y, x].astype(np.float64)
        rx = int(np.ceil(0.5 * sum(abs(u[0]) * sk for u, sk in zip(TABLE1, s)))) + 3
        ry = int(np.ceil(0.5 * sum(abs(u[1]) * sk for u, sk in zip(TABLE1, s)))) + 3
        x0, x1, y0, y1 = max(0, x - rx), min(W, x + rx + 1), max(0, y - ry), min(H, y + ry + 1)
        crop = np.ascontiguousarray(d["img"][y0:y1, x0:x1])
        st = np.ascontiguousarray(steps[:, y0:y1, x0:x1])
        ref = O.alg3(crop, TABLE1, st, pix=np.array([(y - y0) * (x1 - x0) + (x - x0)]))[0]
        assert abs(o64[y, x] - ref) <= TOL, (x, y, o64[y, x], ref)
    np.testing.assert_array_equal(o32, o64.astype(np.float32))


def test_alg3_every_pixel_2048():
    """Every pixel of the covariance-field workload at 2048 x 2048 (steps from
    bsf_cov_to_steps for the box spline of Table 1) against the oracle's
    Alg. 3, block by block: each 128 x 128 block on a crop that holds its
    pixels' footprints (the filter reads nothing outside them).  Over the
    whole frame the oracle's own running sums, of order four, would reach
    about 1e12 max|f| and lose the digits this comparison needs."""
    d = WL.workload_alg3(2048, 2048)
    H, W = d["img"].shape
    note("alg3 every pixel", H, W)
    cfg = bsf.Config(dirs=TABLE1, order=1, max_step=d["max_step"])
    steps = bsf.cov_to_steps(cfg, to_dev(d["cov"])).cpu().numpy()
    o32, o64, flags = run(cfg, d["img"], steps)
    assert flags == 0
    np.testing.assert_array_equal(o32, o64.astype(np.float32))
    S = float(steps.max())
    mx = int(np.ceil(0.5 * S * sum(abs(u[0]) for u in TABLE1))) + 4
    my = int(np.ceil(0.5 * S * sum(abs(u[1]) for u in TABLE1))) + 4
    B = 128
    worst = 0.0
    for y0 in range(0, H, B):
        for x0 in range(0, W, B):
            cx0, cx1, cy0, cy1 = max(0, x0 - mx), min(W, x0 + B + mx), max(0, y0 - my), min(H, y0 + B + my)
            crop = np.ascontiguousarray(d["img"][cy0:cy1, cx0:cx1])
            st = np.ascontiguousarray(steps[:, cy0:cy1, cx0:cx1])
            ys, xs = np.mgrid[y0:min(H, y0 + B), x0:min(W, x0 + B)]
            pix = ((ys - cy0) * (cx1 - cx0) + (xs - cx0)).ravel()
            ref = O.alg3(crop, TABLE1, st, pix=pix).reshape(ys.shape)
            worst = max(worst, float(np.abs(o64[y0:y0 + B, x0:x0 + B] - ref).max()))
    assert worst <= TOL, worst
