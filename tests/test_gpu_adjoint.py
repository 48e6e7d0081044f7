"""GPU parity of the adjoint: gradients with respect to the steps (the
forward's own derivative output times the upstream gradient) and with respect
to the image (fixed-point scatter of the transposed taps, then transposed
running sums), against the FP64 oracle, the dot-product identity, torch
autograd, and central finite differences on the 64x64 crop of the
differentiation workload."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1109_5114_amd as bsf
import workloads as WL
from tests.gpu_util import note

pytestmark = pytest.mark.gpu

DIRS4 = ((1, 0), (0, 1), (1, 1), (1, -1))


def case(shape, planes, lo, hi, seed, smooth=False):
    rng = np.random.default_rng(seed)
    img = rng.random(shape, dtype=np.float32)
    if smooth:
        steps = np.stack([WL.smooth(rng, *shape, lo, hi) for _ in range(planes)]).astype(np.float32)
    else:
        steps = rng.uniform(lo, hi, size=(planes,) + shape).astype(np.float32)
    g = rng.standard_normal(shape).astype(np.float32)
    return img, steps, g


def gpu_grads(cfg, img, steps, g):
    dev = torch.device("cuda:0")
    ti, ts, tg = (torch.from_numpy(a).to(dev) for a in (img, steps, g))
    ds = torch.empty_like(ts)
    out = bsf.filter_varying(cfg, ti, ts, dsteps=ds)
    gi, gs = bsf.filter_backward(cfg, ts, tg, dsteps=ds)
    return out.cpu().numpy(), gi.cpu().numpy(), gs.cpu().numpy(), ds.cpu().numpy()


def assert_grad_close(got, ref, rel_norm=1e-6, rel_max=1e-5, what=""):
    got = got.astype(np.float64)
    err = np.abs(got - ref)
    scale = max(np.abs(ref).max(), 1e-30)
    nrm = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30)
    assert nrm <= rel_norm, "%s: normwise %.3g" % (what, nrm)
    assert err.max() <= rel_max * scale, "%s: max %.3g of %.3g" % (what, err.max(), scale)
    return nrm


@pytest.mark.parametrize("order,tied,shape,hi,smooth", [
    (2, True, (40, 46), 9.0, False),     # tied order-2 four-direction kernels
    (2, True, (33, 37), 14.0, True),
    (1, True, (30, 34), 7.0, False),     # generic kernels, order 1
    (2, False, (11, 13), 3.5, False),    # generic kernels, untied order 2
])
def test_gradients_match_oracle(order, tied, shape, hi, smooth):
    note("adjoint", order, tied, shape)
    planes = 4 if tied else 4 * order
    img, steps, g = case(shape, planes, 1.0, hi, 31 + order, smooth)
    cfg = bsf.Config(order=order, tied=tied, max_step=hi)
    out, gi, gs, ds = gpu_grads(cfg, img, steps, g)
    rgi, rgs = O.grad_real(img, DIRS4, order, tied, steps, g)
    assert_grad_close(gi, rgi, what="grad_img")
    # right derivative at kinks on both sides; a step whose phase sits within
    # float rounding of a kink can take the other one-sided value
    assert_grad_close(gs, rgs, what="grad_steps")


@pytest.mark.parametrize("shape,hi,smooth", [
    ((44, 52), 11.0, True),
    ((120, 136), 12.0, True),     # many tiles through the cluster boxes
    ((61, 77), 9.0, False),       # independent steps: most tiles scatter pixel by pixel
])
def test_gradients_table1_directions(shape, hi, smooth):
    """Step derivatives from the forward's cluster-box kernel in the frame of
    Table 1's directions, and the image gradient from the adjoint's cluster-box
    scatter in that frame (tiles whose boxes do not fit scatter each pixel's
    taps to the window directly), against the oracle's analytic gradients."""
    note("adjoint table1 directions", shape, smooth)
    dirs = ((2, 1), (1, 2), (1, -2), (2, -1))
    img, steps, g = case(shape, 4, 1.0, hi, 71, smooth=smooth)
    cfg = bsf.Config(dirs=dirs, order=2, max_step=hi)
    out, gi, gs, ds = gpu_grads(cfg, img, steps, g)
    rgi, rgs = O.grad_real(img, dirs, 2, True, steps, g)
    assert_grad_close(gi, rgi, what="grad_img")
    assert_grad_close(gs, rgs, what="grad_steps")


def test_dot_product_identity_on_gpu():
    """<K f, g> = <f, K^T g> with the GPU forward and the GPU adjoint."""
    note("dot product")
    img, steps, g = case((64, 70), 4, 1.0, 16.0, 41, smooth=True)
    cfg = bsf.Config(order=2, max_step=16.0)
    out, gi, _, _ = gpu_grads(cfg, img, steps, g)
    lhs = float((out.astype(np.float64) * g).sum())
    rhs = float((img.astype(np.float64) * gi).sum())
    assert abs(lhs - rhs) <= 1e-6 * (np.abs(out * g).sum())


def test_autograd_function():
    note("autograd")
    img, steps, g = case((36, 40), 4, 1.0, 10.0, 43)
    cfg = bsf.Config(order=2, max_step=10.0)
    dev = torch.device("cuda:0")
    ti = torch.from_numpy(img).to(dev).requires_grad_(True)
    ts = torch.from_numpy(steps).to(dev).requires_grad_(True)
    out = bsf.filter(ti, ts, cfg)
    out.backward(torch.from_numpy(g).to(dev))
    _, gi, gs, _ = gpu_grads(cfg, img, steps, g)
    np.testing.assert_array_equal(ti.grad.cpu().numpy(), gi)
    np.testing.assert_array_equal(ts.grad.cpu().numpy(), gs)
    # image only: the steps' derivative is not computed
    ti.grad = None
    ts2 = torch.from_numpy(steps).to(dev)
    bsf.filter(ti, ts2, cfg).backward(torch.from_numpy(g).to(dev))
    np.testing.assert_array_equal(ti.grad.cpu().numpy(), gi)


def test_zero_upstream_gradient():
    note("zero gout")
    img, steps, _ = case((20, 22), 4, 1.0, 6.0, 45)
    cfg = bsf.Config(order=2, max_step=6.0)
    _, gi, gs, _ = gpu_grads(cfg, img, steps, np.zeros((20, 22), np.float32))
    assert not gi.any() and not gs.any()


@pytest.mark.slow
def test_differentiation_workload_crop_finite_differences():
    """Image 0 of the differentiation workload (1024^2, steps in [1.5, 20]):
    the step gradient on the 64x64 crop against FP64 central differences of
    the oracle (h = 1e-3; entries within 2h of a phase kink masked) and against
    the oracle's analytic gradient; the image gradient on the crop against the
    oracle's adjoint."""
    note("fd crop 1024")
    d = WL.workload5(B=1)
    img, steps, g = d["imgs"][0], d["steps"][0], d["gout"][0]
    y0, y1, x0, x1 = d["fd_crop"]
    cfg = bsf.Config(order=2, max_step=20.0)
    out, gi, gs, ds = gpu_grads(cfg, img, steps, g)
    H, W = img.shape
    ys, xs = np.mgrid[y0:y1, x0:x1]
    pix = (ys * W + xs).reshape(-1)
    # analytic oracle gradient on the crop
    _, rgs = O.grad_real(img, DIRS4, 2, True, steps, g, pix=pix, want_img=False)
    got = gs.reshape(4, -1)[:, pix].T
    assert_grad_close(got, rgs, what="grad_steps crop")
    # central differences: out at one pixel depends only on its own steps
    h = 1e-3
    rng = np.random.default_rng(47)
    sel = rng.choice(len(pix), 96, replace=False)
    fd, an = [], []
    for n in sel:
        p = int(pix[n])
        y, x = divmod(p, W)
        for q in range(4):
            s0 = float(steps[q, y, x])
            if abs((s0 - 1) / 2 - round((s0 - 1) / 2)) * 2 < 2 * h:
                continue
            vals = []
            for sgn in (1, -1):
                sv = [float(steps[k, y, x]) for k in range(4)]
                sv[q] = s0 + sgn * h
                kx0, ky0, K = O.kernel_real([u for u in DIRS4 for _ in range(2)], [v for v in sv for _ in range(2)])
                kh, kw = K.shape
                acc = 0.0
                for b in range(kh):
                    yy = y + ky0 + b
                    if 0 <= yy < H:
                        xa, xb = max(0, x + kx0), min(W, x + kx0 + kw)
                        acc += float((K[b, xa - (x + kx0):xb - (x + kx0)] * img[yy, xa:xb]).sum())
                vals.append(acc)
            fd.append(float(g[y, x]) * (vals[0] - vals[1]) / (2 * h))
            an.append(float(gs[q, y, x]))
    fd, an = np.array(fd), np.array(an)
    assert len(fd) > 300
    assert np.abs(fd - an).max() <= 1e-4 * max(1.0, np.abs(fd).max())
    # image gradient on the crop: every output pixel whose footprint can reach
    # the crop contributes (reach < 2 * 11 * 3 + 8 = 74 px)
    m = 74
    rgi, _ = O.grad_real(img, DIRS4, 2, True, steps, g,
                         window=(max(0, x0 - m), min(W, x1 + m), max(0, y0 - m), min(H, y1 + m)),
                         want_steps=False)
    assert_grad_close(gi[y0:y1, x0:x1], rgi[y0:y1, x0:x1], what="grad_img crop")


@pytest.mark.slow
def test_full_size_image_gradient_crops():
    """The 4096 x 4096 order-2 workload (steps up to 48) through the forward
    and the adjoint exactly as the benchmark runs them: the image gradient on
    three 24 x 24 crops (centre, top-left corner, bottom-right edge) against the
    FP64 oracle's adjoint restricted to the output pixels that reach each crop,
    and the step gradient at sampled pixels against the oracle's derivative."""
    note("adjoint 4096 crops")
    d = WL.workload2(4096, 4096)
    img, steps = d["img"], d["steps"]
    g = np.random.default_rng(11095114 + 99).standard_normal(img.shape, dtype=np.float32)
    cfg = bsf.Config(order=2, max_step=d["max_step"])
    out, gi, gs, ds = gpu_grads(cfg, img, steps, g)
    H, W = img.shape
    R = int((d["max_step"] - 1) // 2)
    reach = 2 * (R + 2) * 3 + 2
    for (y0, x0, n) in ((2040, 2040, 24), (0, 0, 24), (H - 24, W - 24, 24)):
        win = (max(0, x0 - reach), min(W, x0 + n + reach), max(0, y0 - reach), min(H, y0 + n + reach))
        rgi, _ = O.grad_real(img, DIRS4, 2, True, steps, g, window=win, want_steps=False)
        assert_grad_close(gi[y0:y0 + n, x0:x0 + n], rgi[y0:y0 + n, x0:x0 + n], rel_norm=1e-6, rel_max=1e-5,
                          what="grad_img crop %d,%d" % (y0, x0))
    rng = np.random.default_rng(53)
    pix = np.concatenate([rng.integers(0, H * W, 40), [0, W - 1, H * W - 1]])
    _, rgs = O.grad_real(img, DIRS4, 2, True, steps, g, pix=pix, want_img=False)
    assert_grad_close(gs.reshape(4, -1)[:, pix].T, rgs, what="grad_steps sampled")


# ----------------------------------------------------------------------------- fixed-point headroom

def backward_only(cfg, steps, g, ws=None):
    dev = torch.device("cuda:0")
    ts, tg = torch.from_numpy(steps).to(dev), torch.from_numpy(g).to(dev)
    H, W = g.shape
    ws = ws or bsf.Workspace(bsf.backward_workspace_bytes(cfg, H, W), dev)
    gi, _ = bsf.filter_backward(cfg, ts, tg, want_steps=False, ws=ws)
    return gi.cpu().numpy(), ws


def test_small_upstream_gradient_keeps_its_bits():
    """The image gradient is linear in g and its fixed point follows the scale
    of g: a mean-style upstream gradient 2^-24 g gives exactly 2^-24 times the
    gradient of g (steps up to 48, as in the 4096^2 workload), and both match
    the FP64 oracle."""
    note("adjoint small g")
    d = WL.workload2(160, 176)
    img, steps = d["img"], d["steps"]
    g = np.random.default_rng(61).standard_normal(img.shape).astype(np.float32)
    gs = (g * np.float32(2.0 ** -24)).astype(np.float32)
    cfg = bsf.Config(order=2, max_step=d["max_step"])
    gi, _ = backward_only(cfg, steps, g)
    gi_s, _ = backward_only(cfg, steps, gs)
    np.testing.assert_array_equal(gi_s, (gi * np.float32(2.0 ** -24)).astype(np.float32))
    rgi, _ = O.grad_real(img, DIRS4, 2, True, steps, gs, want_steps=False)
    assert_grad_close(gi_s, rgi, what="grad_img, g scaled by 2^-24")


def tri(s, d):
    """Order-2 kernel of one direction at odd integer step s, offset d: the
    self-convolution of the length-s box, (s - |d|) / s^2 for |d| < s."""
    d = np.abs(d)
    return np.where(d < s, (s - d) / (s * s), 0.0)


def test_triangle_closed_form_is_the_oracle_factor():
    """Pins tri() to the oracle's factor weights: the convolution of two
    normalised boxes of step s."""
    for s in (1, 3, 7, 21, 101):
        i, w = O.weights_real(float(s))
        phi2 = np.convolve(w / s, w / s)
        dd = np.arange(-2 * i[-1], 2 * i[-1] + 1)
        np.testing.assert_allclose(phi2, tri(s, dd), rtol=0, atol=1e-15)


@pytest.mark.timeout(300)
def test_column_sum_headroom_adversarial():
    """Every pixel's axis steps just reach the centre column and row
    (s = 2 |x - c| + 1 along (1,0), 2 |y - c| + 1 along (0,1), diagonal steps 1),
    so their kernels pile up on the centre: with g = 1 the image gradient there
    is the column sum sum_x k_x(c - x) ~ 22, more than the 16 a fixed 3-bit
    margin allows.  The kernels are separable products of triangles, so the
    whole gradient is the outer product of two 1-D sums, compared at every
    pixel."""
    n, c = 2049, 1024
    S = float(2 * c + 1)
    note("adjoint adversarial column sums", n)
    off = np.abs(np.arange(n) - c)
    s_ax = (2 * off + 1).astype(np.float32)
    steps = np.ones((4, n, n), dtype=np.float32)
    steps[0] = s_ax[None, :]
    steps[1] = s_ax[:, None]
    g = np.ones((n, n), dtype=np.float32)
    # A[p] = sum_x tri(s(x), p - x): the same for rows and columns
    A = np.zeros(n)
    for x in range(n):
        s = int(s_ax[x])
        lo, hi = max(0, x - s + 1), min(n, x + s)
        A[lo:hi] += tri(s, np.arange(lo, hi) - x)
    ref = np.outer(A, A)
    assert ref[c, c] > 16.0
    cfg = bsf.Config(order=2, max_step=S)
    gi, ws = backward_only(cfg, steps, g)
    flags, _, _ = ws.status()
    assert flags == 0
    assert_grad_close(gi, ref, rel_norm=1e-6, rel_max=1e-6, what="adversarial grad_img")


def test_nonfinite_upstream_gradient():
    """A NaN or infinite upstream gradient raises FLAG_NONFINITE and makes the
    image gradient NaN; the next call with a finite gradient is clean again."""
    note("adjoint non-finite g")
    img, steps, g = case((24, 28), 4, 1.0, 7.0, 63)
    cfg = bsf.Config(order=2, max_step=7.0)
    bad = g.copy()
    bad[5, 6] = np.nan
    bad[9, 2] = np.inf
    gi, ws = backward_only(cfg, steps, bad)
    flags, _, _ = ws.status(clear=True)
    assert flags & bsf.FLAG_NONFINITE
    assert np.isnan(gi).all()
    gi2, _ = backward_only(cfg, steps, g, ws=ws)
    flags, _, _ = ws.status()
    assert flags == 0 and np.isfinite(gi2).all()
    rgi, _ = O.grad_real(img, DIRS4, 2, True, steps, g, want_steps=False)
    assert_grad_close(gi2, rgi, what="grad_img after a NaN call")


def test_checked_filter_raises_on_device_flags():
    note("checked filter")
    img, steps, g = case((20, 24), 4, 1.0, 6.0, 65)
    cfg = bsf.Config(order=2, max_step=6.0)
    dev = torch.device("cuda:0")
    steps[1, 3, 3] = np.nan
    ti = torch.from_numpy(img).to(dev).requires_grad_(True)
    ts = torch.from_numpy(steps).to(dev)
    with pytest.raises(bsf.DeviceFlagError):
        bsf.filter(ti, ts, cfg, check=True)
    steps[1, 3, 3] = 2.0
    out = bsf.filter(ti, torch.from_numpy(steps).to(dev), cfg, check=True)
    bad = torch.from_numpy(g).to(dev)
    bad[0, 0] = float("inf")
    with pytest.raises(bsf.DeviceFlagError):
        out.backward(bad)


@pytest.mark.timeout(600)
def test_differentiation_workload_every_image():
    """All 16 images of the differentiation workload (1024^2, steps in
    [1.5, 20], standard-normal upstream gradient), each through the forward
    and the adjoint as the benchmark runs them: the output, the step gradient
    and the image gradient on the 64 x 64 crop of every image against the FP64
    oracle."""
    d = WL.workload5()
    y0, y1, x0, x1 = d["fd_crop"]
    cfg = bsf.Config(order=2, max_step=20.0)
    m = 74   # reach of a step-20 order-2 kernel: 2 (R + 2) 3 + 8
    for b in range(len(d["imgs"])):
        note("workload 5 image", b)
        img, steps, g = d["imgs"][b], d["steps"][b], d["gout"][b]
        out, gi, gs, _ = gpu_grads(cfg, img, steps, g)
        H, W = img.shape
        ys, xs = np.mgrid[y0:y1, x0:x1]
        pix = (ys * W + xs).reshape(-1)
        ref = O.filter(img, DIRS4, 2, True, O.REAL, steps, pix=pix)
        np.testing.assert_allclose(out.reshape(-1)[pix], ref, rtol=2e-7, atol=2e-8)
        _, rgs = O.grad_real(img, DIRS4, 2, True, steps, g, pix=pix, want_img=False)
        assert_grad_close(gs.reshape(4, -1)[:, pix].T, rgs, what="grad_steps image %d" % b)
        rgi, _ = O.grad_real(img, DIRS4, 2, True, steps, g,
                             window=(max(0, x0 - m), min(W, x1 + m), max(0, y0 - m), min(H, y1 + m)),
                             want_steps=False)
        assert_grad_close(gi[y0:y1, x0:x1], rgi[y0:y1, x0:x1], what="grad_img image %d" % b)
