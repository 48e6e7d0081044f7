"""GPU parity of Alg. 1 (isotropic pre-filter of half the condition2 bound,
then the space-variant filter of C - sigma^2 I) and Alg. 2 (two four-direction
box splines chosen per pixel by orientation sector) against the same
algorithms written out with the oracle's pieces."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1109_5114_amd as bsf
import workloads as WL
from tests.gpu_util import note
from tests.test_gpu_cov import cov_field

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def read_status(ws):
    flags, F, _ = ws.status()
    words = ws.buf[:256].cpu().numpy().view(np.int32)
    return flags, F, words


@pytest.mark.parametrize("order", [1, 2])
def test_alg2_matches_oracle(order):
    note("alg2 order", order)
    rng = np.random.default_rng(400 + order)
    H, W = 90, 118
    img = rng.random((H, W), dtype=np.float32)
    cov = cov_field(rng, H, W, rho_max=5.0, bank=2)
    cfg = bsf.Config(order=order, max_step=80.0)
    ws = bsf.Workspace(bsf.lib().bsf_alg2_workspace_bytes(bsf.ctypes.byref(cfg.c()), H, W), DEV)
    bank = torch.empty((H, W), dtype=torch.uint8, device=DEV)
    out = bsf.filter_alg2(cfg, to_dev(img), to_dev(cov), bank=bank, ws=ws).cpu().numpy()
    flags, F, _ = read_status(ws)
    banks = O.alg2_banks(cov)
    np.testing.assert_array_equal(bank.cpu().numpy(), banks)
    assert 0.2 < banks.mean() < 0.8              # both sectors are used
    # the composition, with the steps bsf_cov_to_steps gives for each set
    s1 = bsf.cov_to_steps(bsf.Config(dirs=O.BANK1, order=order, max_step=80.0), to_dev(cov)).cpu().numpy()
    s2 = bsf.cov_to_steps(bsf.Config(dirs=O.BANK2, order=order, max_step=80.0), to_dev(cov)).cpu().numpy()
    ref, _ = O.alg2(img, cov, order, steps=(s1, s2))
    tol = 2.0 ** -(F + 1) + 2.0 ** -24 * np.abs(ref) * 1.01 + 1e-13
    err = np.abs(out.astype(np.float64) - ref)
    assert (err <= tol).all(), (err.max(), np.argmax(err - tol))
    # end to end against the oracle's own steps (the minimum-kurtosis scales
    # agree to a few float roundings)
    ref2, _ = O.alg2(img, cov, order)
    assert np.abs(out - ref2).max() <= 1e-5 * np.abs(ref2).max()
    assert flags & ~bsf.FLAG_RANGE == 0


@pytest.mark.parametrize("order", [1, 2])
def test_alg1_matches_oracle(order):
    note("alg1 order", order)
    rng = np.random.default_rng(410 + order)
    H, W = 84, 101
    img = rng.random((H, W), dtype=np.float32)
    # moderate elongations and sizes >= 4 px: the isotropic part is sizeable
    cov = cov_field(rng, H, W, rho_max=2.5, sig=(4.0, 12.0))
    cfg = bsf.Config(order=order, max_step=80.0)
    ws = bsf.Workspace(bsf.lib().bsf_alg1_workspace_bytes(bsf.ctypes.byref(cfg.c()), H, W), DEV)
    out = bsf.filter_alg1(cfg, to_dev(img), to_dev(cov), ws=ws).cpu().numpy()
    flags, F, words = read_status(ws)
    assert flags == 0
    sigma2 = float(words[25:26].view(np.float32)[0])
    _, rs2, _, _ = O.alg1(img[:2, :2], cov[:, :2, :2], order)   # exercise the oracle's own sigma^2 path
    b = np.array([O.condition2_bound(*cov[:, y, x]) for y in range(H) for x in range(W)])
    np.testing.assert_allclose(sigma2, 0.5 * max(b.min(), 0.0), rtol=1e-6)
    assert sigma2 > 1.0
    s2 = bsf.cov_to_steps(bsf.Config(order=order, max_step=80.0), to_dev(cov), sub=sigma2).cpu().numpy()
    ref, _, _, _ = O.alg1(img, cov, order, sigma2=sigma2, steps2=s2)
    # two fixed-point passes (F of the second reported) and the FP32 rounding
    # of the first pass's output, which the second pass averages
    tol = 2.0 ** -(F + 1) * 2 + 2.0 ** -23 * np.abs(ref) * 1.01 + 2.0 ** -24
    err = np.abs(out.astype(np.float64) - ref)
    assert (err <= tol).all(), (err.max(), tol.min())
    ref2, _, _, _ = O.alg1(img, cov, order)
    assert np.abs(out - ref2).max() <= 1e-5 * np.abs(ref2).max()


def test_alg1_is_one_filter_of_covariance_C():
    """Prop. 1 and 2: the two passes of Alg. 1 on an impulse give a kernel
    with the covariance of the isotropic pass plus that of the pixel's own
    kernel; for a constant covariance field, the sum is C (up to the discrete
    cell-integration term of continuous steps, which both passes share)."""
    note("alg1 impulse covariance")
    H = W = 97
    img = np.zeros((H, W), np.float32)
    img[48, 48] = 1.0
    C = np.array([[30.0, 9.0], [9.0, 14.0]])
    cov = np.zeros((3, H, W), np.float32)
    cov[0], cov[1], cov[2] = C[0, 0], C[0, 1], C[1, 1]
    cfg = bsf.Config(order=1, max_step=80.0)
    out = bsf.filter_alg1(cfg, to_dev(img), to_dev(cov)).cpu().numpy().astype(np.float64)
    assert abs(out.sum() - 1.0) < 1e-5
    ys, xs = np.mgrid[0:H, 0:W] - 48.0
    m = np.array([[(out * xs * xs).sum(), (out * xs * ys).sum()], [(out * xs * ys).sum(), (out * ys * ys).sum()]])
    # the filter reads f(x + d): its impulse response is the kernel mirrored,
    # whose covariance is the same; each continuous box adds the unit-cell
    # term (1 - lambda)lambda-type excess, below 1/4 per direction and pass
    assert np.abs(m - C).max() < 1.5, (m, C)


@pytest.mark.parametrize("order", [1, 2])
def test_alg2_full_size_sampled(order):
    """Alg. 2 on the 4096 x 4096 covariance-field workload (orientation,
    elongation 1-6 and size 2-12 px from smooth fields): the sector of
    sampled pixels against the oracle's rule, and sampled outputs against the
    oracle's filter of the sector's direction set on crops that hold each
    pixel's footprint (outside it the filter reads nothing), with the steps
    bsf_cov_to_steps gives for that set.  At order 2 the taps of both sets come
    from their cluster-box kernels (and the direct reads of tiles whose boxes
    do not fit)."""
    d = WL.workload_alg3()
    img, cov = d["img"], d["cov"]
    H, W = img.shape
    note("alg2 full size order", order, H, W)
    tcov = to_dev(cov)
    smax = 1.0
    for dirs in (O.BANK1, O.BANK2):
        probe = bsf.Config(dirs=dirs, order=order, max_step=1e5)
        smax = max(smax, float(bsf.cov_to_steps(probe, tcov).max().item()))
    cfg = bsf.Config(order=order, max_step=float(np.ceil(smax)))
    ws = bsf.Workspace(bsf.lib().bsf_alg2_workspace_bytes(bsf.ctypes.byref(cfg.c()), H, W), DEV)
    bank = torch.empty((H, W), dtype=torch.uint8, device=DEV)
    out = bsf.filter_alg2(cfg, to_dev(img), tcov, bank=bank, ws=ws).cpu().numpy()
    flags, F, _ = read_status(ws)
    assert flags & ~bsf.FLAG_RANGE == 0
    assert np.isfinite(out).all()
    bank = bank.cpu().numpy()
    rng = np.random.default_rng(450 + order)
    ys, xs = rng.integers(0, H, 3000), rng.integers(0, W, 3000)
    want = [O.bank_of(O.orientation(float(cov[0, y, x]), float(cov[1, y, x]), float(cov[2, y, x])))
            for y, x in zip(ys, xs)]
    np.testing.assert_array_equal(bank[ys, xs], np.array(want, np.uint8))
    assert 0.2 < bank.mean() < 0.8
    # the steps each set's filter uses (clamped to [1, max_step] as the kernels do)
    steps = []
    for dirs in (O.BANK1, O.BANK2):
        st = bsf.cov_to_steps(bsf.Config(dirs=dirs, order=order, max_step=cfg.max_step), tcov).cpu().numpy()
        steps.append(np.where(np.isfinite(st), np.clip(st, 1.0, cfg.max_step), 1.0).astype(np.float32))
    pts = [(0, 0), (W - 1, H - 1), (0, H - 1), (W - 1, 0)] + [tuple(p) for p in rng.integers(0, [W, H], (40, 2))]
    for x, y in pts:
        b = int(bank[y, x])
        dirs, st = (O.BANK1, O.BANK2)[b], steps[b]
        R = np.floor((st[:, y, x].astype(np.float64) - 1.0) / 2.0)
        rx = int(sum(order * (r + 2) * abs(u[0]) for u, r in zip(dirs, R))) + 2
        ry = int(sum(order * (r + 2) * abs(u[1]) for u, r in zip(dirs, R))) + 2
        x0, x1, y0, y1 = max(0, x - rx), min(W, x + rx + 1), max(0, y - ry), min(H, y + ry + 1)
        crop = np.ascontiguousarray(img[y0:y1, x0:x1])
        cst = np.ascontiguousarray(st[:, y0:y1, x0:x1])
        ref = O.filter(crop, dirs, order, True, O.REAL, cst, pix=np.array([(y - y0) * (x1 - x0) + (x - x0)]))[0]
        tol = 2.0 ** -(F + 1) + 2.0 ** -24 * abs(ref) * 1.01 + 1e-13
        assert abs(float(out[y, x]) - ref) <= tol, (x, y, b, float(out[y, x]), ref, tol)


def test_alg2_in_a_captured_graph():
    """Alg. 2 runs its second direction set on a side stream, forked from and
    joined back into the caller's stream by events: captured into a graph on
    the caller's stream, every replay (with eager work between them) gives
    the eager call's output and sectors."""
    note("alg2 graph capture")
    rng = np.random.default_rng(470)
    H, W = 64, 80
    img = to_dev(rng.random((H, W), dtype=np.float32))
    cov = to_dev(cov_field(rng, H, W, rho_max=5.0, bank=2))
    cfg = bsf.Config(order=2, max_step=80.0)
    ws = bsf.Workspace(bsf.lib().bsf_alg2_workspace_bytes(bsf.ctypes.byref(cfg.c()), H, W), DEV)
    out = torch.empty((H, W), dtype=torch.float32, device=DEV)
    bank = torch.empty((H, W), dtype=torch.uint8, device=DEV)
    bsf.filter_alg2(cfg, img, cov, out=out, bank=bank, ws=ws)   # eager: also makes the side stream
    torch.cuda.synchronize()
    ref, ref_bank = out.clone(), bank.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bsf.filter_alg2(cfg, img, cov, out=out, bank=bank, ws=ws)
    for rep in range(3):
        out.fill_(-1.0)
        bank.fill_(7)
        junk = torch.randn(256, 256, device=DEV) @ torch.randn(256, 256, device=DEV)   # eager work between
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
        assert torch.equal(bank, ref_bank), rep
    del junk
