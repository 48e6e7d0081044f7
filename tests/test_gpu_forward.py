"""GPU parity of the forward path (pre-integration, taps, normalisation)
against the CPU oracle, through the C ABI.  Integer work is compared bit for
bit; FP32 outputs within the bound of gpu_util.float_tolerance."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1109_5114_amd as bsf
import workloads as WL
from tests.gpu_util import assert_close, cfg_of, note, run_forward

pytestmark = pytest.mark.gpu

DIRS4 = ((1, 0), (0, 1), (1, 1), (1, -1))


def sample_pixels(H, W, n, seed):
    rng = np.random.default_rng(seed)
    ys = list(rng.integers(0, H, n)) + [0, 0, H - 1, H - 1, H // 2, 0, H - 1]
    xs = list(rng.integers(0, W, n)) + [0, W - 1, 0, W - 1, W // 2, W // 2, W // 3]
    return np.array(ys) * W + np.array(xs)


# ----------------------------------------------------------------------------- pre-integration

@pytest.mark.parametrize("dtype,dirs,order,shape,F", [
    (np.uint8, DIRS4, 1, (37, 53), 0),
    (np.uint8, DIRS4, 2, (29, 41), 0),
    (np.float32, DIRS4, 2, (33, 47), 24),
    (np.float32, DIRS4, 1, (70, 1100), 30),          # rows longer than one 1024-element chunk
    (np.uint16, ((1, 0), (0, 1)), 3, (21, 19), 0),
    (np.uint8, ((1, 1), (2, 1), (1, -2)), 1, (31, 26), 0),
    (np.float32, ((0, 1), (1, 0), (1, 1), (1, -1)), 2, (150, 9), 20),   # tall: many line tiles
    (np.uint8, ((2, 1), (1, 2), (1, -2), (2, -1)), 2, (43, 57), 0),     # Alg. 3 directions
    (np.uint16, ((1, -2), (1, 0), (2, -1), (0, 1)), 1, (60, 35), 0),    # upward passes first
])
def test_preintegrate_bit_exact(dtype, dirs, order, shape, F):
    note("preintegrate", dtype.__name__, dirs, order, shape)
    rng = np.random.default_rng(hash((shape, order)) % 2 ** 32)
    if dtype == np.float32:
        img = rng.random(shape, dtype=np.float32)
    else:
        img = rng.integers(0, np.iinfo(dtype).max + 1, size=shape).astype(dtype)
    cfg = bsf.Config(dirs=dirs, order=order, mode=bsf.STEPS_REAL, max_step=7.0)
    G = bsf.preintegrate(cfg, torch.from_numpy(img).cuda(), F=F).cpu().numpy().view(np.uint64)
    g = bsf.plan(cfg, *shape)
    ref = O.preintegrate(img, dirs, order, F, (g.pad_top, g.pad_bottom, g.pad_left, g.pad_right))
    np.testing.assert_array_equal(G, ref)


# ----------------------------------------------------------------------------- integer steps

@pytest.mark.parametrize("shape", [(150, 170), (1, 37), (37, 1), (2, 2)])
def test_integer_steps_uint8_exact(shape):
    note("int u8", shape)
    d = WL.workload3(*shape)
    cfg = cfg_of(d)
    out, num, den, flags, F = run_forward(cfg, d["img"], d["steps"], want_num=True, want_den=True)
    ref, rnum, rden = O.filter(d["img"], d["dirs"], 1, True, O.INT, d["steps"], want_int=True)
    assert flags == 0
    np.testing.assert_array_equal(num, rnum)
    np.testing.assert_array_equal(den, rden)
    assert_close(out, ref, 0, quantised=False, what="int u8")


@pytest.mark.parametrize("shape", [(96, 112), (256, 256)])
def test_integer_steps_float_image(shape):
    note("int f32", shape)
    d = WL.workload1(*shape)
    cfg = cfg_of(d)
    out, _, den, flags, F = run_forward(cfg, d["img"], d["steps"], want_den=True)
    ref = O.filter(d["img"], d["dirs"], 1, True, O.INT, d["steps"])
    assert flags == 0 and F >= 24      # samples are multiples of 2^-24: exact fixed point
    assert_close(out, ref, F, quantised=False, what="int f32")


@pytest.mark.timeout(600)
def test_integer_steps_full_2048_uint8_every_pixel():
    """The 2048^2 uint8 integer-step workload: every int64 numerator and every
    denominator bit for bit against the oracle."""
    note("int u8 2048 full")
    d = WL.workload3()
    cfg = cfg_of(d)
    out, num, den, flags, F = run_forward(cfg, d["img"], d["steps"], want_num=True, want_den=True)
    assert flags == 0
    note("oracle on every pixel of 2048^2 with", O.num_threads(), "threads")
    ref, rnum, rden = O.filter(d["img"], d["dirs"], 1, True, O.INT, d["steps"], want_int=True)
    np.testing.assert_array_equal(num, rnum)
    np.testing.assert_array_equal(den, rden)
    assert_close(out, ref, 0, quantised=False, what="int u8 2048")


# ----------------------------------------------------------------------------- continuous steps

def rand_steps(shape, planes, lo, hi, seed):
    return np.random.default_rng(seed).uniform(lo, hi, size=(planes,) + shape).astype(np.float32)


@pytest.mark.parametrize("shape,hi", [((70, 90), 9.0), ((17, 5), 4.0)])
def test_continuous_order1(shape, hi):
    note("real order1", shape)
    img = np.random.default_rng(3).random(shape, dtype=np.float32)
    steps = rand_steps(shape, 4, 1.0, hi, 4)
    cfg = bsf.Config(order=1, max_step=hi)
    out, _, _, flags, F = run_forward(cfg, img, steps)
    ref = O.filter(img, DIRS4, 1, True, O.REAL, steps)
    assert flags == 0
    assert_close(out, ref, F, what="real order1")


@pytest.mark.parametrize("shape,lo,hi,smooth", [
    ((64, 72), 1.0, 12.0, False),     # independent steps per pixel: lanes disagree on R
    ((50, 61), 1.0, 20.0, True),
    ((3, 40), 1.0, 6.0, False),
])
def test_continuous_tied_order2(shape, lo, hi, smooth):
    note("real tied order2", shape, smooth)
    rng = np.random.default_rng(5)
    img = rng.random(shape, dtype=np.float32)
    if smooth:
        steps = np.stack([WL.smooth(rng, *shape, lo, hi) for _ in range(4)]).astype(np.float32)
    else:
        steps = rand_steps(shape, 4, lo, hi, 6)
    cfg = bsf.Config(order=2, max_step=hi)
    out, _, _, flags, F = run_forward(cfg, img, steps)
    ref = O.filter(img, DIRS4, 2, True, O.REAL, steps)
    assert flags == 0
    assert_close(out, ref, F, what="real tied order2")


BETA2 = ((2, 1), (1, 2), (1, -2), (2, -1))


@pytest.mark.parametrize("order,mode,shape,hi", [
    (1, "int", (41, 47), 9.0),
    (2, "int", (23, 29), 5.0),
    (1, "real", (52, 38), 11.0),
    (2, "real", (37, 45), 9.0),
])
def test_alg3_directions(order, mode, shape, hi):
    """The directions of Alg. 3 and Table 1, (2,1), (1,2), (-1,2), (-2,1) in
    canonical sign, two of them upward: integer numerators bit for bit, float
    outputs within the fixed-point bound."""
    note("alg3 directions", order, mode, shape)
    rng = np.random.default_rng(30 + order)
    cfg = bsf.Config(dirs=BETA2, order=order, mode=bsf.STEPS_INT if mode == "int" else bsf.STEPS_REAL,
                     max_step=hi)
    if mode == "int":
        img = rng.integers(0, 256, size=shape).astype(np.uint8)
        steps = rng.integers(1, int(hi) + 1, size=(4,) + shape).astype(np.float32)
        out, num, den, flags, F = run_forward(cfg, img, steps, want_num=True, want_den=True)
        ref, rnum, rden = O.filter(img, BETA2, order, True, O.INT, steps, want_int=True)
        np.testing.assert_array_equal(num, rnum)
        np.testing.assert_array_equal(den, rden)
    else:
        img = rng.random(shape, dtype=np.float32)
        steps = np.stack([WL.smooth(rng, *shape, 1.0, hi) for _ in range(4)]).astype(np.float32)
        out, _, _, flags, F = run_forward(cfg, img, steps)
        ref = O.filter(img, BETA2, order, True, O.REAL, steps)
    assert flags == 0
    assert_close(out, ref, F, quantised=mode != "int", what="alg3 directions")


@pytest.mark.parametrize("shape,hi,smooth", [
    ((96, 112), 14.0, True),     # most tiles take the cluster boxes
    ((61, 77), 12.0, False),     # independent steps: most tiles read the window directly
    ((9, 200), 6.0, True),       # one ragged row of tiles
    ((40, 33), 3.0, False),      # small steps, every tile fits
    ((1, 1), 4.0, False),        # one pixel
    ((5, 3), 7.0, False),        # smaller than one tile
])
def test_table1_directions_tied_order2_every_pixel(shape, hi, smooth):
    """The tied order-2 cluster-box kernel in the frame of Table 1's
    directions, given in another order than its own frame: every pixel against
    the oracle (tiles whose step range does not fit the LDS boxes read the
    window directly)."""
    note("table1 cluster boxes", shape, smooth)
    dirs = ((1, -2), (2, 1), (2, -1), (1, 2))
    rng = np.random.default_rng(60 + shape[0])
    img = rng.random(shape, dtype=np.float32)
    if smooth:
        steps = np.stack([WL.smooth(rng, *shape, 1.0, hi) for _ in range(4)]).astype(np.float32)
    else:
        steps = rand_steps(shape, 4, 1.0, hi, 61)
    cfg = bsf.Config(dirs=dirs, order=2, max_step=hi)
    out, _, _, flags, F = run_forward(cfg, img, steps)
    ref = O.filter(img, dirs, 2, True, O.REAL, steps)
    assert flags == 0
    assert_close(out, ref, F, what="table1 tied order2")


def test_continuous_untied_order2_generic():
    note("real untied order2")
    shape = (12, 14)
    img = np.random.default_rng(8).random(shape, dtype=np.float32)
    steps = rand_steps(shape, 8, 1.0, 3.5, 9)
    cfg = bsf.Config(order=2, tied=False, max_step=3.5)
    out, _, _, flags, F = run_forward(cfg, img, steps)
    ref = O.filter(img, DIRS4, 2, False, O.REAL, steps)
    assert_close(out, ref, F, what="real untied order2")


@pytest.mark.timeout(900)
def test_full_4096_order2_every_pixel():
    """The 4096^2 order-2 workload (continuous steps up to 48) exactly as the
    benchmark runs it, every one of its 16.8 M outputs against the FP64 oracle
    (border tiles and tiles that fall back to direct window reads included)."""
    note("real tied order2 4096 full")
    d = WL.workload2()
    cfg = cfg_of(d)
    out, _, _, flags, F = run_forward(cfg, d["img"], d["steps"])
    assert flags == 0
    assert np.isfinite(out).all()
    note("oracle on every pixel, F =", F, "threads", O.num_threads())
    ref = O.filter(d["img"], d["dirs"], 2, True, O.REAL, d["steps"])
    rel = assert_close(out, ref, F, what="4096 order2")
    note("max rel err vs oracle", rel)


# ----------------------------------------------------------------------------- status and edges

def test_status_flags_for_bad_steps():
    note("status flags")
    shape = (20, 24)
    img = np.random.default_rng(12).random(shape, dtype=np.float32)
    steps = rand_steps(shape, 4, 1.0, 5.0, 13)
    steps[0, 3, 4] = np.nan
    steps[2, 10, 11] = 99.0          # above max_step
    steps[1, 0, 0] = 0.25            # below 1
    cfg = bsf.Config(order=2, max_step=5.0)
    out, _, _, flags, F = run_forward(cfg, img, steps)
    assert flags & bsf.FLAG_RANGE
    assert np.isfinite(out).all()


def test_explicit_frac_bits_overflow_flag():
    note("overflow flag")
    shape = (16, 16)
    img = np.random.default_rng(14).random(shape, dtype=np.float32)
    steps = rand_steps(shape, 4, 30.0, 31.0, 15)
    cfg = bsf.Config(order=2, max_step=31.0, frac_bits=40)   # 40 + 1 + 8*5 bits > 62
    _, _, _, flags, F = run_forward(cfg, img, steps)
    assert F == 40 and flags & bsf.FLAG_OVERFLOW


def test_tiny_image_keeps_its_bits():
    """F is not capped at 62: an image scaled by 2^-60 gets F larger by 60, the
    same fixed-point integers and exactly the scaled output."""
    note("tiny image F > 62")
    shape = (30, 34)
    rng = np.random.default_rng(24)
    img = rng.random(shape, dtype=np.float32)
    steps = rand_steps(shape, 4, 1.0, 9.0, 25)
    cfg = bsf.Config(order=2, max_step=9.0)
    out, _, _, flags, F = run_forward(cfg, img, steps)
    small = (img * np.float32(2.0 ** -60)).astype(np.float32)
    out_s, _, _, flags_s, F_s = run_forward(cfg, small, steps)
    assert flags == 0 and flags_s == 0
    assert F_s == F + 60 and F_s > 62
    np.testing.assert_array_equal(out_s, (out * np.float32(2.0 ** -60)).astype(np.float32))


def test_huge_image_negative_F():
    """An image of magnitude 2^100 gets a negative F (coarser fixed point)
    instead of an overflow, and stays within the quantisation bound."""
    note("huge image F < 0")
    shape = (26, 31)
    rng = np.random.default_rng(26)
    img = (rng.random(shape, dtype=np.float32) * np.float32(2.0 ** 100)).astype(np.float32)
    steps = rand_steps(shape, 4, 1.0, 12.0, 27)
    cfg = bsf.Config(order=2, max_step=12.0)
    out, _, _, flags, F = run_forward(cfg, img, steps)
    assert flags == 0 and F < 0
    ref = O.filter(img, DIRS4, 2, True, O.REAL, steps)
    assert_close(out, ref, F, what="huge image")


def test_nonfinite_image_sample_is_flagged():
    """A NaN or infinite sample raises FLAG_NONFINITE; the choice of F ignores
    such samples (run_forward checks it against the documented rule)."""
    note("non-finite image")
    shape = (20, 22)
    img = np.random.default_rng(28).random(shape, dtype=np.float32)
    img[4, 5] = np.inf
    img[7, 1] = np.nan
    steps = rand_steps(shape, 4, 1.0, 5.0, 29)
    cfg = bsf.Config(order=2, max_step=5.0)
    _, _, _, flags, F = run_forward(cfg, img, steps)
    assert flags & bsf.FLAG_NONFINITE and not flags & bsf.FLAG_RANGE


def test_empty_image_is_a_no_op():
    note("empty")
    cfg = bsf.Config(order=2, max_step=5.0)
    img = torch.zeros((0, 7), device="cuda")
    steps = torch.zeros((4, 0, 7), device="cuda")
    out = bsf.filter_varying(cfg, img, steps)
    assert out.shape == (0, 7)


def test_deterministic_bits():
    note("determinism")
    shape = (40, 44)
    img = np.random.default_rng(16).random(shape, dtype=np.float32)
    steps = rand_steps(shape, 4, 1.0, 9.0, 17)
    cfg = bsf.Config(order=2, max_step=9.0)
    a = run_forward(cfg, img, steps)[0]
    b = run_forward(cfg, img, steps)[0]
    np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))


def test_plain_fp64_path_small_case_is_accurate():
    """The plain FP64 path is exact enough on a tiny window at order 1 (its
    cancellation error grows with the window and the order)."""
    note("fp64 plain small")
    shape = (20, 24)
    img = np.random.default_rng(18).random(shape, dtype=np.float32)
    steps = rand_steps(shape, 4, 1.0, 4.0, 19)
    cfg = bsf.Config(order=1, max_step=4.0, arith=bsf.ARITH_FP64)
    out, _, _, flags, F = run_forward(cfg, img, steps)
    ref = O.filter(img, DIRS4, 1, True, O.REAL, steps)
    assert np.abs(out - ref).max() < 1e-5


def test_prepare_then_apply_with_other_steps():
    """One pre-integration serves several step fields (the two banks of Alg. 2
    share a running sum per bank): apply(steps2) on the window built with steps1
    equals the one-call filter with steps2."""
    note("prepare/apply")
    shape = (45, 51)
    rng = np.random.default_rng(20)
    img = rng.random(shape, dtype=np.float32)
    s1 = rand_steps(shape, 4, 1.0, 8.0, 21)
    s2 = rand_steps(shape, 4, 1.0, 8.0, 22)
    cfg = bsf.Config(order=2, max_step=8.0, frac_bits=24)
    dev = torch.device("cuda:0")
    ti, t1, t2 = (torch.from_numpy(a).to(dev) for a in (img, s1, s2))
    ws = bsf.Workspace(bsf.plan(cfg, *shape).workspace_bytes, dev)
    bsf.forward_prepare(cfg, ti, t1, ws)
    out = torch.empty(shape, dtype=torch.float32, device=dev)
    bsf.forward_apply(cfg, bsf.F32, t2, ws, out)
    flags, F, _ = ws.status()
    ref = bsf.filter_varying(cfg, ti, t2)
    assert flags == 0 and F == 24
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), ref.cpu().numpy().view(np.uint32))
    oref = O.filter(img, DIRS4, 2, True, O.REAL, s2)
    assert_close(out.cpu().numpy(), oref, F, what="prepare/apply")


def test_apply_checks_its_own_steps():
    """forward_apply with steps other than the prepared ones: the taps raise
    FLAG_RANGE for a bad step and FLAG_OVERFLOW when the new steps' box
    lengths exceed the headroom of the F chosen for the prepared steps."""
    note("apply-time checks")
    shape = (40, 44)
    rng = np.random.default_rng(32)
    img = rng.random(shape, dtype=np.float32)
    small = rand_steps(shape, 4, 1.0, 2.0, 33)            # F chosen for box lengths 3
    large = rand_steps(shape, 4, 30.0, 31.0, 34)          # lengths 31: 8 * 5 bits more
    cfg = bsf.Config(order=2, max_step=31.0)
    dev = torch.device("cuda:0")
    ti, ts, tl = (torch.from_numpy(a).to(dev) for a in (img, small, large))
    ws = bsf.Workspace(bsf.plan(cfg, *shape).workspace_bytes, dev)
    out = torch.empty(shape, dtype=torch.float32, device=dev)
    bsf.forward_prepare(cfg, ti, ts, ws)
    bsf.forward_apply(cfg, bsf.F32, ts, ws, out)
    flags, F, _ = ws.status()
    assert flags == 0
    bsf.forward_apply(cfg, bsf.F32, tl, ws, out)
    flags, _, _ = ws.status(clear=True)
    assert flags & bsf.FLAG_OVERFLOW and not flags & bsf.FLAG_RANGE
    bad = small.copy()
    bad[3, 5, 6] = np.nan
    bsf.forward_apply(cfg, bsf.F32, torch.from_numpy(bad).to(dev), ws, out)
    flags, _, _ = ws.status(clear=True)
    assert flags & bsf.FLAG_RANGE
