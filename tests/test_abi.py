"""Host-side checks of the C ABI: the library loads, exports every entry point
include/bsf.h declares, and validates arguments before touching a device.
No compute call runs here."""
import ctypes
import os
import re

import pytest

import paper_1109_5114_amd as bsf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "bsf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bsf_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = bsf.lib()
    names = header_functions()
    assert "bsf_filter_varying" in names and "bsf_filter_backward" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(bsf.EXPORTS)


def test_version_and_status_strings():
    assert "gfx950" in bsf.version()
    for code in range(7):
        assert bsf.status_string(code)


def geo(cfg, H=64, W=80):
    return bsf.plan(cfg, H, W)


def test_plan_window_covers_every_tap():
    cfg = bsf.Config(order=2, max_step=15.0)
    g = geo(cfg)
    R = 7
    # per direction the taps reach [-r(R+2), r(R+1)] lattice steps
    assert g.pad_left == 2 * (R + 2) * 3            # three directions with dx = 1
    assert g.pad_right >= 2 * (R + 1) * 3
    assert g.pad_top == 2 * (R + 2) * 2 + 2 * (R + 1)   # (0,1), (1,1) down; (1,-1) up
    assert g.pad_bottom == 2 * (R + 1) * 2 + 2 * (R + 2)
    assert g.win_w % 16 == 0
    assert g.win_h == 64 + g.pad_top + g.pad_bottom
    assert g.g_bytes == g.win_h * g.win_w * 8
    assert g.workspace_bytes >= g.g_bytes + g.workspace_bytes_g_external


@pytest.mark.parametrize("dirs", [
    ((0, 0),),                      # zero vector
    ((2, 0),),                      # not primitive
    ((2, 4), (1, 0)),               # not primitive
    ((-1, 1),),                     # not canonical sign
    ((0, -1),),                     # not canonical sign
    ((1, 0), (0, 1), (1, 0)),       # a direction twice
])
def test_plan_rejects_bad_directions(dirs):
    """Zero, non-primitive, non-canonical or repeated directions are refused
    before anything runs."""
    with pytest.raises(bsf.BsfError) as e:
        geo(bsf.Config(dirs=dirs))
    assert e.value.code == bsf.E_INVALID


@pytest.mark.parametrize("kw,code", [
    (dict(order=0), bsf.E_INVALID),
    (dict(order=5), bsf.E_UNSUPPORTED),
    (dict(order=4, dirs=((1, 0), (0, 1), (1, 1), (1, -1), (2, 1))), bsf.E_INVALID),   # M = 20 > 16
    (dict(max_step=0.5), bsf.E_INVALID),
    (dict(max_step=float("nan")), bsf.E_INVALID),
    (dict(frac_bits=63), bsf.E_INVALID),
    (dict(mode=7), bsf.E_INVALID),
    (dict(arith=3), bsf.E_INVALID),
])
def test_plan_rejects_bad_config(kw, code):
    with pytest.raises(bsf.BsfError) as e:
        geo(bsf.Config(**kw))
    assert e.value.code == code


def test_plan_rejects_bad_sizes():
    with pytest.raises(bsf.BsfError):
        bsf.plan(bsf.Config(), -1, 5)
    g = bsf.plan(bsf.Config(), 0, 0)     # empty image is valid
    assert g.win_h == g.pad_top + g.pad_bottom


def test_entry_points_validate_before_launch():
    """Argument errors return before anything is enqueued (null pointers are
    never dereferenced, so this runs without a device)."""
    L = bsf.lib()
    cfg = bsf.Config().c()
    NULL = None
    # pitch < W
    r = L.bsf_filter_varying(ctypes.byref(cfg), bsf.F32, ctypes.c_void_p(16), 8, 8, 4, ctypes.c_void_p(16),
                             ctypes.c_void_p(16), NULL, NULL, NULL, NULL, ctypes.c_void_p(16), 1 << 30, NULL)
    assert r == bsf.E_INVALID
    # workspace too small
    r = L.bsf_filter_varying(ctypes.byref(cfg), bsf.F32, ctypes.c_void_p(16), 8, 8, 8, ctypes.c_void_p(16),
                             ctypes.c_void_p(16), NULL, NULL, NULL, NULL, ctypes.c_void_p(16), 16, NULL)
    assert r == bsf.E_WORKSPACE
    # bad dtype
    r = L.bsf_filter_varying(ctypes.byref(cfg), 9, ctypes.c_void_p(16), 8, 8, 8, ctypes.c_void_p(16),
                             ctypes.c_void_p(16), NULL, NULL, NULL, NULL, ctypes.c_void_p(16), 1 << 30, NULL)
    assert r == bsf.E_INVALID
    # numerator output only in integer mode
    r = L.bsf_filter_varying(ctypes.byref(cfg), bsf.U8, ctypes.c_void_p(16), 8, 8, 8, ctypes.c_void_p(16),
                             ctypes.c_void_p(16), ctypes.c_void_p(16), NULL, NULL, NULL, ctypes.c_void_p(16),
                             1 << 30, NULL)
    assert r == bsf.E_INVALID
    # preintegrate: F out of range, null G
    r = L.bsf_preintegrate(ctypes.byref(cfg), bsf.F32, ctypes.c_void_p(16), 8, 8, 8, 63, ctypes.c_void_p(16),
                           ctypes.c_void_p(16), 1 << 30, NULL)
    assert r == bsf.E_INVALID
    r = L.bsf_preintegrate(ctypes.byref(cfg), bsf.F32, ctypes.c_void_p(16), 8, 8, 8, 24, NULL,
                           ctypes.c_void_p(16), 1 << 30, NULL)
    assert r == bsf.E_INVALID
    r = L.bsf_workspace_init(ctypes.c_void_p(16), 8, NULL)
    assert r == bsf.E_WORKSPACE
    # derivative output only with continuous steps
    icfg = bsf.Config(mode=bsf.STEPS_INT).c()
    r = L.bsf_filter_varying(ctypes.byref(icfg), bsf.F32, ctypes.c_void_p(16), 8, 8, 8, ctypes.c_void_p(16),
                             ctypes.c_void_p(16), NULL, NULL, ctypes.c_void_p(16), NULL, ctypes.c_void_p(16),
                             1 << 30, NULL)
    assert r == bsf.E_INVALID
    # backward: step gradient needs the saved derivative; integer steps are not differentiable
    r = L.bsf_filter_backward(ctypes.byref(cfg), 8, 8, ctypes.c_void_p(16), ctypes.c_void_p(16), NULL, NULL,
                              ctypes.c_void_p(16), ctypes.c_void_p(16), 1 << 30, NULL)
    assert r == bsf.E_INVALID
    r = L.bsf_filter_backward(ctypes.byref(icfg), 8, 8, ctypes.c_void_p(16), ctypes.c_void_p(16), NULL,
                              ctypes.c_void_p(16), NULL, ctypes.c_void_p(16), 1 << 30, NULL)
    assert r == bsf.E_UNSUPPORTED
    r = L.bsf_filter_backward(ctypes.byref(cfg), 8, 8, ctypes.c_void_p(16), ctypes.c_void_p(16), NULL,
                              ctypes.c_void_p(16), NULL, ctypes.c_void_p(16), 64, NULL)
    assert r == bsf.E_WORKSPACE


def test_tuning_setter_validates_and_round_trips():
    L = bsf.lib()
    wx0, tl0 = bsf.get_tuning()
    assert (wx0, tl0) == (16, 64)
    try:
        for wx, tl in ((8, 16), (32, 256), (64, 4096)):
            bsf.set_tuning(wx, tl)
            assert bsf.get_tuning() == (wx, tl)
        for wx, tl in ((12, 64), (0, 64), (16, 8), (16, 96), (16, 8192)):
            assert L.bsf_set_tuning(wx, tl) == bsf.E_INVALID
            assert bsf.get_tuning() == (64, 4096)          # unchanged
        # the carries of the sheared scans scale with the tile count
        cfg = bsf.Config(order=2, max_step=9.0)
        bsf.set_tuning(16, 16)
        small_tiles = geo(cfg, 512, 512).workspace_bytes
        bsf.set_tuning(16, 512)
        big_tiles = geo(cfg, 512, 512).workspace_bytes
        assert small_tiles > big_tiles
    finally:
        bsf.set_tuning(wx0, tl0)


def _descs(shapes, fake=0x1000):
    arr = (bsf._ImageDesc * max(len(shapes), 1))()
    for b, (H, W) in enumerate(shapes):
        d = arr[b]
        d.img = d.steps = d.out = fake if H * W else 0
        d.H, d.W, d.pitch = H, W, W
    return arr


def test_batched_workspace_is_the_sum_of_image_workspaces():
    L = bsf.lib()
    cfg = bsf.Config(order=2, max_step=9.0)
    c = cfg.c()
    shapes = [(40, 52), (0, 7), (128, 96), (17, 1)]
    total = L.bsf_batched_workspace_bytes(ctypes.byref(c), len(shapes), _descs(shapes))
    per_image = sum((geo(cfg, H, W).workspace_bytes + 255) // 256 * 256 for H, W in shapes)
    # batch status block + launch tables + one single-image workspace per image
    assert total > per_image + 256
    assert total - per_image - 256 < 64 * 1024
    one = L.bsf_batched_workspace_bytes(ctypes.byref(c), 1, _descs(shapes[:1]))
    assert one < total
    assert L.bsf_batched_workspace_bytes(ctypes.byref(c), 0, None) > 0


def test_batched_entry_point_validates_before_launch():
    L = bsf.lib()
    cfg = bsf.Config(order=2, max_step=9.0)
    c = cfg.c()
    shapes = [(40, 52), (30, 31)]
    d = _descs(shapes)
    need = L.bsf_batched_workspace_bytes(ctypes.byref(c), 2, d)
    ws = ctypes.c_void_p(0x100000)
    # invalid count, missing descriptors, missing workspace
    assert L.bsf_batched_workspace_bytes(ctypes.byref(c), -1, d) == 0
    assert L.bsf_filter_batched(ctypes.byref(c), -1, d, ws, need, None, 0) == bsf.E_INVALID
    assert L.bsf_filter_batched(ctypes.byref(c), 2, None, ws, need, None, 0) == bsf.E_INVALID
    assert L.bsf_filter_batched(ctypes.byref(c), 2, d, None, need, None, 0) == bsf.E_INVALID
    # a NULL pointer or a short pitch on a non-empty image
    bad = _descs(shapes)
    bad[1].out = 0
    assert L.bsf_filter_batched(ctypes.byref(c), 2, bad, ws, need, None, 0) == bsf.E_INVALID
    bad = _descs(shapes)
    bad[0].pitch = 51
    assert L.bsf_filter_batched(ctypes.byref(c), 2, bad, ws, need, None, 0) == bsf.E_INVALID
    # an image too large for the plan, and a bad configuration
    big = _descs([(40, 52), (1 << 19, 4)])
    assert L.bsf_filter_batched(ctypes.byref(c), 2, big, ws, need, None, 0) == bsf.E_INVALID
    c_bad = bsf.Config(order=5).c()
    assert L.bsf_filter_batched(ctypes.byref(c_bad), 2, d, ws, need, None, 0) == bsf.E_UNSUPPORTED
    # workspace one byte short
    assert L.bsf_filter_batched(ctypes.byref(c), 2, d, ws, need - 1, None, 0) == bsf.E_WORKSPACE


def test_noalloc_entry_point_rejects_oversize_before_any_launch():
    """bsf_filter_varying_noalloc checks its static scratch limit on the host
    (no device call is reached for an oversize request)."""
    L = bsf.lib()
    cfg = bsf.Config(order=2, max_step=48.0)
    assert bsf.plan(cfg, 4096, 4096).workspace_bytes > bsf.NOALLOC_SCRATCH_BYTES
    rc = L.bsf_filter_varying_noalloc(ctypes.byref(cfg.c()), bsf.F32, None, 4096, 4096, 4096, None, None, None,
                                      None, None, None, None)
    assert rc == bsf.E_WORKSPACE
    rc = L.bsf_filter_varying_noalloc(ctypes.byref(bsf.Config(order=0).c()), bsf.F32, None, 8, 8, 8, None, None,
                                      None, None, None, None, None)
    assert rc == bsf.E_INVALID


@pytest.mark.parametrize("dirs", [
    ((2, 1), (1, 2), (1, -2), (2, -1)),     # the directions of Alg. 3 / Table 1
    ((1, -1), (1, 0), (0, 1), (1, 1)),      # an upward direction first
    ((1, -2), (2, -1)),                     # upward directions only
])
def test_plan_accepts_upward_directions_anywhere(dirs):
    g = geo(bsf.Config(dirs=dirs, order=2, max_step=9.0))
    # every tap stays in the window: per direction r (R + 2) lattice steps back
    # and r (R + 1) forward, R = 4
    lo, hi = 2 * 6, 2 * 5
    assert g.pad_left == sum(lo * dx for dx, dy in dirs)
    assert g.pad_top == sum(lo * dy if dy > 0 else hi * -dy for dx, dy in dirs)
    assert g.pad_bottom == sum(hi * dy if dy > 0 else lo * -dy for dx, dy in dirs)


def test_box_tile_setter_validates():
    h0 = bsf.get_box_tile()
    assert h0 == 8
    try:
        bsf.set_box_tile(4)
        assert bsf.get_box_tile() == 4
        for bad in (0, 2, 6, 16):
            assert bsf.lib().bsf_set_box_tile(bad) == bsf.E_INVALID
        assert bsf.get_box_tile() == 4
    finally:
        bsf.set_box_tile(h0)


TABLE1 = ((2, 1), (1, 2), (1, -2), (2, -1))


def test_alg3_sizes_and_limits():
    """Alg. 3: four directions at order 1, tied, continuous steps; max_step is
    limited by the LDS rectangle one pixel needs (S <= 21 for the directions of
    Table 1: (floor(6 S) + 6 + 1)^2 FP64 values within 148 KiB)."""
    L = bsf.lib()
    ws = lambda cfg, H=64, W=80: L.bsf_alg3_workspace_bytes(ctypes.byref(cfg.c()), H, W)
    ok = bsf.Config(dirs=TABLE1, order=1, max_step=21.0)
    tiles = 4 * 5
    assert ws(ok) == 256 + 2 * ((tiles * 4 + 255) // 256 * 256)
    assert ws(bsf.Config(dirs=TABLE1, order=1, max_step=21.8)) > 0
    assert ws(bsf.Config(dirs=TABLE1, order=1, max_step=22.0)) == 0
    assert ws(bsf.Config(dirs=TABLE1, order=2, max_step=4.0)) == 0
    assert ws(bsf.Config(dirs=TABLE1[:3], order=1, max_step=4.0)) == 0
    assert ws(bsf.Config(dirs=TABLE1, order=1, max_step=4.0, mode=bsf.STEPS_INT)) == 0
    assert ws(bsf.Config(dirs=TABLE1, order=1, max_step=4.0, tied=False)) == 0   # the documented contract: tied
    # the directions of Section 1.1 reach less far: larger steps fit
    assert ws(bsf.Config(dirs=((1, 0), (0, 1), (1, 1), (1, -1)), order=1, max_step=40.0)) > 0


def test_alg3_entry_point_validates_before_launch():
    L = bsf.lib()
    cfg = bsf.Config(dirs=TABLE1, order=1, max_step=8.0).c()
    P = ctypes.c_void_p
    need = L.bsf_alg3_workspace_bytes(ctypes.byref(cfg), 8, 8)
    # no output at all
    r = L.bsf_filter_alg3(ctypes.byref(cfg), bsf.F32, P(16), 8, 8, 8, P(16), None, None, P(16), need, None)
    assert r == bsf.E_INVALID
    # pitch < W, bad dtype, null workspace
    r = L.bsf_filter_alg3(ctypes.byref(cfg), bsf.F32, P(16), 8, 8, 4, P(16), P(16), None, P(16), need, None)
    assert r == bsf.E_INVALID
    r = L.bsf_filter_alg3(ctypes.byref(cfg), 9, P(16), 8, 8, 8, P(16), P(16), None, P(16), need, None)
    assert r == bsf.E_INVALID
    r = L.bsf_filter_alg3(ctypes.byref(cfg), bsf.F32, P(16), 8, 8, 8, P(16), P(16), None, None, need, None)
    assert r == bsf.E_INVALID
    # workspace too small
    r = L.bsf_filter_alg3(ctypes.byref(cfg), bsf.F32, P(16), 8, 8, 8, P(16), P(16), None, P(16), need - 1, None)
    assert r == bsf.E_WORKSPACE
    # configurations it does not take
    bad = bsf.Config(dirs=TABLE1, order=2, max_step=8.0).c()
    r = L.bsf_filter_alg3(ctypes.byref(bad), bsf.F32, P(16), 8, 8, 8, P(16), P(16), None, P(16), need, None)
    assert r == bsf.E_UNSUPPORTED
    # an empty image enqueues nothing
    r = L.bsf_filter_alg3(ctypes.byref(cfg), bsf.F32, P(16), 0, 8, 8, P(16), P(16), None, P(16), need, None)
    assert r == bsf.OK
