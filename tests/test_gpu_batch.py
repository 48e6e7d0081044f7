"""GPU checks of the batched forward and the launch-shape tuning: a batch of
uneven images gives bit for bit the outputs of one call per image, recorded
graphs replay the current inputs, the batch status gathers the per-image
flags, the batched outputs match the oracle on sampled pixels, and every
tuning setting gives identical results."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1109_5114_amd as bsf
import workloads as WL
from tests.gpu_util import assert_close, cfg_of, expected_F, note

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def make_batch(shapes, planes, lo, hi, seed, smooth=True, integer=False):
    rng = np.random.default_rng(seed)
    imgs, steps = [], []
    for H, W in shapes:
        imgs.append(rng.random((H, W), dtype=np.float32))
        if integer:
            s = rng.integers(int(lo), int(hi) + 1, size=(planes, H, W)).astype(np.float32)
        elif smooth and H * W:
            s = np.stack([WL.smooth(rng, H, W, lo, hi) for _ in range(planes)]).astype(np.float32)
        else:
            s = rng.uniform(lo, hi, size=(planes, H, W)).astype(np.float32)
        steps.append(s)
    return imgs, steps


def to_dev(arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in arrs]


def per_image(cfg, imgs, steps):
    outs = []
    for im, st in zip(imgs, steps):
        if im.numel() == 0:
            outs.append(torch.empty(tuple(im.shape), dtype=torch.float32, device=DEV))
            continue
        outs.append(bsf.filter_varying(cfg, im, st))
    return [o.cpu().numpy() for o in outs]


CASES = [
    # tied order-2 four-direction kernels (the contiguous-tap gather)
    ("t2n4", dict(order=2, max_step=12.0), [(40, 52), (0, 9), (129, 77), (1, 300), (256, 256), (17, 1)], 4),
    # order 1, generic continuous-step gather
    ("order1", dict(order=1, max_step=9.0), [(33, 35), (70, 20), (5, 130)], 4),
    # untied order 2, generic gather with eight planes
    ("untied", dict(order=2, tied=False, max_step=5.0), [(21, 23), (12, 40)], 8),
    # integer steps
    ("int", dict(order=1, mode=bsf.STEPS_INT, max_step=11.0), [(64, 48), (31, 95), (2, 2)], 4),
]


@pytest.mark.parametrize("name,kw,shapes,planes", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_per_image_calls(name, kw, shapes, planes, use_graph):
    note("batch vs single", name, shapes, "graph" if use_graph else "eager")
    cfg = bsf.Config(**kw)
    imgs, steps = make_batch(shapes, planes, 1.0, cfg.max_step, 71, integer=cfg.mode == bsf.STEPS_INT)
    ti, ts = to_dev(imgs), to_dev(steps)
    batch = bsf.Batch(cfg, ti, ts)
    got = [o.cpu().numpy() for o in batch.run(use_graph=use_graph)]
    ref = per_image(cfg, ti, ts)
    for b, (g, r) in enumerate(zip(got, ref)):
        assert g.shape == r.shape
        np.testing.assert_array_equal(g, r, err_msg="image %d" % b)
    flags, F, _ = batch.ws.status()
    assert flags == 0


def test_graph_replays_follow_the_inputs():
    """Replays read the buffers as they are at replay time: change the
    images and steps in place between replays, with eager work and
    synchronisations in between, and compare each replay with eager calls."""
    note("graph replays")
    cfg = bsf.Config(order=2, max_step=10.0)
    shapes = [(64, 80), (33, 129), (150, 40)]
    batch_imgs, batch_steps = make_batch(shapes, 4, 1.0, 10.0, 73)
    ti, ts = to_dev(batch_imgs), to_dev(batch_steps)
    batch = bsf.Batch(cfg, ti, ts)
    rng = np.random.default_rng(75)
    for rep in range(4):
        for im, st in zip(ti, ts):
            im.copy_(torch.from_numpy(rng.random(tuple(im.shape), dtype=np.float32)).to(DEV))
            st.copy_(torch.from_numpy(rng.uniform(1.0, 10.0, size=tuple(st.shape)).astype(np.float32)).to(DEV))
        torch.cuda.synchronize()
        got = [o.clone() for o in batch.run(use_graph=True)]
        _ = (ti[0] * 2).sum().item()            # unrelated eager work between replays
        ref = per_image(cfg, ti, ts)
        for b in range(len(shapes)):
            np.testing.assert_array_equal(got[b].cpu().numpy(), ref[b], err_msg="replay %d image %d" % (rep, b))


def test_batch_status_collects_image_flags():
    note("batch status")
    cfg = bsf.Config(order=2, max_step=8.0)
    imgs, steps = make_batch([(20, 24), (18, 30)], 4, 1.0, 8.0, 77, smooth=False)
    steps[1][2, 5, 7] = 9.5                       # above max_step: range flag
    batch = bsf.Batch(cfg, to_dev(imgs), to_dev(steps))
    batch.run(use_graph=False)
    flags, F, bound = batch.ws.status(clear=True)
    assert flags & bsf.FLAG_RANGE
    assert F == min(expected_F(cfg, im, st) for im, st in zip(imgs, steps))
    flags, _, _ = batch.ws.status()
    assert flags == 0


def test_isotropic_batch_matches_oracle():
    """Eight images of the isotropic batched workload (sides 24..200) against
    the FP64 oracle on sampled pixels of every image."""
    note("workload4 small vs oracle")
    d = WL.workload4(B=8, lo=24, hi=200)
    cfg = cfg_of(d)
    imgs = [it["img"] for it in d["items"]]
    steps = [it["steps"] for it in d["items"]]
    batch = bsf.Batch(cfg, to_dev(imgs), to_dev(steps))
    outs = [o.cpu().numpy() for o in batch.run(use_graph=True)]
    _, F, _ = batch.ws.status()
    assert F == min(expected_F(cfg, im, st) for im, st in zip(imgs, steps))
    rng = np.random.default_rng(79)
    for b, (im, st, out) in enumerate(zip(imgs, steps, outs)):
        H, W = im.shape
        pix = np.unique(np.concatenate([rng.integers(0, H * W, 40), [0, W - 1, H * W - 1]]))
        ref = O.filter(im, d["dirs"], 2, True, O.REAL, st, pix=pix)
        # F is the smallest over the batch; every image's own F is at least that
        assert_close(out.reshape(-1)[pix], ref, F, what="image %d" % b)


@pytest.mark.parametrize("wx,tl,bh", [(8, 16, 4), (32, 128, 8), (64, 1024, 4)])
def test_tuning_does_not_change_results(wx, tl, bh):
    note("tuning", wx, tl, bh)
    cfg = bsf.Config(order=2, max_step=14.0)
    imgs, steps = make_batch([(97, 211)], 4, 1.0, 14.0, 81)
    ti, ts = to_dev(imgs)[0], to_dev(steps)[0]
    ref = bsf.filter_varying(cfg, ti, ts).cpu().numpy()
    G_ref = bsf.preintegrate(cfg, ti, F=24).cpu().numpy()
    old, old_h = bsf.get_tuning(), bsf.get_box_tile()
    try:
        bsf.set_tuning(wx, tl)
        bsf.set_box_tile(bh)
        got = bsf.filter_varying(cfg, ti, ts).cpu().numpy()
        G = bsf.preintegrate(cfg, ti, F=24).cpu().numpy()
        batch = bsf.Batch(cfg, [ti], [ts])
        got_b = batch.run(use_graph=False)[0].cpu().numpy()
    finally:
        bsf.set_tuning(*old)
        bsf.set_box_tile(old_h)
    np.testing.assert_array_equal(G, G_ref)
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(got_b, ref)


@pytest.mark.slow
def test_full_isotropic_batch_matches_oracle():
    """The whole batched workload (64 images with sides 128..2048, isotropic
    order-2 steps, sigma in [1, 16]) in one graph-captured call, as the
    benchmark runs it: sampled pixels of every image against the FP64 oracle,
    borders included."""
    note("workload4 full vs oracle")
    d = WL.workload4()
    cfg = cfg_of(d)
    imgs = [it["img"] for it in d["items"]]
    steps = [it["steps"] for it in d["items"]]
    batch = bsf.Batch(cfg, to_dev(imgs), to_dev(steps))
    outs = [o.cpu().numpy() for o in batch.run(use_graph=True)]
    flags, F, _ = batch.ws.status()
    assert flags == 0
    assert F == min(expected_F(cfg, im, st) for im, st in zip(imgs, steps))
    rng = np.random.default_rng(83)
    for b, (im, st, out) in enumerate(zip(imgs, steps, outs)):
        H, W = im.shape
        pix = np.unique(np.concatenate([rng.integers(0, H * W, 12), [0, W - 1, (H - 1) * W, H * W - 1]]))
        ref = O.filter(im, d["dirs"], 2, True, O.REAL, st, pix=pix)
        assert_close(out.reshape(-1)[pix], ref, F, what="image %d" % b)


@pytest.mark.parametrize("bh", [4, 8])
def test_box_tile_shapes_match_oracle(bh):
    """Both cluster-box tile heights against the oracle on a frame whose steps
    vary slowly in some places and quickly in others (tiles that fit the boxes
    and tiles that fall back)."""
    note("box tile", bh)
    rng = np.random.default_rng(85)
    H, W = 140, 150
    img = rng.random((H, W), dtype=np.float32)
    st = np.stack([WL.smooth(rng, H, W, 1.0, 30.0) for _ in range(4)]).astype(np.float32)
    st[:, 60:80, :] = rng.uniform(1.0, 30.0, size=(4, 20, W)).astype(np.float32)   # a band of rough steps
    cfg = bsf.Config(order=2, max_step=30.0)
    old_h = bsf.get_box_tile()
    try:
        bsf.set_box_tile(bh)
        out = bsf.filter_varying(cfg, to_dev([img])[0], to_dev([st])[0]).cpu().numpy()
    finally:
        bsf.set_box_tile(old_h)
    ref = O.filter(img, bsf.DIRS4, 2, True, O.REAL, st)
    F = expected_F(cfg, img, st)
    assert_close(out, ref, F, what="box tile %d" % bh)
