"""The allocation-free forward entry point (bsf_filter_varying_noalloc, the
library's static per-GPU scratch) against bsf_filter_varying, through the C
ABI: bit-identical outputs on consecutive calls, the second with a smaller
input (the scratch keeps the previous call's contents), per-call flags, and
the size limit."""
import numpy as np
import pytest
import torch

import paper_1109_5114_amd as bsf
import workloads as WL
from tests.gpu_util import expected_F, note

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def inputs(shape, hi, seed, planes=4):
    rng = np.random.default_rng(seed)
    img = rng.random(shape, dtype=np.float32)
    steps = np.stack([WL.smooth(rng, *shape, 1.0, hi) for _ in range(planes)]).astype(np.float32)
    return img, steps


def both(cfg, img, steps, want_ds=False):
    ti, ts = torch.from_numpy(img).to(DEV), torch.from_numpy(steps).to(DEV)
    H, W = img.shape
    ws = bsf.Workspace(bsf.plan(cfg, H, W).workspace_bytes, DEV)
    ds_ref = torch.empty_like(ts) if want_ds else None
    ref = bsf.filter_varying(cfg, ti, ts, ws=ws, dsteps=ds_ref)
    flags_ref, F_ref, _ = ws.status()
    out = torch.full((H, W), float("nan"), dtype=torch.float32, device=DEV)
    ds = torch.full_like(ts, float("nan")) if want_ds else None
    st = torch.full((4,), -7, dtype=torch.int32, device=DEV)
    bsf.filter_varying_noalloc(cfg, ti, ts, out, dsteps=ds, status_out=st)
    torch.cuda.synchronize()
    got = st.cpu().numpy()
    assert got[0] == flags_ref and got[1] == F_ref, (got, flags_ref, F_ref)
    assert got[1] == expected_F(cfg, img, steps)
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint32), ref.cpu().numpy().view(np.uint32))
    if want_ds:
        np.testing.assert_array_equal(ds.cpu().numpy().view(np.uint32), ds_ref.cpu().numpy().view(np.uint32))
    return got


def test_noalloc_matches_workspace_entry_point_twice():
    cfg = bsf.Config(order=2, max_step=14.0)
    note("noalloc call 1 (190, 233)")
    img, steps = inputs((190, 233), 14.0, 301)
    st = both(cfg, img, steps, want_ds=True)
    assert st[0] == 0
    note("noalloc call 2 (61, 47), smaller")
    img, steps = inputs((61, 47), 14.0, 302)
    st = both(cfg, img, steps)
    assert st[0] == 0


def test_noalloc_integer_steps_and_flags():
    note("noalloc integer steps u8")
    d = WL.workload3(96, 130)
    cfg = bsf.Config(order=1, mode=bsf.STEPS_INT, max_step=float(d["max_step"]))
    ti = torch.from_numpy(d["img"]).to(DEV)
    ts = torch.from_numpy(d["steps"]).to(DEV)
    H, W = d["img"].shape
    num_ref, den_ref = bsf.filter_varying(cfg, ti, ts, want_num=True, want_den=True)[1:]
    out = torch.empty((H, W), dtype=torch.float32, device=DEV)
    num = torch.empty((H, W), dtype=torch.int64, device=DEV)
    den = torch.empty((H, W), dtype=torch.int64, device=DEV)
    st = torch.zeros(4, dtype=torch.int32, device=DEV)
    bsf.filter_varying_noalloc(cfg, ti, ts, out, num=num, den=den, status_out=st)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(num.cpu().numpy(), num_ref.cpu().numpy())
    np.testing.assert_array_equal(den.cpu().numpy(), den_ref.cpu().numpy())
    assert st.cpu().numpy()[0] == 0
    # a bad step raises the flag of that call only
    note("noalloc flags per call")
    cfg2 = bsf.Config(order=2, max_step=6.0)
    img, steps = inputs((20, 24), 6.0, 303)
    bad = steps.copy()
    bad[2, 4, 4] = np.nan
    o = torch.empty((20, 24), dtype=torch.float32, device=DEV)
    bsf.filter_varying_noalloc(cfg2, torch.from_numpy(img).to(DEV), torch.from_numpy(bad).to(DEV), o, status_out=st)
    torch.cuda.synchronize()
    assert st.cpu().numpy()[0] & bsf.FLAG_RANGE
    bsf.filter_varying_noalloc(cfg2, torch.from_numpy(img).to(DEV), torch.from_numpy(steps).to(DEV), o,
                               status_out=st)
    torch.cuda.synchronize()
    assert st.cpu().numpy()[0] == 0


def test_noalloc_rejects_sizes_beyond_its_scratch():
    note("noalloc size limit")
    cfg = bsf.Config(order=2, max_step=48.0)
    assert bsf.plan(cfg, 4096, 4096).workspace_bytes > bsf.NOALLOC_SCRATCH_BYTES
    img = torch.zeros((4096, 4096), dtype=torch.float32, device=DEV)
    steps = torch.ones((4, 4096, 4096), dtype=torch.float32, device=DEV)
    out = torch.empty_like(img)
    with pytest.raises(bsf.BsfError) as e:
        bsf.filter_varying_noalloc(cfg, img, steps, out)
    assert e.value.code == bsf.E_WORKSPACE
