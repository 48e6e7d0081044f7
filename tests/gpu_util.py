"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
state the tolerances against the oracle."""
import sys

import numpy as np
import torch

import paper_1109_5114_amd as bsf


def note(*a):
    """Print (and flush) what the next GPU step is, so a failing run names its case."""
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def cfg_of(d, **kw):
    mode = bsf.STEPS_INT if d["mode"] == "int" else bsf.STEPS_REAL
    args = dict(dirs=tuple(tuple(u) for u in d["dirs"]), order=d["order"], tied=d["tied"], mode=mode,
                max_step=float(d["max_step"]))
    args.update(kw)
    return bsf.Config(**args)


def run_forward(cfg, img, steps, want_num=False, want_den=False, ws=None):
    """Returns (out, num, den, flags, F) as numpy."""
    dev = torch.device("cuda:0")
    ti = torch.from_numpy(np.ascontiguousarray(img)).to(dev)
    ts = torch.from_numpy(np.ascontiguousarray(steps, dtype=np.float32)).to(dev)
    g = bsf.plan(cfg, *img.shape)
    ws = ws or bsf.Workspace(g.workspace_bytes, dev)
    res = bsf.filter_varying(cfg, ti, ts, want_num=want_num, want_den=want_den, ws=ws)
    if not isinstance(res, tuple):
        res = (res,)
    flags, F, _ = ws.status()
    out = res[0].cpu().numpy()
    num = res[1].cpu().numpy() if want_num else None
    den = res[-1].cpu().numpy() if want_den else None
    return out, num, den, flags, F


def float_tolerance(ref, F, quantised=True):
    """Bound on |gpu - oracle| for FP32 outputs.

    - fixed-point input: |f_q 2^-F - f| <= 2^-(F+1) per sample, and the kernel's
      weights are non-negative with sum 1, so the output moves by at most
      2^-(F+1) (zero when the samples are multiples of 2^-F);
    - the exact integer combination times FP64 phase weights and the FP64
      division carry a relative error of a few 2^-53;
    - the single rounding to FP32 adds at most 2^-24 relative.
    """
    q = 2.0 ** -(F + 1) if quantised else 0.0
    return q + (2.0 ** -24) * np.abs(ref) * (1 + 1e-6) + 1e-13 * np.abs(ref) + 1e-300


def assert_close(gpu, ref, F, quantised=True, what=""):
    tol = float_tolerance(ref, F, quantised)
    err = np.abs(gpu.astype(np.float64) - ref)
    bad = err > tol
    if bad.any():
        i = np.argmax(err - tol)
        raise AssertionError("%s: %d/%d outside tolerance; worst at %d: gpu %r ref %r err %.3g tol %.3g"
                             % (what, bad.sum(), bad.size, i, gpu.flat[i], ref.flat[i], err.flat[i], tol.flat[i]))
    return float((err / np.maximum(np.abs(ref), 2 ** -10)).max())
