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


def _ceil_log2(v):
    """ceil(log2 v) of float64 values >= 1, from the binary exponent."""
    m, e = np.frexp(np.asarray(v, dtype=np.float64))
    return np.where(m == 0.5, e - 1, e)


def expected_F(cfg, img, steps):
    """The fixed-point bits F the library must choose for this input, computed
    on the host from the rule it documents:
        F = 62 - ceil(log2 max|f|) - max_x ceil(log2 prod_j L_j(x)),
    L_j = 2 floor((s_j - 1)/2) + 3 for continuous steps and s_j for integer
    steps (steps clamped to [1, max_step] in float32), the product taken in
    float64 and raised by 2^-40 so that it stays an upper bound; integer
    images use F = 0 and a fixed frac_bits is used as given.  Tests assert that
    the device chose exactly this F, so a tolerance sized from it does not
    follow a regression of the device's choice."""
    if img.dtype != np.float32:
        return 0
    if cfg.frac_bits >= 0:
        return int(cfg.frac_bits)
    planes = steps.shape[0]
    per_plane = cfg.order if cfg.tied else 1
    prod = np.ones(steps.shape[1:], dtype=np.float64)
    for q in range(planes):
        sc = np.fmin(np.fmax(steps[q].astype(np.float32), np.float32(1.0)), np.float32(cfg.max_step))
        if cfg.mode == bsf.STEPS_INT:
            ln = np.rint(sc).astype(np.float64)
        else:
            ln = (np.float32(2.0) * np.floor((sc - np.float32(1.0)) * np.float32(0.5)) + np.float32(3.0))
            ln = ln.astype(np.float64)
        for _ in range(per_plane):
            prod = prod * ln
    eP = int(_ceil_log2(prod * (1.0 + 2.0 ** -40)).max()) if prod.size else 0
    fmax = float(np.abs(img[np.isfinite(img)]).max()) if img.size else 0.0
    ef = 0 if fmax == 0.0 else int(_ceil_log2(fmax))
    return 62 - ef - eP


def run_forward(cfg, img, steps, want_num=False, want_den=False, ws=None):
    """Returns (out, num, den, flags, F) as numpy.  F is the host's expected
    F (expected_F), after checking that the device used exactly that."""
    dev = torch.device("cuda:0")
    ti = torch.from_numpy(np.ascontiguousarray(img)).to(dev)
    ts = torch.from_numpy(np.ascontiguousarray(steps, dtype=np.float32)).to(dev)
    g = bsf.plan(cfg, *img.shape)
    ws = ws or bsf.Workspace(g.workspace_bytes, dev)
    res = bsf.filter_varying(cfg, ti, ts, want_num=want_num, want_den=want_den, ws=ws)
    if not isinstance(res, tuple):
        res = (res,)
    flags, F_dev, _ = ws.status()
    F = expected_F(cfg, np.asarray(img), np.asarray(steps, dtype=np.float32))
    assert F_dev == F, "device chose F = %d, the documented rule gives %d" % (F_dev, F)
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
