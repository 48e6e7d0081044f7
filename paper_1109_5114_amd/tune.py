"""Autotuner for the launch shapes of libbsf (bsf_set_tuning, bsf_set_box_tile).

Three shapes are free and do not change any result:
  * line_tl   -- steps per tile of the sheared running sums; it trades the
                 number of tiles (parallelism, carry traffic) against the
                 length of each tile's serial walk;
  * gather_wx -- width of one wavefront's pixel block in the tied order-2
                 four-direction gather for direction sets other than
                 (1,0), (0,1), (1,1), (1,-1); it sets which rows of the
                 running-sum window a wavefront's taps touch together;
  * box_h     -- tile height (4 or 8) of the cluster-box gather used for
                 (1,0), (0,1), (1,1), (1,-1): short tiles copy less of the window
                 per pixel but fall back to direct reads where the steps vary
                 quickly, so the choice depends on the step field.
The scans and the gather are separate launches, so each shape is timed on its
own stage: the running sums through bsf_preintegrate for every tile length,
then the per-pixel taps through bsf_forward_apply for every gather shape, on
the caller's image and steps when given (the step field decides the gather),
otherwise on a synthetic image with smooth steps over the workload's range.
A batch is tuned as a whole (tune_batch): bsf_filter_batched is timed with
each box height.  Each candidate's time is the median of a few runs bracketed
by HIP events on the launch stream.

Winners are kept in a JSON file keyed by device, configuration and size class
(log2 of the pixel count), so a process that has tuned once for a workload
reuses the choice (tune(..., cache=path)).
"""
import json
import math
import os
from typing import Dict, Optional, Sequence, Tuple

import torch

from . import (ARITH_EXACT, STEPS_INT, Batch, Config, Workspace, forward_apply, forward_prepare, get_box_tile,
               get_tuning, plan, preintegrate, set_box_tile, set_tuning)

LINE_TL = (32, 64, 128, 256, 512)
GATHER_WX = (8, 16, 32, 64)
BOX_H = (8, 4)


def _median_ms(fn, reps: int, stream) -> float:
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def _synthetic(cfg: Config, H: int, W: int, device, seed: int = 0) -> Tuple[torch.Tensor, torch.Tensor]:
    """A uniform image and, per step plane, a smooth field over [1, max_step]
    (a few low-frequency cosines), as step fields from covariance maps are."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    img = torch.rand((H, W), generator=g, dtype=torch.float32)
    yy = torch.arange(H, dtype=torch.float64)[:, None] / max(H, 1)
    xx = torch.arange(W, dtype=torch.float64)[None, :] / max(W, 1)
    planes = []
    for _ in range(cfg.planes):
        f = torch.zeros((H, W), dtype=torch.float64)
        for _ in range(6):
            kx, ky = torch.randint(-3, 4, (2,), generator=g).tolist()
            ph = float(torch.rand((1,), generator=g)) * 2 * math.pi
            f += torch.cos(2 * math.pi * (kx * xx + ky * yy) + ph)
        f = (f - f.min()) / max(float(f.max() - f.min()), 1e-12)
        s = 1.0 + (cfg.max_step - 1.0) * f
        planes.append(torch.round(s) if cfg.mode == STEPS_INT else s)
    steps = torch.stack(planes).to(torch.float32)
    return img.to(device), steps.to(device)


def _key(cfg: Config, H: int, W: int, device) -> str:
    name = torch.cuda.get_device_name(device)
    size_class = int(round(math.log2(max(H * W, 1))))
    return "%s|dirs=%s|r=%d|tied=%d|mode=%d|max=%g|arith=%d|px=2^%d" % (
        name, cfg.dirs, cfg.order, int(cfg.tied), cfg.mode, cfg.max_step, cfg.arith, size_class)


def _load(path: Optional[str]) -> Dict[str, Dict[str, int]]:
    if path and os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def tune(cfg: Config, H: int, W: int, device="cuda", reps: int = 3, cache: Optional[str] = None,
         line_tl: Sequence[int] = LINE_TL, gather_wx: Sequence[int] = GATHER_WX, box_h: Sequence[int] = BOX_H,
         img: Optional[torch.Tensor] = None, steps: Optional[torch.Tensor] = None, verbose: bool = False):
    """Pick (gather_wx, line_tl, box_h) for images of about H x W under cfg
    (timed on img and steps when given), set them process-wide and return
    {"gather_wx", "line_tl", "box_h", "timings"}."""
    device = torch.device(device)
    key = _key(cfg, H, W, device)
    table = _load(cache)
    if key in table:
        best = table[key]
        set_tuning(best["gather_wx"], best["line_tl"])
        set_box_tile(best.get("box_h", get_box_tile()))
        return dict(best, cached=True)
    old, old_h = get_tuning(), get_box_tile()
    if img is None or steps is None:
        img, steps = _synthetic(cfg, H, W, device)
    H, W = img.shape
    stream = torch.cuda.current_stream(device)
    timings = {"line_tl": {}, "gather": {}}
    try:
        # running sums: every tile length, the gather's shape left as it is
        for tl in line_tl:
            set_tuning(old[0], tl)
            g = plan(cfg, H, W)
            ws = Workspace(g.workspace_bytes_g_external, device)
            preintegrate(cfg, img, F=24, ws=ws)      # warm-up
            ms = _median_ms(lambda: preintegrate(cfg, img, F=24, ws=ws), reps, stream)
            timings["line_tl"][tl] = ms
            del ws
        best_tl = min(timings["line_tl"], key=timings["line_tl"].get)
        # taps: every gather shape on one prepared window
        set_tuning(old[0], best_tl)
        g = plan(cfg, H, W)
        ws = Workspace(g.workspace_bytes, device)
        forward_prepare(cfg, img, steps, ws)
        out = torch.empty((H, W), dtype=torch.float32, device=device)
        canonical = sorted(map(tuple, cfg.dirs)) == sorted(((1, 0), (0, 1), (1, 1), (1, -1)))
        t2n4 = cfg.mode != STEPS_INT and cfg.order == 2 and cfg.tied and cfg.n_dirs == 4 \
            and cfg.arith == ARITH_EXACT
        table1 = sorted(map(tuple, cfg.dirs)) == sorted(((2, 1), (1, 2), (1, -2), (2, -1)))
        if t2n4 and canonical:
            shapes = [(old[0], h) for h in box_h]
        elif t2n4 and table1:
            shapes = [(old[0], old_h)]   # its cluster-box kernel has one tile shape
        elif t2n4:
            shapes = [(wx, old_h) for wx in gather_wx]
        else:
            shapes = [(old[0], old_h)]
        for wx, h in shapes:
            set_tuning(wx, best_tl)
            set_box_tile(h)
            forward_apply(cfg, 3, steps, ws, out)    # warm-up
            ms = _median_ms(lambda: forward_apply(cfg, 3, steps, ws, out), reps, stream)
            timings["gather"]["%d,%d" % (wx, h)] = ms
        best_wx, best_h = min(shapes, key=lambda sh: timings["gather"]["%d,%d" % sh])
    except Exception:
        set_tuning(*old)
        set_box_tile(old_h)
        raise
    set_tuning(best_wx, best_tl)
    set_box_tile(best_h)
    best = {"gather_wx": int(best_wx), "line_tl": int(best_tl), "box_h": int(best_h)}
    if verbose:
        print("tune %s -> %s %s" % (key, best, timings), flush=True)
    if cache:
        table = _load(cache)
        table[key] = best
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(best, timings=timings, cached=False)


def tune_batch(cfg: Config, imgs: Sequence[torch.Tensor], steps: Sequence[torch.Tensor], reps: int = 3,
               box_h: Sequence[int] = BOX_H, verbose: bool = False):
    """Pick the cluster-box tile height for a batch by timing the batched call
    (without graph capture) on the caller's images and steps with each; sets it
    process-wide and returns {"box_h", "timings"}."""
    if not imgs:
        return {"box_h": get_box_tile(), "timings": {}}
    device = imgs[0].device
    stream = torch.cuda.current_stream(device)
    old_h = get_box_tile()
    timings = {}
    try:
        for h in box_h:
            set_box_tile(h)
            b = Batch(cfg, imgs, steps)
            b.run(use_graph=False)                   # warm-up
            timings[h] = _median_ms(lambda: b.run(use_graph=False), reps, stream)
            del b
    except Exception:
        set_box_tile(old_h)
        raise
    best = min(timings, key=timings.get)
    set_box_tile(best)
    if verbose:
        print("tune_batch -> box_h %d %s" % (best, timings), flush=True)
    return {"box_h": int(best), "timings": timings}
