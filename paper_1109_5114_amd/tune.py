"""Autotuner for the launch shapes of libbsf (bsf_set_tuning).

Two shapes are free and do not change any result:
  * line_tl   -- steps per tile of the sheared running sums; it trades the
                 number of tiles (parallelism, carry traffic) against the
                 length of each tile's serial walk;
  * gather_wx -- width of one wavefront's pixel block in the tied order-2
                 four-direction gather; it sets which rows of the running-sum
                 window a wavefront's taps touch together (cache reuse).
The scans and the gather are separate launches, so each shape is timed on its
own stage: the running sums through bsf_preintegrate for every tile length,
then the per-pixel taps through bsf_forward_apply for every block width, on a
synthetic image of the workload's size and step range.  Each candidate's time
is the median of a few runs bracketed by HIP events on the launch stream.

Winners are kept in a JSON file keyed by device, configuration and size class
(log2 of the pixel count), so a process that has tuned once for a workload
reuses the choice (tune(..., cache=path)).
"""
import json
import math
import os
from typing import Dict, Optional, Sequence, Tuple

import torch

from . import (ARITH_EXACT, STEPS_INT, Config, Workspace, forward_apply, forward_prepare, get_tuning, plan,
               preintegrate, set_tuning)

LINE_TL = (32, 64, 128, 256, 512)
GATHER_WX = (8, 16, 32, 64)


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
    g = torch.Generator(device="cpu").manual_seed(seed)
    img = torch.rand((H, W), generator=g, dtype=torch.float32)
    if cfg.mode == STEPS_INT:
        steps = torch.randint(1, int(cfg.max_step) + 1, (cfg.planes, H, W), generator=g).to(torch.float32)
    else:
        steps = 1.0 + (cfg.max_step - 1.0) * torch.rand((cfg.planes, H, W), generator=g, dtype=torch.float32)
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
         line_tl: Sequence[int] = LINE_TL, gather_wx: Sequence[int] = GATHER_WX, verbose: bool = False):
    """Pick (gather_wx, line_tl) for images of about H x W under cfg, set it
    process-wide and return {"gather_wx", "line_tl", "timings"}."""
    device = torch.device(device)
    key = _key(cfg, H, W, device)
    table = _load(cache)
    if key in table:
        best = table[key]
        set_tuning(best["gather_wx"], best["line_tl"])
        return dict(best, cached=True)
    old = get_tuning()
    img, steps = _synthetic(cfg, H, W, device)
    stream = torch.cuda.current_stream(device)
    timings = {"line_tl": {}, "gather_wx": {}}
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
        # taps: every block width on one prepared window
        set_tuning(old[0], best_tl)
        g = plan(cfg, H, W)
        ws = Workspace(g.workspace_bytes, device)
        forward_prepare(cfg, img, steps, ws)
        out = torch.empty((H, W), dtype=torch.float32, device=device)
        # the block width only shapes the tied order-2 kernel for direction sets
        # other than (1,0), (0,1), (1,1), (1,-1); those use the cluster-box kernel
        canonical = sorted(map(tuple, cfg.dirs)) == sorted(((1, 0), (0, 1), (1, 1), (1, -1)))
        uses_wx = cfg.mode != STEPS_INT and cfg.order == 2 and cfg.tied and cfg.n_dirs == 4 \
            and cfg.arith == ARITH_EXACT and not canonical
        for wx in (gather_wx if uses_wx else (old[0],)):
            set_tuning(wx, best_tl)
            forward_apply(cfg, 3, steps, ws, out)    # warm-up
            ms = _median_ms(lambda: forward_apply(cfg, 3, steps, ws, out), reps, stream)
            timings["gather_wx"][wx] = ms
        best_wx = min(timings["gather_wx"], key=timings["gather_wx"].get)
    except Exception:
        set_tuning(*old)
        raise
    set_tuning(best_wx, best_tl)
    best = {"gather_wx": int(best_wx), "line_tl": int(best_tl)}
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
