#!/usr/bin/env python3
"""Benchmark of the space-variant box-spline filter on one MI355X.

Workload: a 4096 x 4096 FP32 image (uniform [0,1) plus 5% salt-and-pepper),
four directions (1,0), (0,1), (1,1), (1,-1) each pre-integrated twice (order 2,
steps tied per direction), continuous per-pixel steps from a smooth elliptical
covariance field (workloads.workload2).  One step = the whole forward hot path
on inputs already resident in HBM: range check and fixed-point choice, the
running sums, and the per-pixel taps with exact integer combination.

Prints one JSON line.  Also times the plain FP64 path on the same workload and
the CPU oracle on a bounded sample of pixels (rank 0, one GPU only).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixels/s and HBM GB/s, fwd and fwd+adjoint, 4096^2 N=4 order-2 vs plain path"
HBM_PEAK_GBS = 8000.0
# int64 adds per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 64-bit
# add (v_lshl_add_u64) per lane per cycle
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# exact separable contraction of the 9^4 taps of one pixel: 729 + 243 + 81 + 27
# groups of nine values reduced to three operator outputs, 8 int64 adds each
INT64_OPS_PER_PIXEL = (729 + 243 + 81 + 27) * 8
FP64_PEAK_TFLOPS = 78.6
# wave instructions per second: 256 CUs, each one VALU wave instruction per clock
VALU_ISSUE_PER_S = 256 * 2.4e9


def measured_traffic(box_h):
    """HBM bytes per launch of the tap kernel instance the timed run used (tile
    height box_h, no step derivatives) from the committed counter runs
    (profiles/traffic.json), or None when the kernel sources have changed since
    they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for name in rec.get("sources", []):
        with open(os.path.join(ROOT, name), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec.get("sha256"):
        return None
    entry = rec.get("kernels", {}).get("k_gather_t2n4_box<false, %d, false, 0>" % box_h)
    return None if entry is None else entry.get("bytes_per_launch")


def alg3_counters():
    """FP64 flops and VALU instructions per launch of the Alg. 3 kernel from the
    committed counter run (profiles/alg3_counters.json), or None when its source
    has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "alg3_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for name in rec.get("sources", []):
        with open(os.path.join(ROOT, name), "rb") as fh:
            h.update(fh.read())
    return rec if h.hexdigest() == rec.get("sha256") else None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check-pixels", type=int, default=48)
    ap.add_argument("--adjoint-steps", type=int, default=3)
    ap.add_argument("--batch", type=int, default=64, help="images in the batched workload (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--int-size", type=int, default=2048, help="integer-step uint8 workload side (0: skip)")
    ap.add_argument("--int-steps", type=int, default=20)
    ap.add_argument("--diff-images", type=int, default=16, help="images of the differentiation workload (0: skip)")
    ap.add_argument("--diff-steps", type=int, default=3)
    ap.add_argument("--alg3-size", type=int, default=4096, help="Alg. 3 workload side (0: skip)")
    ap.add_argument("--alg3-steps", type=int, default=5)
    ap.add_argument("--alg2-size", type=int, default=4096, help="Alg. 2 workload side (0: skip)")
    ap.add_argument("--alg2-steps", type=int, default=3)
    ap.add_argument("--alg2-orders", default="1,2",
                    help="orders of Alg. 2's box splines, comma-separated (the paper's is 1)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the timed region, one device copy of this size (profiler byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the filter would shard by "
              "row strips with a halo; see the design notes).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1109_5114_amd as bsf
    import paper_1109_5114_amd.tune as tuner
    import workloads as WL

    dev = torch.device("cuda:0")
    t = time.time()
    d = WL.workload2(args.size, args.size)
    log("inputs generated in %.1f s" % (time.time() - t))
    H, W = d["img"].shape
    cfg = bsf.Config(dirs=d["dirs"], order=2, tied=True, mode=bsf.STEPS_REAL, max_step=d["max_step"])
    img = torch.from_numpy(d["img"]).to(dev)
    steps = torch.from_numpy(d["steps"]).to(dev)
    tuning = None
    if not args.no_tune:
        t = time.time()
        tuning = tuner.tune(cfg, H, W, dev, img=img, steps=steps)
        log("tuned in %.1f s: gather_wx %d line_tl %d box_h %d" % (time.time() - t, tuning["gather_wx"],
                                                                   tuning["line_tl"], tuning["box_h"]))
    box_h = bsf.get_box_tile()  # the tap kernel's tile for the timed forward
    geo = bsf.plan(cfg, H, W)
    ws = bsf.Workspace(geo.workspace_bytes, dev)
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        bsf.forward_prepare(cfg, img, steps, ws)
        bsf.forward_apply(cfg, bsf.F32, steps, ws, out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k in range(K):
        ev[k][0].record(stream)
        bsf.forward_prepare(cfg, img, steps, ws)
        ev[k][1].record(stream)
        bsf.forward_apply(cfg, bsf.F32, steps, ws, out)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - w0) / K * 1e3
    # medians over the timed steps (HIP events on the launch stream)
    prep_ms = float(np.median([e[0].elapsed_time(e[1]) for e in ev]))
    apply_ms = float(np.median([e[1].elapsed_time(e[2]) for e in ev]))
    step_ms = float(np.median([e[0].elapsed_time(e[2]) for e in ev]))
    flags, F, log2b = ws.status()
    mpx = H * W / (step_ms / 1e3) / 1e6
    # algorithmic HBM bytes of the forward as built (what each pass must move
    # at least once): the range/F pass reads the four FP32 step planes and the
    # image; the first running sum reads the image and writes the window; each
    # sheared pass reads its input twice (aggregates, rescan) and writes it
    # once; the taps read the window once, the steps, and write the output
    win = geo.win_h * geo.win_w
    px = H * W
    forward_bytes = px * (16 + 4) + (px * 4 + win * 8) + 3 * win * 24 + (win * 8 + px * (16 + 4))
    # backward with the step derivative: the forward writes d out / d steps
    # (16 B/px); the adjoint reads g (twice: its range and the scatter), writes
    # the window once, runs four transposed passes (row 16, sheared 24 B per
    # element) and reads the window, g and d out / d steps to write both gradients
    backward_bytes = px * 16 + px * 8 + win * 8 + win * (16 + 3 * 24) + (win * 8 + px * (4 + 16 + 4 + 16))
    minimum_bytes = 40 * px
    log("step %.3f ms (prepare %.3f, apply %.3f, wall %.3f), F=%d flags=%d" % (step_ms, prep_ms, apply_ms, wall,
                                                                          F, flags))

    # ---- parity spot check against the oracle on sampled pixels (outside the timed region)
    import oracle as O
    rng = np.random.default_rng(4242)
    pix = np.concatenate([rng.integers(0, H * W, args.check_pixels), [0, W - 1, H * W - 1]])
    got = out.cpu().numpy().reshape(-1)[pix].astype(np.float64)
    t = time.time()
    ref = O.filter(d["img"], d["dirs"], 2, True, O.REAL, d["steps"], pix=pix)
    cpu_check_s = time.time() - t
    rel = float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 2.0 ** -10)))
    abs_err = float(np.max(np.abs(got - ref)))

    # ---- plain FP64 path on the same workload
    cfg64 = bsf.Config(dirs=d["dirs"], order=2, tied=True, mode=bsf.STEPS_REAL, max_step=d["max_step"],
                       arith=bsf.ARITH_FP64)
    out64 = torch.empty_like(out)
    ws64 = bsf.Workspace(bsf.plan(cfg64, H, W).workspace_bytes, dev)
    bsf.forward_prepare(cfg64, img, steps, ws64)
    bsf.forward_apply(cfg64, bsf.F32, steps, ws64, out64)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.plain_steps):
        bsf.forward_prepare(cfg64, img, steps, ws64)
        bsf.forward_apply(cfg64, bsf.F32, steps, ws64, out64)
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / args.plain_steps
    got64 = out64.cpu().numpy().reshape(-1)[pix].astype(np.float64)
    plain_abs = float(np.max(np.abs(got64 - ref)))
    plain_rel = float(np.max(np.abs(got64 - ref) / np.maximum(np.abs(ref), 2.0 ** -10)))
    log("plain fp64 %.3f ms, max abs err %.3g" % (plain_ms, plain_abs))

    # ---- forward + adjoint (image and step gradients) on the same workload
    fa = None
    if args.adjoint_steps > 0:
        gen = np.random.default_rng(11095114 + 99)
        gout = torch.from_numpy(gen.standard_normal((H, W), dtype=np.float32)).to(dev)
        ds = torch.empty_like(steps)
        gi = torch.empty_like(out)
        gs = torch.empty_like(steps)
        wsb = bsf.Workspace(bsf.backward_workspace_bytes(cfg, H, W), dev)

        def bwd():
            bsf.filter_backward(cfg, steps, gout, dsteps=ds, ws=wsb, grad_img=gi, grad_steps=gs)

        def fwd_adj():
            bsf.forward_prepare(cfg, img, steps, ws)
            bsf.forward_apply(cfg, bsf.F32, steps, ws, out, dsteps=ds)
            bwd()

        fwd_adj()
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        fwd_ms, bwd_ms = [], []
        for _ in range(args.adjoint_steps):
            e0.record(stream)
            bsf.forward_prepare(cfg, img, steps, ws)
            bsf.forward_apply(cfg, bsf.F32, steps, ws, out, dsteps=ds)
            e1.record(stream)
            bwd()
            e2.record(stream)
            torch.cuda.synchronize()
            fwd_ms.append(e0.elapsed_time(e1))
            bwd_ms.append(e1.elapsed_time(e2))
        # step-gradient spot check against the oracle's analytic derivative
        sub = pix[:16]
        _, rgs = O.grad_real(d["img"], d["dirs"], 2, True, d["steps"], gout.cpu().numpy(), pix=sub,
                             want_img=False)
        ggs = gs.cpu().numpy().reshape(4, -1)[:, sub].T
        gerr = float(np.max(np.abs(ggs - rgs)) / max(np.abs(rgs).max(), 1e-30))
        t_fa = float(np.median(fwd_ms) + np.median(bwd_ms))
        fa_bytes = forward_bytes + backward_bytes
        fa = {"ms_per_step": t_fa, "value": H * W / (t_fa / 1e3) / 1e6, "unit": "Mpixels/s",
              "forward_with_derivative_ms": float(np.median(fwd_ms)), "backward_ms": float(np.median(bwd_ms)),
              "hbm_gbs": fa_bytes / (t_fa / 1e3) / 1e9, "hbm_frac": fa_bytes / (t_fa / 1e3) / 1e9 / HBM_PEAK_GBS,
              "algorithmic_bytes": fa_bytes,
              "steps": args.adjoint_steps, "grad_steps_max_rel_err_vs_oracle": gerr}
        log("fwd+adjoint %.3f ms (fwd %.3f, bwd %.3f)" % (t_fa, np.median(fwd_ms), np.median(bwd_ms)))

    # ---- differentiation workload: 16 images of 1024^2, forward with the step
    # derivative and the adjoint for every image
    diff = None
    if args.diff_images > 0:
        d5 = WL.workload5(B=args.diff_images)
        cfg5 = bsf.Config(dirs=d5["dirs"], order=2, tied=True, mode=bsf.STEPS_REAL, max_step=d5["max_step"])
        H5, W5 = d5["imgs"][0].shape
        ws5 = bsf.Workspace(bsf.plan(cfg5, H5, W5).workspace_bytes, dev)
        wsb5 = bsf.Workspace(bsf.backward_workspace_bytes(cfg5, H5, W5), dev)
        imgs5 = [torch.from_numpy(a).to(dev) for a in d5["imgs"]]
        steps5 = [torch.from_numpy(a).to(dev) for a in d5["steps"]]
        gouts5 = [torch.from_numpy(a).to(dev) for a in d5["gout"]]
        out5, ds5 = torch.empty((H5, W5), dtype=torch.float32, device=dev), torch.empty_like(steps5[0])
        gi5, gs5 = torch.empty_like(out5), torch.empty_like(steps5[0])

        def diff_step():
            for im, st, g in zip(imgs5, steps5, gouts5):
                bsf.forward_prepare(cfg5, im, st, ws5)
                bsf.forward_apply(cfg5, bsf.F32, st, ws5, out5, dsteps=ds5)
                bsf.filter_backward(cfg5, st, g, dsteps=ds5, ws=wsb5, grad_img=gi5, grad_steps=gs5)

        diff_step()
        torch.cuda.synchronize()
        t5 = []
        for _ in range(args.diff_steps):
            e0.record(stream)
            diff_step()
            e1.record(stream)
            torch.cuda.synchronize()
            t5.append(e0.elapsed_time(e1))
        ms5 = float(np.median(t5))
        px5 = len(imgs5) * H5 * W5
        diff = {"workload": d5["name"], "images": len(imgs5), "ms_per_step": ms5,
                "value": px5 / (ms5 / 1e3) / 1e6, "unit": "Mpixels/s", "steps": args.diff_steps}
        log("differentiation %d x %dx%d fwd+adjoint: %.3f ms" % (len(imgs5), H5, W5, ms5))
        del imgs5, steps5, gouts5, ws5, wsb5

    # ---- Alg. 3: the box spline of Table 1 read through eq. interpolation,
    # FP64, on a covariance field (minimum-kurtosis steps for that box spline)
    alg3 = None
    if args.alg3_size > 0:
        da = WL.workload_alg3(args.alg3_size, args.alg3_size)
        Ha, Wa = da["img"].shape
        cfga = bsf.Config(dirs=da["dirs"], order=1, tied=True, mode=bsf.STEPS_REAL, max_step=da["max_step"])
        imga = torch.from_numpy(da["img"]).to(dev)
        stepsa = bsf.cov_to_steps(cfga, torch.from_numpy(da["cov"]).to(dev))
        wsa = bsf.Workspace(bsf.lib().bsf_alg3_workspace_bytes(bsf.ctypes.byref(cfga.c()), Ha, Wa), dev)
        outa = torch.empty((Ha, Wa), dtype=torch.float32, device=dev)
        out64a = torch.empty((Ha, Wa), dtype=torch.float64, device=dev)
        bsf.filter_alg3(cfga, imga, stepsa, out=outa, out_f64=out64a, ws=wsa)
        torch.cuda.synchronize()
        ta = []
        for _ in range(args.alg3_steps):
            e0.record(stream)
            bsf.filter_alg3(cfga, imga, stepsa, out=outa, ws=wsa)
            e1.record(stream)
            torch.cuda.synchronize()
            ta.append(e0.elapsed_time(e1))
        msa = float(np.median(ta))
        # sampled pixels against the oracle's Alg. 3 on crops holding each footprint
        sa = stepsa.cpu().numpy()
        o64 = out64a.cpu().numpy()
        erra = 0.0
        for x, y in rng.integers(0, [Wa, Ha], (16, 2)):
            s_ = sa[:, y, x].astype(np.float64)
            rx = int(np.ceil(0.5 * sum(abs(u[0]) * v for u, v in zip(da["dirs"], s_)))) + 3
            ry = int(np.ceil(0.5 * sum(abs(u[1]) * v for u, v in zip(da["dirs"], s_)))) + 3
            x0, x1, y0, y1 = max(0, x - rx), min(Wa, x + rx + 1), max(0, y - ry), min(Ha, y + ry + 1)
            ref = O.alg3(np.ascontiguousarray(da["img"][y0:y1, x0:x1]), da["dirs"],
                         np.ascontiguousarray(sa[:, y0:y1, x0:x1]),
                         pix=np.array([(y - y0) * (x1 - x0) + (x - x0)]))[0]
            erra = max(erra, abs(float(o64[y, x]) - ref))
        flags_a, _, _ = wsa.status()
        # VALU-bound: FP64 flops the hardware counted, against the FP64 vector
        # peak, and the VALU issue rate (one wave instruction per CU per cycle)
        ca = alg3_counters() if (Ha, Wa) == (4096, 4096) else None
        roof_a = None
        if ca is not None:
            ach = ca["fp64_flops_per_launch"] / (msa / 1e3) / 1e12
            roof_a = {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": ach / FP64_PEAK_TFLOPS,
                      "valu_issue_frac": ca["valu_instructions_per_launch"] / (msa / 1e3) / VALU_ISSUE_PER_S}
        alg3 = {"workload": da["name"], "ms_per_step": msa, "value": Ha * Wa / (msa / 1e3) / 1e6,
                "roofline": roof_a,
                "unit": "Mpixels/s", "dtype": "f64", "steps": args.alg3_steps,
                "max_abs_err_vs_oracle": erra, "pixels_checked": 16, "device_flags": flags_a,
                "step_percentiles_50_99_100": [float(v) for v in np.percentile(sa, [50, 99, 100])]}
        log("alg3 %dx%d: %.3f ms, max abs err %.2e" % (Ha, Wa, msa, erra))
        del imga, stepsa, wsa, outa, out64a

    # ---- Alg. 2: both four-direction sets, each pixel filtered by the set its
    # orientation sector picks, against one set alone (the paper puts the cost
    # of the second set at 10-15 %)
    alg2 = None
    if args.alg2_size > 0:
        alg2 = []
        d2 = WL.workload_alg3(args.alg2_size, args.alg2_size)
        H2, W2 = d2["img"].shape
        img2 = torch.from_numpy(d2["img"]).to(dev)
        cov2 = torch.from_numpy(d2["cov"]).to(dev)
    for order2 in ([int(o) for o in args.alg2_orders.split(",") if o] if args.alg2_size > 0 else []):
        # max_step from the data: the largest step either set needs for this field
        smax = 1.0
        for dirs in (((1, 0), (0, 1), (1, 1), (1, -1)), WL.DIRS_TABLE1):
            probe = bsf.Config(dirs=dirs, order=order2, tied=True, mode=bsf.STEPS_REAL, max_step=1e5)
            smax = max(smax, float(bsf.cov_to_steps(probe, cov2).max().item()))
        cfg2 = bsf.Config(order=order2, tied=True, mode=bsf.STEPS_REAL, max_step=float(np.ceil(smax)))
        ws2 = bsf.Workspace(bsf.lib().bsf_alg2_workspace_bytes(bsf.ctypes.byref(cfg2.c()), H2, W2), dev)
        bank2 = torch.empty((H2, W2), dtype=torch.uint8, device=dev)
        out2 = torch.empty((H2, W2), dtype=torch.float32, device=dev)
        wsc = bsf.Workspace(256, dev)
        steps1 = torch.empty((4, H2, W2), dtype=torch.float32, device=dev)
        ws1 = bsf.Workspace(bsf.plan(cfg2, H2, W2).workspace_bytes, dev)

        def two_sets():
            bsf.filter_alg2(cfg2, img2, cov2, out=out2, bank=bank2, ws=ws2)

        def one_set():
            bsf.cov_to_steps(cfg2, cov2, steps=steps1, ws=wsc)
            bsf.forward_prepare(cfg2, img2, steps1, ws1)
            bsf.forward_apply(cfg2, bsf.F32, steps1, ws1, out2)

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t = []
            for _ in range(args.alg2_steps):
                e0.record(stream)
                fn()
                e1.record(stream)
                torch.cuda.synchronize()
                t.append(e0.elapsed_time(e1))
            return float(np.median(t))
        ms_two, ms_one = timed(two_sets), timed(one_set)
        frac2 = float(bank2.float().mean().item())
        alg2.append({"workload": "%dx%d covariance field (sigma 2-12 px), order %d, max_step %g"
                                 % (H2, W2, order2, cfg2.max_step),
                     "order": order2, "ms_two_sets": ms_two, "ms_one_set": ms_one, "cost_ratio": ms_two / ms_one,
                     "pixels_on_second_set": frac2, "steps": args.alg2_steps})
        log("alg2 %dx%d order %d: two sets %.3f ms, one set %.3f ms (x%.2f), %.0f%% of pixels on the second"
            % (H2, W2, order2, ms_two, ms_one, ms_two / ms_one, 100 * frac2))
        del ws2, bank2, out2, steps1, ws1
    if args.alg2_size > 0:
        del img2, cov2

    # ---- integer steps on a uint8 image: exact int64 numerator and prod s
    integer = None
    if args.int_size > 0:
        d3 = WL.workload3(args.int_size, args.int_size)
        H3, W3 = d3["img"].shape
        cfg3 = bsf.Config(dirs=d3["dirs"], order=1, tied=True, mode=bsf.STEPS_INT, max_step=d3["max_step"])
        img3 = torch.from_numpy(d3["img"]).to(dev)
        steps3 = torch.from_numpy(d3["steps"]).to(dev)
        # launch shapes for this workload (its image is smaller: shorter line
        # tiles give its scans more parallel work); the workspace size depends
        # on them, so it is sized after
        tuning3 = None if args.no_tune else tuner.tune(cfg3, H3, W3, dev, img=img3, steps=steps3)
        ws3 = bsf.Workspace(bsf.plan(cfg3, H3, W3).workspace_bytes, dev)
        out3 = torch.empty((H3, W3), dtype=torch.float32, device=dev)
        num3 = torch.empty((H3, W3), dtype=torch.int64, device=dev)
        den3 = torch.empty_like(num3)

        def step3():
            bsf.forward_prepare(cfg3, img3, steps3, ws3)
            bsf.forward_apply(cfg3, bsf.U8, steps3, ws3, out3, num=num3, den=den3)

        step3()
        torch.cuda.synchronize()
        ev3 = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.int_steps)]
        for k in range(args.int_steps):
            ev3[k][0].record(stream)
            bsf.forward_prepare(cfg3, img3, steps3, ws3)
            ev3[k][1].record(stream)
            bsf.forward_apply(cfg3, bsf.U8, steps3, ws3, out3, num=num3, den=den3)
            ev3[k][2].record(stream)
        torch.cuda.synchronize()
        p3 = float(np.median([e[0].elapsed_time(e[1]) for e in ev3]))
        a3 = float(np.median([e[1].elapsed_time(e[2]) for e in ev3]))
        pix3 = rng.integers(0, H3 * W3, 64)
        _, rnum, rden = O.filter(d3["img"], d3["dirs"], 1, True, O.INT, d3["steps"], pix=pix3, want_int=True)
        exact = bool(np.array_equal(num3.cpu().numpy().reshape(-1)[pix3], rnum)
                     and np.array_equal(den3.cpu().numpy().reshape(-1)[pix3], rden))
        # algorithmic HBM bytes of the tap kernel per pixel: four FP32 step
        # planes, the running-sum window once, FP32 out, int64 numerator and
        # product of steps
        g3 = bsf.plan(cfg3, H3, W3)
        tap_bytes = H3 * W3 * (16 + 4 + 8 + 8) + g3.g_bytes
        integer = {"workload": d3["name"], "ms_per_step": p3 + a3, "prepare_ms": p3, "apply_ms": a3,
                   "tuning": None if tuning3 is None else {k: tuning3[k] for k in ("gather_wx", "line_tl", "box_h")},
                   "value": H3 * W3 / ((p3 + a3) / 1e3) / 1e6, "unit": "Mpixels/s",
                   "apply_hbm_gbs": tap_bytes / (a3 / 1e3) / 1e9,
                   "apply_hbm_frac": tap_bytes / (a3 / 1e3) / 1e9 / HBM_PEAK_GBS,
                   "bit_exact_sampled": exact, "pixels_checked": int(len(pix3))}
        log("integer %dx%d: %.3f ms (prepare %.3f, apply %.3f), exact=%s" % (H3, W3, p3 + a3, p3, a3, exact))
        del ws3, img3, steps3, out3, num3, den3

    # ---- batched: images of uneven sizes, each stage one launch over the batch, replayed as a graph
    batched = None
    if args.batch > 0:
        del ws64, out64
        t = time.time()
        d4 = WL.workload4(B=args.batch)
        log("batched inputs generated in %.1f s" % (time.time() - t))
        cfg4 = bsf.Config(dirs=d4["dirs"], order=2, tied=True, mode=bsf.STEPS_REAL, max_step=d4["max_step"])
        px = [it["img"].size for it in d4["items"]]
        side = int(math.sqrt(sum(px) / len(px)))
        tuning4 = None if args.no_tune else tuner.tune(cfg4, side, side, dev)
        imgs4 = [torch.from_numpy(it["img"]).to(dev) for it in d4["items"]]
        steps4 = [torch.from_numpy(it["steps"]).to(dev) for it in d4["items"]]
        if tuning4 is not None:
            # the batch's own gather tile, timed on its own images and steps
            tuning4["box_h"] = tuner.tune_batch(cfg4, imgs4, steps4)["box_h"]
        batch = bsf.Batch(cfg4, imgs4, steps4)
        batch.run(use_graph=True)                       # records the graph
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.batch_steps):
            batch.run(use_graph=True)
        e1.record(stream)
        torch.cuda.synchronize()
        b_ms = e0.elapsed_time(e1) / args.batch_steps
        bflags, bF, _ = batch.ws.status()
        # the same images one call each, for context
        wsi = bsf.Workspace(max(bsf.plan(cfg4, *im.shape).workspace_bytes for im in imgs4), dev)
        e0.record(stream)
        for im, st, o in zip(imgs4, steps4, batch.outs):
            bsf.filter_varying(cfg4, im, st, out=o, ws=wsi)
        e1.record(stream)
        torch.cuda.synchronize()
        loop_ms = e0.elapsed_time(e1)
        # oracle spot check on sampled pixels of a few images
        berr = 0.0
        for b in range(0, len(imgs4), max(1, len(imgs4) // 4)):
            it = d4["items"][b]
            hh, ww = it["img"].shape
            pb = rng.integers(0, hh * ww, 8)
            refb = O.filter(it["img"], d4["dirs"], 2, True, O.REAL, it["steps"], pix=pb)
            gotb = batch.outs[b].cpu().numpy().reshape(-1)[pb].astype(np.float64)
            berr = max(berr, float(np.max(np.abs(gotb - refb) / np.maximum(np.abs(refb), 2.0 ** -10))))
        batched = {"value": sum(px) / (b_ms / 1e3) / 1e6, "unit": "Mpixels/s", "ms_per_step": b_ms,
                   "images": len(px), "pixels": int(sum(px)), "graph": True, "steps": args.batch_steps,
                   "per_image_calls_ms": loop_ms, "frac_bits": bF, "device_flags": bflags,
                   "max_rel_err_vs_oracle": berr,
                   "tuning": None if tuning4 is None else {k: tuning4[k] for k in ("gather_wx", "line_tl", "box_h")},
                   "workload": d4["name"]}
        log("batched %d images %.1f Mpx: %.3f ms (per-image calls %.3f ms)" % (len(px), sum(px) / 1e6, b_ms,
                                                                                loop_ms))
        del batch, imgs4, steps4, wsi

    # ---- CPU oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        # calibrate on a few thousand pixels (the first oracle call above also
        # paid for thread start-up), then size the sample to ~cpu_seconds
        calib = rng.integers(0, H * W, 2000)
        t = time.time()
        O.filter(d["img"], d["dirs"], 2, True, O.REAL, d["steps"], pix=calib)
        per_px = (time.time() - t) / len(calib)
        n = int(max(16, min(H * W, args.cpu_seconds / max(per_px, 1e-9))))
        sample = rng.integers(0, H * W, n)
        t = time.time()
        O.filter(d["img"], d["dirs"], 2, True, O.REAL, d["steps"], pix=sample)
        dt = time.time() - t
        cpu = {"value": n / dt / 1e6, "unit": "Mpixels/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": "%d random pixels of the 4096x4096 order-2 workload, %.1f s" % (n, dt)}
        log("cpu oracle %d px in %.1f s" % (n, dt))

    if args.copy_mib > 0:
        # a plain streaming kernel of known size: reads and writes copy_mib MiB
        # (an elementwise multiply by one, so it shows as its own dispatch)
        src = torch.ones((args.copy_mib << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    ops = INT64_OPS_PER_PIXEL * H * W
    achieved = ops / (apply_ms / 1e3) / 1e12
    traffic = measured_traffic(box_h)
    res = {
        "metric": METRIC,
        "value": mpx,
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "%dx%d fp32 image, directions (1,0),(0,1),(1,1),(1,-1), order 2 tied, "
                               "continuous steps from a covariance field (sigma 2-24 px)" % (H, W),
                   "H": H, "W": W, "order": 2, "n_dirs": 4, "max_step": d["max_step"],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / ALU_PEAK_TOPS,
                     "traffic": traffic,
                     "kernel": "per-pixel taps (forward_apply)", "kernel_ms": apply_ms},
        "cpu_baseline": cpu,
        "stages_ms": {"prepare": prep_ms, "apply": apply_ms, "wall_per_step": wall},
        "accuracy": {"max_rel_err_vs_oracle": rel, "max_abs_err_vs_oracle": abs_err,
                     "pixels_checked": int(len(pix)), "frac_bits": F, "device_flags": flags},
        "plain_fp64": {"ms_per_step": plain_ms, "value": H * W / (plain_ms / 1e3) / 1e6,
                       "max_abs_err_vs_oracle": plain_abs, "max_rel_err_vs_oracle": plain_rel},
        "fwd_adjoint": fa,
        "batched": batched,
        "integer_steps": integer,
        "hbm": {"gbs": forward_bytes / (step_ms / 1e3) / 1e9,
                "frac": forward_bytes / (step_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                "algorithmic_bytes": forward_bytes, "minimum_bytes": minimum_bytes,
                "minimum_gbs": minimum_bytes / (step_ms / 1e3) / 1e9,
                "peak_gbs": HBM_PEAK_GBS,
                # the tap kernel's calibrated counter bytes over its stage time
                "tap_kernel_measured_bytes": traffic,
                "tap_kernel_measured_gbs": None if traffic is None else traffic / (apply_ms / 1e3) / 1e9},
        "differentiation": diff,
        "alg3": alg3,
        "alg2": alg2,
        "tuning": None if tuning is None else {k: tuning[k] for k in ("gather_wx", "line_tl", "box_h")},
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
