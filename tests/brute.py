"""Brute-force evaluations used to pin the CPU oracle.  Written directly from
the definitions with explicit enumeration; no code shared with ``oracle/`` or
with the GPU library.  Tiny inputs only."""
import itertools
import math
from fractions import Fraction

import numpy as np


def box_cell_weight(i, s):
    """|[i-1/2, i+1/2] ^ [-s/2, s/2]| as an exact Fraction (s a Fraction)."""
    lo = max(Fraction(2 * i - 1, 2), -s / 2)
    hi = min(Fraction(2 * i + 1, 2), s / 2)
    return hi - lo if hi > lo else Fraction(0)


def box_int_offsets(s):
    """Offsets i with weight 1 for the half-open box (-s/2, s/2] used as a
    convolution kernel: sample f(x - t) for t in the box, i = -t."""
    return [-t for t in range(-s, s + 1) if Fraction(-s, 2) < t <= Fraction(s, 2)]


def kernel_by_enumeration_real(fdirs, steps):
    """dict offset -> exact weight (Fraction), normalised by prod(steps), by
    enumerating every i in Z^M with nonzero factor weights."""
    S = [Fraction(s).limit_denominator(1 << 30) if not isinstance(s, Fraction) else s for s in steps]
    supports = []
    for s in S:
        h = int(math.floor(s / 2 + Fraction(1, 2))) + 1
        supports.append([(i, box_cell_weight(i, s)) for i in range(-h, h + 1)
                         if box_cell_weight(i, s) != 0])
    den = Fraction(1)
    for s in S:
        den *= s
    out = {}
    for combo in itertools.product(*supports):
        w = Fraction(1)
        px = py = 0
        for (i, wi), (dx, dy) in zip(combo, fdirs):
            w *= wi
            px += i * dx
            py += i * dy
        out[(px, py)] = out.get((px, py), 0) + w
    return {k: v / den for k, v in out.items()}


def kernel_by_enumeration_int(fdirs, steps):
    """dict offset -> sample count for integer steps."""
    supports = [box_int_offsets(int(s)) for s in steps]
    out = {}
    for combo in itertools.product(*supports):
        px = sum(i * d[0] for i, d in zip(combo, fdirs))
        py = sum(i * d[1] for i, d in zip(combo, fdirs))
        out[(px, py)] = out.get((px, py), 0) + 1
    return out


def dense(kdict):
    xs = [p[0] for p in kdict]
    ys = [p[1] for p in kdict]
    x0, y0 = min(xs), min(ys)
    K = np.zeros((max(ys) - y0 + 1, max(xs) - x0 + 1))
    for (x, y), v in kdict.items():
        K[y - y0, x - x0] = float(v)
    return x0, y0, K


def preintegrate_by_definition(f, fdirs, window):
    """G(p) = sum over k in N^M of f(p - sum_j k_j u_j), f zero outside the
    image, evaluated on window = (y_lo, y_hi, x_lo, x_hi) with Python ints.
    Enumerates k up to the point where every term is outside the image."""
    H, W = f.shape
    y_lo, y_hi, x_lo, x_hi = window
    span = (y_hi - y_lo) + (x_hi - x_lo) + H + W
    pts = [(y, x, int(f[y, x])) for y in range(H) for x in range(W) if f[y, x] != 0]
    G = {}
    # count representations v = sum_j k_j u_j with k_j >= 0 for every needed v
    counts = {}
    for ks in itertools.product(range(span + 1), repeat=len(fdirs)):
        vx = sum(k * d[0] for k, d in zip(ks, fdirs))
        vy = sum(k * d[1] for k, d in zip(ks, fdirs))
        if abs(vx) > span or abs(vy) > span:
            continue
        counts[(vx, vy)] = counts.get((vx, vy), 0) + 1
    for y in range(y_lo, y_hi):
        for x in range(x_lo, x_hi):
            acc = 0
            for (py, px, v) in pts:
                c = counts.get((x - px, y - py), 0)
                if c:
                    acc += c * v
            G[(y, x)] = acc
    return G


def dtft(K, x0, y0, wx, wy):
    """sum_p K(p) exp(-i (wx px + wy py))."""
    h, w = K.shape
    xs = (x0 + np.arange(w))[None, :]
    ys = (y0 + np.arange(h))[:, None]
    return np.sum(K * np.exp(-1j * (wx * xs + wy * ys)))
