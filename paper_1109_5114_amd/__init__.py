"""Python binding of libbsf, the MI355X space-variant box-spline filter.

This module only marshals arguments: PyTorch provides device memory and the
current HIP stream, and every step of the filter runs in the HIP kernels of
libbsf.so behind the C ABI declared in include/bsf.h.  There is no CPU
fallback: if the library is missing, importing the ops raises.
"""
import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbsf.so")

OK, E_INVALID, E_RANGE, E_OVERFLOW, E_WORKSPACE, E_DEVICE, E_UNSUPPORTED = range(7)
U8, U16, F32 = 1, 2, 3
STEPS_INT, STEPS_REAL = 0, 1
ARITH_EXACT, ARITH_FP64 = 0, 1
FLAG_RANGE, FLAG_OVERFLOW, FLAG_NONFINITE = 1, 2, 4
MAX_DIRS = 8
DIRS4 = ((1, 0), (0, 1), (1, 1), (1, -1))


class BsfError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__("%s: %s" % (what, status_string(code)))


class _Config(ctypes.Structure):
    _fields_ = [("n_dirs", ctypes.c_int32), ("dirs", ctypes.c_int32 * (2 * MAX_DIRS)),
                ("order", ctypes.c_int32), ("tied", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("max_step", ctypes.c_float), ("frac_bits", ctypes.c_int32), ("arith", ctypes.c_int32)]


class Geometry(ctypes.Structure):
    _fields_ = [("pad_top", ctypes.c_int64), ("pad_bottom", ctypes.c_int64),
                ("pad_left", ctypes.c_int64), ("pad_right", ctypes.c_int64),
                ("win_h", ctypes.c_int64), ("win_w", ctypes.c_int64),
                ("g_bytes", ctypes.c_size_t), ("workspace_bytes", ctypes.c_size_t),
                ("workspace_bytes_g_external", ctypes.c_size_t)]


class _ImageDesc(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("steps", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("H", ctypes.c_int64), ("W", ctypes.c_int64), ("pitch", ctypes.c_int64)]


_lib = None

EXPORTS = ("bsf_workspace_init", "bsf_plan", "bsf_preintegrate", "bsf_filter_varying",
           "bsf_forward_prepare", "bsf_forward_apply",
           "bsf_backward_workspace_bytes", "bsf_filter_backward", "bsf_batched_workspace_bytes",
           "bsf_filter_batched", "bsf_set_tuning", "bsf_get_tuning", "bsf_read_device_status",
           "bsf_status_string", "bsf_version", "bsf_filter_varying_noalloc", "bsf_cov_to_steps",
           "bsf_alg1_workspace_bytes", "bsf_filter_alg1", "bsf_alg2_workspace_bytes", "bsf_filter_alg2",
           "bsf_set_box_tile", "bsf_get_box_tile", "bsf_alg3_workspace_bytes", "bsf_filter_alg3")
NOALLOC_SCRATCH_BYTES = 64 << 20


def lib():
    """The loaded libbsf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbsf.so is not built; run paper_1109_5114_amd/build.py "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        cfgp = ctypes.POINTER(_Config)
        L.bsf_workspace_init.argtypes = [P, sz, P]
        L.bsf_plan.argtypes = [cfgp, i64, i64, ctypes.POINTER(Geometry)]
        L.bsf_preintegrate.argtypes = [cfgp, i32, P, i64, i64, i64, i32, P, P, sz, P]
        L.bsf_filter_varying.argtypes = [cfgp, i32, P, i64, i64, i64, P, P, P, P, P, P, P, sz, P]
        L.bsf_forward_prepare.argtypes = [cfgp, i32, P, i64, i64, i64, P, P, P, sz, P]
        L.bsf_forward_apply.argtypes = [cfgp, i32, i64, i64, P, P, P, P, P, P, P, sz, P]
        L.bsf_backward_workspace_bytes.argtypes = [cfgp, i64, i64]
        L.bsf_backward_workspace_bytes.restype = sz
        L.bsf_filter_backward.argtypes = [cfgp, i64, i64, P, P, P, P, P, P, sz, P]
        L.bsf_batched_workspace_bytes.argtypes = [cfgp, i32, ctypes.POINTER(_ImageDesc)]
        L.bsf_batched_workspace_bytes.restype = sz
        L.bsf_filter_batched.argtypes = [cfgp, i32, ctypes.POINTER(_ImageDesc), P, sz, P, i32]
        L.bsf_set_tuning.argtypes = [i32, i32]
        L.bsf_get_tuning.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.bsf_get_tuning.restype = None
        L.bsf_read_device_status.argtypes = [P, P, ctypes.POINTER(ctypes.c_uint32),
                                             ctypes.POINTER(i32), ctypes.POINTER(i32), i32]
        L.bsf_filter_varying_noalloc.argtypes = [cfgp, i32, P, i64, i64, i64, P, P, P, P, P, P, P]
        L.bsf_cov_to_steps.argtypes = [cfgp, P, i64, i64, ctypes.c_float, P, P, sz, P]
        L.bsf_alg1_workspace_bytes.argtypes = [cfgp, i64, i64]
        L.bsf_alg1_workspace_bytes.restype = sz
        L.bsf_filter_alg1.argtypes = [cfgp, P, i64, i64, i64, P, P, P, sz, P]
        L.bsf_alg2_workspace_bytes.argtypes = [cfgp, i64, i64]
        L.bsf_alg2_workspace_bytes.restype = sz
        L.bsf_filter_alg2.argtypes = [cfgp, i32, P, i64, i64, i64, P, P, P, P, sz, P]
        L.bsf_alg3_workspace_bytes.argtypes = [cfgp, i64, i64]
        L.bsf_alg3_workspace_bytes.restype = sz
        L.bsf_filter_alg3.argtypes = [cfgp, i32, P, i64, i64, i64, P, P, P, P, sz, P]
        L.bsf_set_box_tile.argtypes = [i32]
        L.bsf_get_box_tile.argtypes = []
        L.bsf_get_box_tile.restype = i32
        L.bsf_status_string.argtypes = [i32]
        L.bsf_status_string.restype = ctypes.c_char_p
        L.bsf_version.restype = ctypes.c_char_p
        for name in ("bsf_workspace_init", "bsf_plan", "bsf_preintegrate", "bsf_filter_varying",
                     "bsf_forward_prepare", "bsf_forward_apply",
                     "bsf_filter_backward", "bsf_filter_batched", "bsf_set_tuning",
                     "bsf_read_device_status", "bsf_filter_varying_noalloc", "bsf_cov_to_steps",
                     "bsf_filter_alg1", "bsf_filter_alg2", "bsf_set_box_tile", "bsf_filter_alg3"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def status_string(code):
    try:
        return lib().bsf_status_string(int(code)).decode()
    except ImportError:
        return "status %d" % code


def _check(code, what):
    if code != OK:
        raise BsfError(code, what)


@dataclass(frozen=True)
class Config:
    """Filter configuration (mirrors bsf_config)."""
    dirs: Tuple[Tuple[int, int], ...] = DIRS4
    order: int = 1
    tied: bool = True
    mode: int = STEPS_REAL
    max_step: float = 16.0
    frac_bits: int = -1
    arith: int = ARITH_EXACT

    @property
    def n_dirs(self):
        return len(self.dirs)

    @property
    def planes(self):
        return self.n_dirs if self.tied else self.n_dirs * self.order

    def c(self):
        c = _Config()
        c.n_dirs = len(self.dirs)
        for k, (dx, dy) in enumerate(self.dirs):
            c.dirs[2 * k] = int(dx)
            c.dirs[2 * k + 1] = int(dy)
        c.order = int(self.order)
        c.tied = int(bool(self.tied))
        c.mode = int(self.mode)
        c.max_step = float(self.max_step)
        c.frac_bits = int(self.frac_bits)
        c.arith = int(self.arith)
        return c


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dtype_code(t: torch.Tensor):
    if t.dtype == torch.uint8:
        return U8
    if t.dtype == torch.uint16:
        return U16
    if t.dtype == torch.float32:
        return F32
    raise TypeError("images are uint8, uint16 or float32, got %s" % t.dtype)


def plan(cfg: Config, H: int, W: int) -> Geometry:
    g = Geometry()
    _check(lib().bsf_plan(ctypes.byref(cfg.c()), int(H), int(W), ctypes.byref(g)), "bsf_plan")
    return g


class Workspace:
    """Device scratch owned by the caller (here: a torch uint8 tensor)."""

    def __init__(self, nbytes: int, device="cuda"):
        self.nbytes = max(int(nbytes), 256)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        _check(lib().bsf_workspace_init(_ptr(self.buf), self.nbytes, _stream(self.buf.device)),
               "bsf_workspace_init")

    def ensure(self, nbytes: int):
        if nbytes > self.nbytes:
            self.__init__(nbytes, self.buf.device)
        return self

    def ptr(self):
        return _ptr(self.buf)

    def status(self, clear=False):
        """Synchronises the current stream; returns (flags, F_used, log2_bound)."""
        fl, F, b = ctypes.c_uint32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().bsf_read_device_status(self.ptr(), _stream(self.buf.device), ctypes.byref(fl),
                                            ctypes.byref(F), ctypes.byref(b), int(bool(clear))),
               "bsf_read_device_status")
        return fl.value, F.value, b.value


_ws_cache = {}


def _workspace(device, nbytes):
    key = (str(device),)
    ws = _ws_cache.get(key)
    if ws is None:
        ws = _ws_cache[key] = Workspace(nbytes, device)
    return ws.ensure(nbytes)


def _check_image(img):
    if not img.is_cuda or img.dim() != 2:
        raise ValueError("image must be a 2-D device tensor")
    if img.numel() and img.stride(1) != 1:
        raise ValueError("image rows must be contiguous")


def _pitch(img):
    return img.stride(0) if img.numel() else img.shape[1]


def _check_steps(cfg, steps, H, W):
    if steps.dtype != torch.float32 or not steps.is_cuda or not steps.is_contiguous():
        raise ValueError("steps must be a contiguous float32 device tensor")
    if tuple(steps.shape) != (cfg.planes, H, W):
        raise ValueError("steps must have shape %s, got %s" % ((cfg.planes, H, W), tuple(steps.shape)))


def preintegrate(cfg: Config, img: torch.Tensor, F: int = 24, ws: Optional[Workspace] = None) -> torch.Tensor:
    """Running sums on the window; returns the [win_h][win_w] int64 (or float64) tensor."""
    _check_image(img)
    H, W = img.shape
    g = plan(cfg, H, W)
    dt = torch.float64 if cfg.arith == ARITH_FP64 else torch.int64
    G = torch.empty((g.win_h, g.win_w), dtype=dt, device=img.device)
    ws = ws or _workspace(img.device, g.workspace_bytes_g_external)
    ws.ensure(g.workspace_bytes_g_external)
    _check(lib().bsf_preintegrate(ctypes.byref(cfg.c()), _dtype_code(img), _ptr(img), H, W, _pitch(img),
                                  int(F), _ptr(G), ws.ptr(), ws.nbytes, _stream(img.device)),
           "bsf_preintegrate")
    return G


def filter_varying(cfg: Config, img: torch.Tensor, steps: torch.Tensor, out: Optional[torch.Tensor] = None,
                   want_num: bool = False, want_den: bool = False, save_G: bool = False,
                   ws: Optional[Workspace] = None, dsteps: Optional[torch.Tensor] = None):
    """Forward space-variant filter.  Returns out (float32 [H][W]) and, on
    request, num/den (int64, integer-step mode) and the saved window G.  When
    dsteps (float32 [planes][H][W]) is given it receives d out / d steps."""
    _check_image(img)
    H, W = img.shape
    _check_steps(cfg, steps, H, W)
    g = plan(cfg, H, W)
    dev = img.device
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=dev)
    num = torch.empty((H, W), dtype=torch.int64, device=dev) if want_num else None
    den = torch.empty((H, W), dtype=torch.int64, device=dev) if want_den else None
    G = None
    if save_G:
        G = torch.empty((g.win_h, g.win_w), dtype=torch.float64 if cfg.arith == ARITH_FP64 else torch.int64,
                        device=dev)
    need = g.workspace_bytes_g_external if save_G else g.workspace_bytes
    ws = ws or _workspace(dev, need)
    ws.ensure(need)
    if dsteps is not None:
        _check_steps(cfg, dsteps, H, W)
    _check(lib().bsf_filter_varying(ctypes.byref(cfg.c()), _dtype_code(img), _ptr(img), H, W, _pitch(img),
                                    _ptr(steps), _ptr(out), _ptr(num), _ptr(den), _ptr(dsteps), _ptr(G), ws.ptr(),
                                    ws.nbytes, _stream(dev)),
           "bsf_filter_varying")
    res = [out]
    if want_num:
        res.append(num)
    if want_den:
        res.append(den)
    if save_G:
        res.append(G)
    return res[0] if len(res) == 1 else tuple(res)


def filter_varying_noalloc(cfg: Config, img: torch.Tensor, steps: torch.Tensor, out: torch.Tensor,
                           num: Optional[torch.Tensor] = None, den: Optional[torch.Tensor] = None,
                           dsteps: Optional[torch.Tensor] = None, status_out: Optional[torch.Tensor] = None):
    """The forward filter through bsf_filter_varying_noalloc: no workspace, the
    library's per-GPU static scratch (at most NOALLOC_SCRATCH_BYTES of window,
    carries and status).  Every output tensor is passed in; status_out (int32
    [4], device) receives this call's flags, F_used and log2_bound."""
    _check_image(img)
    H, W = img.shape
    _check_steps(cfg, steps, H, W)
    if status_out is not None and (status_out.dtype != torch.int32 or status_out.numel() < 4
                                   or not status_out.is_cuda):
        raise ValueError("status_out must be an int32 device tensor of 4 entries")
    if dsteps is not None:
        _check_steps(cfg, dsteps, H, W)
    _check(lib().bsf_filter_varying_noalloc(ctypes.byref(cfg.c()), _dtype_code(img), _ptr(img), H, W, _pitch(img),
                                            _ptr(steps), _ptr(out), _ptr(num), _ptr(den), _ptr(dsteps),
                                            _ptr(status_out), _stream(img.device)),
           "bsf_filter_varying_noalloc")
    return out


def cov_to_steps(cfg: Config, cov: torch.Tensor, sub: float = 0.0, steps: Optional[torch.Tensor] = None,
                 ws: Optional[Workspace] = None) -> torch.Tensor:
    """Minimum-kurtosis steps of the configuration's four directions for a
    covariance field cov (float32 [3][H][W]: C11, C12, C22), sub subtracted
    from the diagonal first.  Returns steps float32 [planes][H][W]."""
    if cov.dtype != torch.float32 or not cov.is_cuda or not cov.is_contiguous() or cov.dim() != 3 \
            or cov.shape[0] != 3:
        raise ValueError("cov must be a contiguous float32 [3][H][W] device tensor")
    _, H, W = cov.shape
    if steps is None:
        steps = torch.empty((cfg.planes, H, W), dtype=torch.float32, device=cov.device)
    _check_steps(cfg, steps, H, W)
    ws = ws or _workspace(cov.device, 256)
    _check(lib().bsf_cov_to_steps(ctypes.byref(cfg.c()), _ptr(cov), H, W, float(sub), _ptr(steps), ws.ptr(),
                                  ws.nbytes, _stream(cov.device)), "bsf_cov_to_steps")
    return steps


def _check_cov(cov, H, W):
    if cov.dtype != torch.float32 or not cov.is_cuda or not cov.is_contiguous() or tuple(cov.shape) != (3, H, W):
        raise ValueError("cov must be a contiguous float32 [3][H][W] device tensor")


def filter_alg1(cfg: Config, img: torch.Tensor, cov: torch.Tensor, out: Optional[torch.Tensor] = None,
                ws: Optional[Workspace] = None) -> torch.Tensor:
    """Alg. 1: isotropic pre-filter of half the condition2 bound, then the
    space-variant filter of C - sigma^2 I (bsf_filter_alg1)."""
    _check_image(img)
    H, W = img.shape
    _check_cov(cov, H, W)
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=img.device)
    need = lib().bsf_alg1_workspace_bytes(ctypes.byref(cfg.c()), H, W)
    if need == 0:
        raise BsfError(E_UNSUPPORTED, "bsf_alg1_workspace_bytes")
    ws = ws or _workspace(img.device, need)
    ws.ensure(need)
    _check(lib().bsf_filter_alg1(ctypes.byref(cfg.c()), _ptr(img), H, W, _pitch(img), _ptr(cov), _ptr(out),
                                 ws.ptr(), ws.nbytes, _stream(img.device)), "bsf_filter_alg1")
    return out


def filter_alg2(cfg: Config, img: torch.Tensor, cov: torch.Tensor, out: Optional[torch.Tensor] = None,
                bank: Optional[torch.Tensor] = None, ws: Optional[Workspace] = None) -> torch.Tensor:
    """Alg. 2: per-pixel choice between the two four-direction box splines by
    orientation sector (bsf_filter_alg2).  bank (uint8 [H][W]) receives the
    choice when given."""
    _check_image(img)
    H, W = img.shape
    _check_cov(cov, H, W)
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=img.device)
    if bank is not None and (bank.dtype != torch.uint8 or tuple(bank.shape) != (H, W) or not bank.is_contiguous()):
        raise ValueError("bank must be a contiguous uint8 [H][W] device tensor")
    need = lib().bsf_alg2_workspace_bytes(ctypes.byref(cfg.c()), H, W)
    if need == 0:
        raise BsfError(E_UNSUPPORTED, "bsf_alg2_workspace_bytes")
    ws = ws or _workspace(img.device, need)
    ws.ensure(need)
    _check(lib().bsf_filter_alg2(ctypes.byref(cfg.c()), _dtype_code(img), _ptr(img), H, W, _pitch(img), _ptr(cov),
                                 _ptr(out), _ptr(bank), ws.ptr(), ws.nbytes, _stream(img.device)), "bsf_filter_alg2")
    return out


def filter_alg3(cfg: Config, img: torch.Tensor, steps: torch.Tensor, out: Optional[torch.Tensor] = None,
                out_f64: Optional[torch.Tensor] = None, ws: Optional[Workspace] = None):
    """Alg. 3 in FP64 (bsf_filter_alg3): running sums, the 16 taps of Table 1
    read through eq. interpolation.  Fills out (float32) and/or out_f64
    (float64); with neither given, returns a new float32 tensor."""
    _check_image(img)
    H, W = img.shape
    _check_steps(cfg, steps, H, W)
    if out is None and out_f64 is None:
        out = torch.empty((H, W), dtype=torch.float32, device=img.device)
    for t, dt in ((out, torch.float32), (out_f64, torch.float64)):
        if t is not None and (t.dtype != dt or tuple(t.shape) != (H, W) or not t.is_contiguous()):
            raise ValueError("outputs must be contiguous [H][W] device tensors of float32 / float64")
    need = lib().bsf_alg3_workspace_bytes(ctypes.byref(cfg.c()), H, W)
    if need == 0:
        raise BsfError(E_UNSUPPORTED, "bsf_alg3_workspace_bytes")
    ws = ws or _workspace(img.device, need)
    ws.ensure(need)
    _check(lib().bsf_filter_alg3(ctypes.byref(cfg.c()), _dtype_code(img), _ptr(img), H, W, _pitch(img),
                                 _ptr(steps), _ptr(out), _ptr(out_f64), ws.ptr(), ws.nbytes, _stream(img.device)),
           "bsf_filter_alg3")
    return out if out is not None else out_f64


def forward_prepare(cfg: Config, img: torch.Tensor, steps: torch.Tensor, ws: Workspace,
                    G: Optional[torch.Tensor] = None):
    """Range check, choice of F and running sums (into G, or into ws when G is None)."""
    _check_image(img)
    H, W = img.shape
    _check_steps(cfg, steps, H, W)
    _check(lib().bsf_forward_prepare(ctypes.byref(cfg.c()), _dtype_code(img), _ptr(img), H, W, _pitch(img),
                                     _ptr(steps), _ptr(G), ws.ptr(), ws.nbytes, _stream(img.device)),
           "bsf_forward_prepare")


def forward_apply(cfg: Config, dtype_code: int, steps: torch.Tensor, ws: Workspace, out: torch.Tensor,
                  G: Optional[torch.Tensor] = None, num: Optional[torch.Tensor] = None,
                  den: Optional[torch.Tensor] = None, dsteps: Optional[torch.Tensor] = None):
    """Per-pixel taps of the running sums left by forward_prepare."""
    _, H, W = steps.shape
    _check_steps(cfg, steps, H, W)
    _check(lib().bsf_forward_apply(ctypes.byref(cfg.c()), int(dtype_code), H, W, _ptr(steps), _ptr(G), _ptr(out),
                                   _ptr(num), _ptr(den), _ptr(dsteps), ws.ptr(), ws.nbytes, _stream(steps.device)),
           "bsf_forward_apply")
    return out


def backward_workspace_bytes(cfg: Config, H: int, W: int) -> int:
    n = lib().bsf_backward_workspace_bytes(ctypes.byref(cfg.c()), int(H), int(W))
    if n == 0:
        raise BsfError(E_INVALID, "bsf_backward_workspace_bytes")
    return n


def filter_backward(cfg: Config, steps: torch.Tensor, gout: torch.Tensor, dsteps: Optional[torch.Tensor] = None,
                    want_img: bool = True, want_steps: bool = True, ws: Optional[Workspace] = None,
                    grad_img: Optional[torch.Tensor] = None, grad_steps: Optional[torch.Tensor] = None):
    """Adjoint: returns (grad_img or None, grad_steps or None).  grad_steps
    needs dsteps (d out / d steps from the forward call).  Output tensors may
    be passed in (grad_img / grad_steps); otherwise they are allocated."""
    _, H, W = steps.shape
    _check_steps(cfg, steps, H, W)
    if gout.dtype != torch.float32 or not gout.is_contiguous() or tuple(gout.shape) != (H, W):
        raise ValueError("gout must be a contiguous float32 [H][W] device tensor")
    dev = steps.device
    gi = gs = None
    if want_img:
        gi = grad_img if grad_img is not None else torch.empty((H, W), dtype=torch.float32, device=dev)
        if gi.dtype != torch.float32 or not gi.is_contiguous() or tuple(gi.shape) != (H, W):
            raise ValueError("grad_img must be a contiguous float32 [H][W] device tensor")
    if want_steps:
        gs = grad_steps if grad_steps is not None else torch.empty_like(steps)
        _check_steps(cfg, gs, H, W)
    need = backward_workspace_bytes(cfg, H, W)
    ws = ws or _workspace(dev, need)
    ws.ensure(need)
    _check(lib().bsf_filter_backward(ctypes.byref(cfg.c()), H, W, _ptr(steps), _ptr(gout), _ptr(dsteps), _ptr(gi),
                                     _ptr(gs), ws.ptr(), ws.nbytes, _stream(dev)),
           "bsf_filter_backward")
    return gi, gs


def set_tuning(gather_wx: int, line_tl: int):
    """Launch shapes of the tied order-2 gather and the sheared running sums
    (process-wide; results do not depend on them)."""
    _check(lib().bsf_set_tuning(int(gather_wx), int(line_tl)), "bsf_set_tuning")


def set_box_tile(tile_h: int):
    """Tile height (4 or 8) of the tied order-2 cluster-box gather (process-wide;
    results do not depend on it)."""
    _check(lib().bsf_set_box_tile(int(tile_h)), "bsf_set_box_tile")


def get_box_tile() -> int:
    return int(lib().bsf_get_box_tile())


def get_tuning() -> Tuple[int, int]:
    wx, tl = ctypes.c_int32(), ctypes.c_int32()
    lib().bsf_get_tuning(ctypes.byref(wx), ctypes.byref(tl))
    return wx.value, tl.value


class Batch:
    """A fixed set of FP32 images, step fields and outputs filtered together
    by bsf_filter_batched.  The descriptors and the workspace stay the same
    between runs, so with use_graph the launches are recorded once and
    replayed."""

    def __init__(self, cfg: Config, imgs: Sequence[torch.Tensor], steps: Sequence[torch.Tensor],
                 outs: Optional[Sequence[torch.Tensor]] = None):
        if len(imgs) != len(steps):
            raise ValueError("one step field per image")
        self.cfg = cfg
        self.imgs, self.steps = list(imgs), list(steps)
        dev = self.imgs[0].device if self.imgs else torch.device("cuda")
        for im, st in zip(self.imgs, self.steps):
            _check_image(im)
            if im.dtype != torch.float32:
                raise TypeError("batched images are float32")
            _check_steps(cfg, st, *im.shape)
        if outs is None:
            outs = [torch.empty(tuple(im.shape), dtype=torch.float32, device=dev) for im in self.imgs]
        self.outs = list(outs)
        for im, o in zip(self.imgs, self.outs):
            if o.dtype != torch.float32 or not o.is_contiguous() or o.shape != im.shape:
                raise ValueError("outputs are contiguous float32 tensors of the images' shapes")
        B = len(self.imgs)
        self.descs = (_ImageDesc * max(B, 1))()
        for b, (im, st, o) in enumerate(zip(self.imgs, self.steps, self.outs)):
            d = self.descs[b]
            d.img, d.steps, d.out = im.data_ptr(), st.data_ptr(), o.data_ptr()
            d.H, d.W = im.shape[0], im.shape[1]
            d.pitch = _pitch(im)
        self.B = B
        self._cfg_c = cfg.c()
        need = lib().bsf_batched_workspace_bytes(ctypes.byref(self._cfg_c), B, self.descs)
        if need == 0:
            raise BsfError(E_INVALID, "bsf_batched_workspace_bytes")
        self.ws = Workspace(need, dev)

    def run(self, use_graph: bool = True):
        _check(lib().bsf_filter_batched(ctypes.byref(self._cfg_c), self.B, self.descs, self.ws.ptr(),
                                        self.ws.nbytes, _stream(self.ws.buf.device), int(bool(use_graph))),
               "bsf_filter_batched")
        return self.outs


def filter_batched(cfg: Config, imgs: Sequence[torch.Tensor], steps: Sequence[torch.Tensor],
                   use_graph: bool = False):
    """One-shot batched forward; returns the list of outputs."""
    return Batch(cfg, imgs, steps).run(use_graph)


class DeviceFlagError(RuntimeError):
    """A checked call found device status flags (FLAG_*) raised."""

    def __init__(self, flags, what):
        self.flags = flags
        names = [n for n, b in (("RANGE", FLAG_RANGE), ("OVERFLOW", FLAG_OVERFLOW),
                                ("NONFINITE", FLAG_NONFINITE)) if flags & b]
        super().__init__("%s: device flags %s" % (what, "|".join(names) or hex(flags)))


def check_flags(ws: Workspace, what: str = "bsf"):
    """Synchronises, reads and clears the workspace's sticky flags, and raises
    DeviceFlagError if any is set (a step out of range or NaN, a fixed-point
    overflow, or a non-finite image sample or upstream gradient)."""
    flags, _, _ = ws.status(clear=True)
    if flags:
        raise DeviceFlagError(flags, what)


class _Filter(torch.autograd.Function):
    """out = space-variant box-spline filter of img with per-pixel steps.  The
    forward keeps d out / d steps (the filter is local in its steps); the
    backward scatters the upstream gradient through the transposed taps and
    running sums for the image."""

    @staticmethod
    def forward(ctx, img, steps, cfg, check):
        need_s = ctx.needs_input_grad[1]
        ds = torch.empty_like(steps) if need_s else None
        H, W = img.shape
        ws = _workspace(img.device, plan(cfg, H, W).workspace_bytes)
        if check:
            ws.status(clear=True)
        out = filter_varying(cfg, img, steps, dsteps=ds, ws=ws)
        if check:
            check_flags(ws, "filter forward")
        ctx.cfg = cfg
        ctx.check = check
        ctx.save_for_backward(steps, ds if need_s else steps)
        ctx.has_ds = need_s
        return out

    @staticmethod
    def backward(ctx, gout):
        steps, ds = ctx.saved_tensors
        _, H, W = steps.shape
        ws = _workspace(steps.device, backward_workspace_bytes(ctx.cfg, H, W))
        if ctx.check:
            ws.status(clear=True)
        gi, gs = filter_backward(ctx.cfg, steps, gout.contiguous(), dsteps=ds if ctx.has_ds else None,
                                 want_img=ctx.needs_input_grad[0], want_steps=ctx.has_ds, ws=ws)
        if ctx.check:
            check_flags(ws, "filter backward")
        return gi, gs, None, None


def filter(img: torch.Tensor, steps: torch.Tensor, cfg: Config, check: bool = False) -> torch.Tensor:
    """Differentiable space-variant filter (continuous steps, float32 image).

    Steps outside [1, max_step] (or NaN) are clamped on the device and raise
    FLAG_RANGE; their step derivative is that of the clamped step.  A NaN or
    infinite image sample or upstream gradient raises FLAG_NONFINITE (and makes
    the image gradient NaN).  With check=True the forward and the backward
    each read the flags (a synchronisation) and raise DeviceFlagError; without
    it the caller reads them through Workspace.status()."""
    if cfg.mode != STEPS_REAL or img.dtype != torch.float32:
        raise ValueError("the differentiable filter takes a float32 image and continuous steps")
    return _Filter.apply(img, steps, cfg, bool(check))


def version():
    return lib().bsf_version().decode()
