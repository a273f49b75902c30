"""Python binding of libstokes2d (free-space 2D Stokes layer potentials with
periodic near images, hand-written HIP for MI355X / gfx950).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every arithmetic step runs in the library's kernels.  The functions
keep the C names (include/stokes2d.h):

    stokes2d_init(device)
    stokes2d_workspace_size(op, mode, src, trg)
    stokes2d_slp_eval(mode, src, trg, d, img_lo, img_hi, mu, u, v, accumulate, ws, stream)
    stokes2d_dlp_eval(mode, src, trg, d, img_lo, img_hi, u, v, accumulate, ws, stream)

`Curves` / `Targets` hold the device tensors of a curve set and a target set.
Loading fails loudly if the compiled library is missing: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "S2D_OK", "S2D_FP64", "S2D_FP32C", "S2D_OP_SLP", "S2D_OP_DLP", "S2DError",
    "Curves", "Targets", "lib", "library_path",
    "stokes2d_init", "stokes2d_workspace_size", "stokes2d_slp_eval", "stokes2d_slp_eval_noalloc",
    "stokes2d_dlp_eval",
    "stokes2d_last_error", "stokes2d_version", "stokes2d_profile_enable", "stokes2d_profile_read",
    "BatchInstance", "stokes2d_batch_workspace_size", "stokes2d_batch_eval", "stokes2d_batch_release",
    "stokes2d_batch_tuned", "S2D_OP_SLP_PRESSURE", "S2D_OP_DLP_PRESSURE", "S2D_OP_SLP_TRACTION",
    "stokes2d_slp_pressure_eval", "stokes2d_dlp_pressure_eval", "stokes2d_slp_traction_eval",
]

S2D_OK, S2D_EINVAL, S2D_EHIP, S2D_ENOTSUP, S2D_EWORKSPACE, S2D_ENOINIT = 0, -1, -2, -3, -4, -5
S2D_FP64, S2D_FP32C = 0, 1
S2D_OP_SLP, S2D_OP_DLP, S2D_OP_SLP_PRESSURE, S2D_OP_DLP_PRESSURE, S2D_OP_SLP_TRACTION = 0, 1, 2, 3, 4

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libstokes2d.so")


class S2DError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libstokes2d error {code}: {msg}")
        self.code = code


class _Curves(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_curves", ctypes.c_int32),
                ("curve_off", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("nx", ctypes.c_void_p), ("ny", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("kappa", ctypes.c_void_p),
                ("fx", ctypes.c_void_p), ("fy", ctypes.c_void_p)]


class _Targets(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("on_curve", ctypes.c_void_p), ("on_node", ctypes.c_void_p)]


class _Instance(ctypes.Structure):
    _fields_ = [("ves", _Curves), ("wall", _Curves), ("trg_ves", _Targets), ("trg_wall", _Targets),
                ("d", ctypes.c_double), ("mu", ctypes.c_double),
                ("u", ctypes.c_void_p), ("v", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded libstokes2d.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise ImportError(f"{library_path} is missing: build it with "
                              "`python -m paper_1510_05616_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(library_path)
        P, I, I32, I64, D, SZ = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int32,
                                 ctypes.c_int64, ctypes.c_double, ctypes.c_size_t)
        L.stokes2d_init.argtypes = [I]
        L.stokes2d_init.restype = I
        L.stokes2d_workspace_size.argtypes = [I, I, P, P]
        L.stokes2d_workspace_size.restype = SZ
        L.stokes2d_slp_eval.argtypes = [I, P, P, D, I32, I32, D, P, P, I, P, SZ, P]
        L.stokes2d_slp_eval.restype = I
        L.stokes2d_slp_eval_noalloc.argtypes = [I, P, P, D, I32, I32, D, P, P, I, P]
        L.stokes2d_slp_eval_noalloc.restype = I
        L.stokes2d_dlp_eval.argtypes = [I, P, P, D, I32, I32, P, P, I, P, SZ, P]
        L.stokes2d_dlp_eval.restype = I
        L.stokes2d_slp_pressure_eval.argtypes = [I, P, P, D, I32, I32, P, I, P, SZ, P]
        L.stokes2d_slp_pressure_eval.restype = I
        L.stokes2d_dlp_pressure_eval.argtypes = [I, P, P, D, I32, I32, D, P, I, P, SZ, P]
        L.stokes2d_dlp_pressure_eval.restype = I
        L.stokes2d_slp_traction_eval.argtypes = [I, P, P, P, P, D, I32, I32, P, P, I, P, SZ, P]
        L.stokes2d_slp_traction_eval.restype = I
        L.stokes2d_last_error.argtypes = []
        L.stokes2d_last_error.restype = ctypes.c_char_p
        L.stokes2d_version.argtypes = []
        L.stokes2d_version.restype = I
        L.stokes2d_batch_workspace_size.argtypes = [I, I32, P]
        L.stokes2d_batch_workspace_size.restype = SZ
        L.stokes2d_batch_eval.argtypes = [I, I32, P, P, SZ, P]
        L.stokes2d_batch_eval.restype = I
        L.stokes2d_batch_release.argtypes = []
        L.stokes2d_batch_release.restype = I
        L.stokes2d_batch_tuned.argtypes = [I, I32, P, P, P, P]
        L.stokes2d_batch_tuned.restype = I
        L.stokes2d_profile_enable.argtypes = [I]
        L.stokes2d_profile_enable.restype = I
        L.stokes2d_profile_read.argtypes = [I, P, P]
        L.stokes2d_profile_read.restype = I
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_f64(a, device):
    import torch
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(a, dtype=torch.float64, device=device).contiguous()


def _dev_i32(a, device):
    import torch
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.int32).contiguous()
    return torch.as_tensor(a, dtype=torch.int32, device=device).contiguous()


class Curves:
    """Device copy of a curve set (any object with x, y, nx, ny, w, kappa, fx,
    fy, curve_off arrays, e.g. synth.CurveSet)."""

    def __init__(self, cs, device="cuda"):
        self.device = device
        for k in ("x", "y", "nx", "ny", "w", "kappa", "fx", "fy"):
            setattr(self, k, _dev_f64(getattr(cs, k, None), device))
        self.curve_off = _dev_i32(cs.curve_off, device)
        self.n_nodes = int(self.x.shape[0])
        self.n_curves = int(self.curve_off.shape[0]) - 1

    def struct(self):
        return _Curves(self.n_nodes, self.n_curves, _ptr(self.curve_off), _ptr(self.x), _ptr(self.y),
                       _ptr(self.nx), _ptr(self.ny), _ptr(self.w), _ptr(self.kappa),
                       _ptr(self.fx), _ptr(self.fy))


class Targets:
    """Device copy of targets; on_curve/on_node optional (both or neither)."""

    def __init__(self, x, y, on_curve=None, on_node=None, device="cuda"):
        self.x = _dev_f64(x, device)
        self.y = _dev_f64(y, device)
        self.on_curve = _dev_i32(on_curve, device)
        self.on_node = _dev_i32(on_node, device)
        self.n = int(self.x.shape[0])

    def struct(self):
        return _Targets(self.n, _ptr(self.x), _ptr(self.y), _ptr(self.on_curve), _ptr(self.on_node))


def _check(rc):
    if rc != S2D_OK:
        raise S2DError(rc, stokes2d_last_error())


def stokes2d_last_error() -> str:
    m = lib().stokes2d_last_error()
    return m.decode() if m else ""


def stokes2d_version() -> int:
    return int(lib().stokes2d_version())


def stokes2d_profile_enable(on: bool) -> None:
    _check(lib().stokes2d_profile_enable(int(bool(on))))


def stokes2d_profile_read(op: int):
    """(total milliseconds, launch count) of the pair kernels of op recorded
    since the last read."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().stokes2d_profile_read(int(op), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def stokes2d_init(device: int = 0) -> None:
    _check(lib().stokes2d_init(int(device)))


def stokes2d_workspace_size(op: int, mode: int, src: Curves, trg: Targets) -> int:
    cs, ts = src.struct(), trg.struct()
    return int(lib().stokes2d_workspace_size(int(op), int(mode), ctypes.byref(cs), ctypes.byref(ts)))


def _workspace(nbytes, device, ws):
    import torch
    if ws is not None:
        return ws
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def stokes2d_slp_eval(mode, src: Curves, trg: Targets, d, img_lo, img_hi, mu, u, v,
                      accumulate=0, ws=None, stream=None) -> None:
    """u, v: device float64 tensors of length trg.n (written, or added to)."""
    cs, ts = src.struct(), trg.struct()
    ws = _workspace(stokes2d_workspace_size(S2D_OP_SLP, mode, src, trg), u.device, ws)
    _check(lib().stokes2d_slp_eval(int(mode), ctypes.byref(cs), ctypes.byref(ts), float(d),
                                   int(img_lo), int(img_hi), float(mu), _ptr(u), _ptr(v),
                                   int(bool(accumulate)), _ptr(ws), ws.numel(), _stream(stream)))


def stokes2d_slp_eval_noalloc(mode, src: Curves, trg: Targets, d, img_lo, img_hi, mu, u, v,
                              accumulate=0, stream=None) -> None:
    """stokes2d_slp_eval without a workspace (the library's per-device scratch
    memory; no allocation on this path)."""
    cs, ts = src.struct(), trg.struct()
    _check(lib().stokes2d_slp_eval_noalloc(int(mode), ctypes.byref(cs), ctypes.byref(ts), float(d),
                                           int(img_lo), int(img_hi), float(mu), _ptr(u), _ptr(v),
                                           int(bool(accumulate)), _stream(stream)))


def stokes2d_dlp_eval(mode, src: Curves, trg: Targets, d, img_lo, img_hi, u, v,
                      accumulate=0, ws=None, stream=None) -> None:
    cs, ts = src.struct(), trg.struct()
    ws = _workspace(stokes2d_workspace_size(S2D_OP_DLP, mode, src, trg), u.device, ws)
    _check(lib().stokes2d_dlp_eval(int(mode), ctypes.byref(cs), ctypes.byref(ts), float(d),
                                   int(img_lo), int(img_hi), _ptr(u), _ptr(v),
                                   int(bool(accumulate)), _ptr(ws), ws.numel(), _stream(stream)))


def stokes2d_slp_pressure_eval(mode, src: Curves, trg: Targets, d, img_lo, img_hi, p,
                               accumulate=0, ws=None, stream=None) -> None:
    """Single-layer pressure at free targets (trg without on-curve
    references); p: device float64 tensor of length trg.n."""
    cs, ts = src.struct(), trg.struct()
    ws = _workspace(stokes2d_workspace_size(S2D_OP_SLP_PRESSURE, mode, src, trg), p.device, ws)
    _check(lib().stokes2d_slp_pressure_eval(int(mode), ctypes.byref(cs), ctypes.byref(ts), float(d), int(img_lo),
                                            int(img_hi), _ptr(p), int(bool(accumulate)), _ptr(ws), ws.numel(),
                                            _stream(stream)))


def stokes2d_dlp_pressure_eval(mode, src: Curves, trg: Targets, d, img_lo, img_hi, mu, p,
                               accumulate=0, ws=None, stream=None) -> None:
    """Double-layer pressure at free targets."""
    cs, ts = src.struct(), trg.struct()
    ws = _workspace(stokes2d_workspace_size(S2D_OP_DLP_PRESSURE, mode, src, trg), p.device, ws)
    _check(lib().stokes2d_dlp_pressure_eval(int(mode), ctypes.byref(cs), ctypes.byref(ts), float(d), int(img_lo),
                                            int(img_hi), float(mu), _ptr(p), int(bool(accumulate)), _ptr(ws),
                                            ws.numel(), _stream(stream)))


def stokes2d_slp_traction_eval(mode, src: Curves, trg: Targets, nx, ny, d, img_lo, img_hi, tx, ty,
                               accumulate=0, ws=None, stream=None) -> None:
    """Single-layer traction at free targets with unit normals nx, ny
    (device float64 tensors of length trg.n)."""
    cs, ts = src.struct(), trg.struct()
    ws = _workspace(stokes2d_workspace_size(S2D_OP_SLP_TRACTION, mode, src, trg), tx.device, ws)
    _check(lib().stokes2d_slp_traction_eval(int(mode), ctypes.byref(cs), ctypes.byref(ts), _ptr(nx), _ptr(ny),
                                            float(d), int(img_lo), int(img_hi), _ptr(tx), _ptr(ty),
                                            int(bool(accumulate)), _ptr(ws), ws.numel(), _stream(stream)))


class BatchInstance:
    """One channel instance of a batched evaluation: vesicle curves (single
    layer), wall curves (double layer), the target points with their on-curve
    references to each set, period d, viscosity mu and the outputs u, v."""

    def __init__(self, ves: Curves, wall: Curves, trg_ves: Targets, trg_wall: Targets, d, mu, u, v):
        self.ves, self.wall, self.trg_ves, self.trg_wall = ves, wall, trg_ves, trg_wall
        self.d, self.mu, self.u, self.v = float(d), float(mu), u, v

    def struct(self):
        return _Instance(self.ves.struct(), self.wall.struct(), self.trg_ves.struct(), self.trg_wall.struct(),
                         self.d, self.mu, _ptr(self.u), _ptr(self.v))


def _inst_array(instances):
    arr = (_Instance * max(len(instances), 1))()
    for i, b in enumerate(instances):
        arr[i] = b.struct()
    return arr


def stokes2d_batch_workspace_size(mode, instances) -> int:
    arr = _inst_array(instances)
    return int(lib().stokes2d_batch_workspace_size(int(mode), len(instances), arr))


def stokes2d_batch_eval(mode, instances, ws, stream=None) -> None:
    """ws: a device uint8 tensor of at least stokes2d_batch_workspace_size()
    bytes; keep passing the same one so repeated calls replay the cached graph."""
    arr = _inst_array(instances)
    _check(lib().stokes2d_batch_eval(int(mode), len(instances), arr, _ptr(ws), ws.numel(), _stream(stream)))


def stokes2d_batch_release() -> None:
    _check(lib().stokes2d_batch_release())


def stokes2d_batch_tuned(mode, instances) -> dict:
    """The tile shape the batched call uses for these instances' size bucket
    and whether it came from the tuner (True) or is the default (False)."""
    arr = _inst_array(instances)
    t, b, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    rc = lib().stokes2d_batch_tuned(int(mode), len(instances), arr, ctypes.byref(t), ctypes.byref(b),
                                    ctypes.byref(w))
    if rc < 0:
        _check(rc)
    return {"targets_per_lane": t.value, "superblocks_per_split": b.value, "waves_per_cu": w.value,
            "tuned": rc == 1}
