"""Binding of the near-field correction entry points of libstokes2d, and the
training loop of the near-field MLP.

This module only orchestrates library calls: labels come from the library's
FFT-upsampled FP64 quadrature, features from its feature kernel, every
training step (forward, backward, gradient sums, Adam) from its training
kernels, and the BF16 inference blob from its packing kernel.  torch supplies
device memory, the minibatch permutation and the per-bin statistics of the
calibration.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import (Curves, Targets, _check, _ptr, _stream, lib)

S2D_NEAR_UPSAMPLE, S2D_NEAR_MLP, S2D_NEAR_AUTO = 0, 1, 2
NFEAT = 20
NPARAM = 9834
# offsets in the FP32 master parameter vector
OFF = dict(mu=0, sd=20, W1=40, b1=1320, W2=1384, b2=5480, W3=5544, b3=9640, W4=9704, b4=9832)
SHAPES = dict(W1=(20, 64), b1=(64,), W2=(64, 64), b2=(64,), W3=(64, 64), b3=(64,), W4=(64, 2), b4=(2,))
BIN_LO, BIN_W, N_BINS = math.log10(0.05), 2.0 / 64, 64   # bins of log10(|normal offset| / h)

_bound = False


def _bind():
    global _bound
    L = lib()
    if _bound:
        return L
    P, I, I32, I64, D, F, SZ = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int32, ctypes.c_int64,
                                ctypes.c_double, ctypes.c_float, ctypes.c_size_t)
    L.near_workspace_size.argtypes = [I, P, P, I32]
    L.near_workspace_size.restype = SZ
    L.near_correct_eval.argtypes = [I, P, P, P, I32, P, D, D, P, P, P, P, SZ, P]
    L.near_correct_eval.restype = I
    L.near_upsampled_slp_workspace_size.argtypes = [P, P, I32]
    L.near_upsampled_slp_workspace_size.restype = SZ
    L.near_upsampled_slp.argtypes = [P, P, P, I32, D, P, P, P, P, P, SZ, P]
    L.near_upsampled_slp.restype = I
    L.near_features_eval.argtypes = [P, P, P, P, P, P]
    L.near_features_eval.restype = I
    L.near_scale_labels.argtypes = [I64, P, P, P, D, P, P]
    L.near_scale_labels.restype = I
    L.near_mlp_train_workspace_size.argtypes = [I32]
    L.near_mlp_train_workspace_size.restype = SZ
    L.near_mlp_train_step.argtypes = [I32, P, P, P, P, P, P, I32, F, P, P, P, SZ, P]
    L.near_mlp_train_step.restype = I
    L.near_mlp_forward.argtypes = [I64, P, P, P, P]
    L.near_mlp_forward.restype = I
    L.near_mlp_blob_size.argtypes = []
    L.near_mlp_blob_size.restype = SZ
    L.near_mlp_pack.argtypes = [P, P, P, I32, F, F, P, P]
    L.near_mlp_pack.restype = I
    L.stokes2d_wall_upsample_workspace_size.argtypes = [P, I32]
    L.stokes2d_wall_upsample_workspace_size.restype = SZ
    L.stokes2d_wall_upsample.argtypes = [P, D, I32, P, P, P, P, P, P, P, P, P, SZ, P]
    L.stokes2d_wall_upsample.restype = I
    L.near_wall_workspace_size.argtypes = [I, P, P, I32]
    L.near_wall_workspace_size.restype = SZ
    L.near_wall_correct_eval.argtypes = [I, P, P, P, D, I32, I32, I32, P, D, P, P, P, I, P, SZ, P]
    L.near_wall_correct_eval.restype = I
    L.near_wall_features_eval.argtypes = [P, P, P, D, P, P, P]
    L.near_wall_features_eval.restype = I
    L.near_wall_scale_labels.argtypes = [I64, P, P, P, P, P]
    L.near_wall_scale_labels.restype = I
    _bound = True
    return L


def _empty(nbytes, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def near_workspace_size(method, ves: Curves, trg: Targets, upsample: int) -> int:
    L = _bind()
    cs, ts = ves.struct(), trg.struct()
    return int(L.near_workspace_size(int(method), ctypes.byref(cs), ctypes.byref(ts), int(upsample)))


def near_correct_eval(method, ves: Curves, trg: Targets, trg_curve, upsample, blob, threshold, mu, du, dv,
                      used_fallback=None, ws=None, stream=None) -> None:
    L = _bind()
    cs, ts = ves.struct(), trg.struct()
    if ws is None:
        ws = _empty(near_workspace_size(method, ves, trg, upsample), du.device)
    _check(L.near_correct_eval(int(method), ctypes.byref(cs), ctypes.byref(ts), _ptr(trg_curve), int(upsample),
                               _ptr(blob), float(threshold), float(mu), _ptr(du), _ptr(dv), _ptr(used_fallback),
                               _ptr(ws), ws.numel(), _stream(stream)))


def near_upsampled_slp(ves: Curves, trg: Targets, trg_curve, upsample, mu, u_up, v_up, u_trap, v_trap,
                       ws=None, stream=None) -> None:
    L = _bind()
    cs, ts = ves.struct(), trg.struct()
    if ws is None:
        ws = _empty(L.near_upsampled_slp_workspace_size(ctypes.byref(cs), ctypes.byref(ts), int(upsample)),
                    u_up.device)
    _check(L.near_upsampled_slp(ctypes.byref(cs), ctypes.byref(ts), _ptr(trg_curve), int(upsample), float(mu),
                                _ptr(u_up), _ptr(v_up), _ptr(u_trap), _ptr(v_trap), _ptr(ws), ws.numel(),
                                _stream(stream)))


def stokes2d_wall_upsample(walls: Curves, d, upsample, ws=None, stream=None) -> Curves:
    """The P-times refined wall curves (nodes, normals, weights, density and
    curve offsets computed by the library); kappa is left unset."""
    import types
    import torch
    L = _bind()
    cs = walls.struct()
    nf = int(upsample) * walls.n_nodes
    f64 = dict(dtype=torch.float64, device=walls.device)
    out = {k: torch.empty(nf, **f64) for k in ("x", "y", "nx", "ny", "w", "fx", "fy")}
    off = torch.empty(walls.n_curves + 1, dtype=torch.int32, device=walls.device)
    if ws is None:
        ws = _empty(L.stokes2d_wall_upsample_workspace_size(ctypes.byref(cs), int(upsample)), walls.device)
    _check(L.stokes2d_wall_upsample(ctypes.byref(cs), float(d), int(upsample), *(_ptr(out[k]) for k in
                                    ("x", "y", "nx", "ny", "w", "fx", "fy")), _ptr(off), _ptr(ws), ws.numel(),
                                    _stream(stream)))
    return Curves(types.SimpleNamespace(kappa=None, curve_off=off, **out), walls.device)


def near_wall_workspace_size(walls: Curves, trg: Targets, upsample: int, method=S2D_NEAR_UPSAMPLE) -> int:
    L = _bind()
    cs, ts = walls.struct(), trg.struct()
    return int(L.near_wall_workspace_size(int(method), ctypes.byref(cs), ctypes.byref(ts), int(upsample)))


def near_wall_correct_eval(walls: Curves, trg: Targets, d, img_lo, img_hi, upsample, du, dv, accumulate=0,
                           method=S2D_NEAR_UPSAMPLE, trg_curve=None, blob=None, threshold=0.0, used_fallback=None,
                           ws=None, stream=None) -> None:
    """du, dv (device float64, [trg.n]) = (or +=) D_P - D_1 of the walls:
    by the refined walls (UPSAMPLE), the network (MLP) or per target
    (AUTO; trg_curve names each target's wall)."""
    L = _bind()
    cs, ts = walls.struct(), trg.struct()
    if ws is None:
        ws = _empty(near_wall_workspace_size(walls, trg, upsample, method), du.device)
    _check(L.near_wall_correct_eval(int(method), ctypes.byref(cs), ctypes.byref(ts), _ptr(trg_curve), float(d),
                                    int(img_lo), int(img_hi), int(upsample), _ptr(blob), float(threshold), _ptr(du),
                                    _ptr(dv), _ptr(used_fallback), int(accumulate), _ptr(ws), ws.numel(),
                                    _stream(stream)))


def near_wall_features_eval(walls: Curves, trg: Targets, trg_curve, d, X, frame, stream=None) -> None:
    L = _bind()
    cs, ts = walls.struct(), trg.struct()
    _check(L.near_wall_features_eval(ctypes.byref(cs), ctypes.byref(ts), _ptr(trg_curve), float(d), _ptr(X),
                                     _ptr(frame), _stream(stream)))


def near_wall_scale_labels(du, dv, frame, Y, stream=None) -> None:
    _check(_bind().near_wall_scale_labels(int(du.shape[0]), _ptr(du), _ptr(dv), _ptr(frame), _ptr(Y),
                                          _stream(stream)))


def near_features_eval(ves: Curves, trg: Targets, trg_curve, X, frame, stream=None) -> None:
    L = _bind()
    cs, ts = ves.struct(), trg.struct()
    _check(L.near_features_eval(ctypes.byref(cs), ctypes.byref(ts), _ptr(trg_curve), _ptr(X), _ptr(frame),
                                _stream(stream)))


def near_scale_labels(du, dv, frame, mu, Y, stream=None) -> None:
    L = _bind()
    _check(L.near_scale_labels(du.numel(), _ptr(du), _ptr(dv), _ptr(frame), float(mu), _ptr(Y), _stream(stream)))


def near_mlp_train_workspace_size(batch: int) -> int:
    return int(_bind().near_mlp_train_workspace_size(int(batch)))


def near_mlp_train_step(batch, idx, X, Y, params, m, v, step, lr, grad, loss, ws, stream=None) -> None:
    L = _bind()
    _check(L.near_mlp_train_step(int(batch), _ptr(idx), _ptr(X), _ptr(Y), _ptr(params), _ptr(m), _ptr(v),
                                 int(step), float(lr), _ptr(grad), _ptr(loss), _ptr(ws), ws.numel(),
                                 _stream(stream)))


def near_mlp_forward(X, params, Y, stream=None) -> None:
    L = _bind()
    _check(L.near_mlp_forward(X.shape[0], _ptr(X), _ptr(params), _ptr(Y), _stream(stream)))


def near_mlp_blob_size() -> int:
    return int(_bind().near_mlp_blob_size())


def near_mlp_pack(params, bound, n_bins, bin_lo, bin_w, blob, bound_zero=None, stream=None) -> None:
    L = _bind()
    _check(L.near_mlp_pack(_ptr(params), _ptr(bound), _ptr(bound_zero), int(n_bins), float(bin_lo), float(bin_w),
                           _ptr(blob), _stream(stream)))


# ----------------------------------------------------------------------------
# parameters
# ----------------------------------------------------------------------------
def params_to_dict(p: np.ndarray) -> dict:
    p = np.asarray(p, dtype=np.float64)
    d = {"mu_in": p[0:20].copy(), "sd_in": p[20:40].copy()}
    for k, shp in SHAPES.items():
        n = int(np.prod(shp))
        d[k] = p[OFF[k]:OFF[k] + n].reshape(shp).copy()
    return d


def dict_to_params(d: dict) -> np.ndarray:
    p = np.zeros(NPARAM)
    p[0:20] = d["mu_in"]
    p[20:40] = d["sd_in"]
    for k, shp in SHAPES.items():
        n = int(np.prod(shp))
        p[OFF[k]:OFF[k] + n] = np.asarray(d[k]).reshape(-1)
    return p


def init_params(mu_in, sd_in, seed=0) -> np.ndarray:
    rng = np.random.default_rng([seed, 2])
    d = {"mu_in": np.asarray(mu_in, float), "sd_in": np.asarray(sd_in, float)}
    for k, shp in SHAPES.items():
        d[k] = rng.normal(size=shp) * math.sqrt(2.0 / shp[0]) if k.startswith("W") else np.zeros(shp)
    return dict_to_params(d)


# ----------------------------------------------------------------------------
# data and training
# ----------------------------------------------------------------------------
class NearData:
    """Device copy of a near-field dataset with its features, frames and
    (optionally) FP64 upsampled labels."""

    def __init__(self, curves, tx, ty, tc, mu=1.0, upsample=8, labels=True, device="cuda"):
        import torch
        self.curves = Curves(curves, device)
        self.trg = Targets(tx, ty, device=device)
        self.tc = torch.as_tensor(np.ascontiguousarray(tc, dtype=np.int32), device=device)
        self.n = self.trg.n
        self.mu = mu
        self.P = upsample
        self.X = torch.empty((self.n, NFEAT), dtype=torch.float32, device=device)
        self.frame = torch.empty((self.n, 6), dtype=torch.float64, device=device)
        near_features_eval(self.curves, self.trg, self.tc, self.X, self.frame)
        self.du = self.dv = self.Y = None
        if labels:
            self.du = torch.empty(self.n, dtype=torch.float64, device=device)
            self.dv = torch.empty_like(self.du)
            near_correct_eval(S2D_NEAR_UPSAMPLE, self.curves, self.trg, self.tc, upsample, None, 0.0, mu,
                              self.du, self.dv)
            self.Y = torch.empty((self.n, 2), dtype=torch.float32, device=device)
            near_scale_labels(self.du, self.dv, self.frame, mu, self.Y)

    def correct(self, method, blob, threshold, du, dv, used_fallback=None):
        near_correct_eval(method, self.curves, self.trg, self.tc, self.P, blob, threshold, self.mu, du, dv,
                          used_fallback)


# the walls' labels are scaled by pi / F; with the frame's length factor 1
# this is the single layer's 4 pi mu / (h F) at mu = 1/4, so the training,
# error and calibration helpers serve both
WALL_MU = 0.25


class WallNearData:
    """Near-wall dataset: targets near periodic walls (trg_curve naming each
    one's wall), their features and frames, and (optionally) FP64 labels from
    the refined-wall quadrature (images img_lo..img_hi of period d)."""

    def __init__(self, walls, d, tx, ty, tc, upsample=8, img=(-1, 1), labels=True, device="cuda"):
        import torch
        self.curves = Curves(walls, device)
        self.trg = Targets(tx, ty, device=device)
        self.tc = torch.as_tensor(np.ascontiguousarray(tc, dtype=np.int32), device=device)
        self.n = self.trg.n
        self.d, self.img = float(d), img
        self.mu = WALL_MU
        self.P = upsample
        self.X = torch.empty((self.n, NFEAT), dtype=torch.float32, device=device)
        self.frame = torch.empty((self.n, 6), dtype=torch.float64, device=device)
        near_wall_features_eval(self.curves, self.trg, self.tc, self.d, self.X, self.frame)
        self.du = self.dv = self.Y = None
        if labels:
            self.du = torch.empty(self.n, dtype=torch.float64, device=device)
            self.dv = torch.empty_like(self.du)
            near_wall_correct_eval(self.curves, self.trg, self.d, img[0], img[1], upsample, self.du, self.dv)
            self.Y = torch.empty((self.n, 2), dtype=torch.float32, device=device)
            near_wall_scale_labels(self.du, self.dv, self.frame, self.Y)

    def correct(self, method, blob, threshold, du, dv, used_fallback=None):
        near_wall_correct_eval(self.curves, self.trg, self.d, self.img[0], self.img[1], self.P, du, dv,
                               method=method, trg_curve=self.tc, blob=blob, threshold=threshold,
                               used_fallback=used_fallback)


def train(data: NearData, epochs=60, batch=1024, lr=2e-3, lr_min=2e-5, seed=0, log=None):
    """Trains the MLP on data.X -> data.Y with the library's kernels; returns
    (params tensor, list of epoch losses)."""
    import torch
    dev = data.X.device
    Xc = data.X.double()
    mu_in = Xc.mean(0).cpu().numpy()
    sd_in = Xc.std(0).clamp_min(1e-6).cpu().numpy()
    params = torch.as_tensor(init_params(mu_in, sd_in, seed), dtype=torch.float32, device=dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    ws = _empty(near_mlp_train_workspace_size(batch), dev)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    n = data.n
    steps_per_epoch = n // batch
    total = max(1, epochs * steps_per_epoch)
    step = 0
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(device=dev, dtype=torch.int32)
        acc = 0.0
        for b in range(steps_per_epoch):
            step += 1
            frac = (step - 1) / total
            cur = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * frac))
            idx = perm[b * batch:(b + 1) * batch]
            near_mlp_train_step(batch, idx, data.X, data.Y, params, m, v, step, cur, grad, loss, ws)
            if b % 50 == 0:
                acc += float(loss.item())
        hist.append(acc / max(1, (steps_per_epoch + 49) // 50))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.3e}")
    return params, hist


def scaled_errors(data: NearData, du_pred, dv_pred):
    """Per-target error of a prediction in the scaled units of the labels."""
    import torch
    fr = data.frame
    sc = 4 * math.pi * data.mu / (fr[:, 4] * fr[:, 5])
    return torch.hypot(du_pred - data.du, dv_pred - data.dv) * sc


def calibrate(data: NearData, params, quantile=1.0, safety=1.5):
    """Per-bin error bounds on validation data (bins of log10 |normal
    offset| / h), in scaled units: the max (quantile 1) error of the BF16
    network and of no correction at all, times `safety`.  Returns (blob
    tensor, network bound, no-correction bound) (numpy arrays)."""
    import torch
    dev = data.X.device
    blob = torch.zeros(near_mlp_blob_size(), dtype=torch.uint8, device=dev)
    zero = torch.zeros(N_BINS, dtype=torch.float32, device=dev)
    near_mlp_pack(params, zero, N_BINS, BIN_LO, BIN_W, blob)
    du = torch.empty_like(data.du)
    dv = torch.empty_like(data.dv)
    data.correct(S2D_NEAR_MLP, blob, 0.0, du, dv)
    err = scaled_errors(data, du, dv).cpu().numpy()
    err0 = scaled_errors(data, torch.zeros_like(du), torch.zeros_like(dv)).cpu().numpy()
    noff = np.abs(data.X[:, 1].double().cpu().numpy())
    b = np.clip(np.floor((np.log10(np.maximum(noff, 1e-30)) - BIN_LO) / BIN_W).astype(int), 0, N_BINS - 1)
    bound = np.full(N_BINS, np.inf)
    bound0 = np.full(N_BINS, np.inf)
    for k in range(N_BINS):
        sel = b == k
        if sel.any():
            q = (lambda e: np.quantile(e, quantile)) if quantile < 1 else np.max
            bound[k] = q(err[sel]) * safety
            bound0[k] = q(err0[sel]) * safety
    cap = lambda a: torch.as_tensor(np.minimum(a, 3e38), dtype=torch.float32, device=dev)
    near_mlp_pack(params, cap(bound), N_BINS, BIN_LO, BIN_W, blob, bound_zero=cap(bound0))
    return blob, bound, bound0
