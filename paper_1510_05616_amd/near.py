"""Binding of the near-field correction entry points of libstokes2d, and the
training and calibration drivers of the learned correction.

This module only orchestrates library calls: labels come from the library's
FFT-upsampled FP64 quadrature, node derivatives, features and frames from its
kernels, training records (the straight-line part subtracted) from its
target kernel, every training step (forward, backward, gradient sums, Adam)
from its training kernels, the input standardisation and the calibrated
per-bin bounds from its statistics kernels, and the BF16 inference blob from
its packing kernel.  torch supplies device memory, the minibatch indices and
the error summaries the tests print.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import (Curves, Targets, _check, _ptr, _stream, lib)

S2D_NEAR_UPSAMPLE, S2D_NEAR_MLP, S2D_NEAR_AUTO = 0, 1, 2
S2D_OP_SLP, S2D_OP_DLP = 0, 1
NFEAT = 14           # geometry features per target
NFRAME = 20          # FP64 frame words per target
NDERIV = 10          # FP64 derivative-table words per node
TSTRIDE = 14         # FP32 training-record words per sample
NOUT = 20            # network outputs dC[p][out][in]
NPARAM = 10608
# offsets in the FP32 master parameter vector
OFF = dict(mu=0, sd=14, W1=28, b1=924, W2=988, b2=5084, W3=5148, b3=9244, W4=9308, b4=10588)
SHAPES = dict(W1=(14, 64), b1=(64,), W2=(64, 64), b2=(64,), W3=(64, 64), b3=(64,), W4=(64, 20), b4=(20,))
# AUTO's bins: log10 b (b the normal offset in units of the local spacing),
# each split into CELL cells of |s| (S_BINS of width 1/8, the last, |s| >= 1/2,
# open: calibration never admits the learned route there) and
# log10 |kappa h| (K_BINS of width 3/16 from -2, both ends open): tables of
# N_BINS * CELL entries
B_MIN = 0.05
BIN_LO, BIN_W, N_BINS = math.log10(B_MIN), 2.0 / 32, 32
S_BINS, K_BINS = 5, 8
CELL = S_BINS * K_BINS
B_MAX = 10.0 ** (BIN_LO + N_BINS * BIN_W)    # the last bin's upper edge (5.0)


def table_index(b, s, kh, n_bins=N_BINS, bin_lo=BIN_LO, bin_w=BIN_W):
    """AUTO's table entry of targets (numpy, FP32 like the kernels; -1
    below the first b bin, the last b bin's cells past it)."""
    f = np.float32
    pos = np.floor((np.log10(np.asarray(b, f)) - f(bin_lo)) / f(bin_w))
    a = np.abs(np.asarray(s, f)) * f(8)
    j = np.where(a < S_BINS - 1, np.nan_to_num(a, nan=S_BINS - 1).astype(int), S_BINS - 1)
    k = (np.log10(np.abs(np.asarray(kh, f))) + f(2)) * f(16.0 / 3.0)
    m = np.where(k < 1, 0, np.where(k < K_BINS - 1, np.nan_to_num(k, nan=K_BINS - 1).astype(int), K_BINS - 1))
    kb = np.where(pos < n_bins, pos, n_bins - 1)
    return np.where(pos >= 0, kb * CELL + j * K_BINS + m, -1).astype(int)
WEIGHT_GAIN = 1e4    # constant factor on the loss weights (keeps the gradients well above Adam's eps)

_bound = False


def _bind():
    global _bound
    L = lib()
    if _bound:
        return L
    P, I, I32, I64, D, F, SZ = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int32, ctypes.c_int64,
                                ctypes.c_double, ctypes.c_float, ctypes.c_size_t)
    sig = {
        "near_workspace_size": ([I, P, P, I32], SZ),
        "near_correct_eval": ([I, P, P, P, I32, P, D, P, D, P, P, P, P, SZ, P], I),
        "near_upsampled_slp_workspace_size": ([P, P, I32], SZ),
        "near_upsampled_slp": ([P, P, P, I32, D, P, P, P, P, P, SZ, P], I),
        "near_derivs_workspace_size": ([P], SZ),
        "near_derivs_eval": ([P, P, P, SZ, P], I),
        "near_features_eval": ([P, P, P, P, P, P, P], I),
        "near_train_targets": ([I, I64, P, P, P, P, I32, P, P, D, I32, F, P, P, P], I),
        "near_mlp_train_workspace_size": ([I32], SZ),
        "near_mlp_train_step": ([I32, P, P, P, P, P, P, I32, F, P, P, P, SZ, P], I),
        "near_mlp_forward": ([I64, P, P, P, P], I),
        "near_feature_stats": ([I64, P, P, P], I),
        "near_calibrate": ([I, I64, P, P, P, P, P, D, I32, F, F, F, F, F, P, P, P, P], I),
        "near_mlp_blob_size": ([], SZ),
        "near_mlp_pack": ([P, P, P, I32, F, F, F, I32, P, P], I),
        "stokes2d_wall_upsample_workspace_size": ([P, I32], SZ),
        "stokes2d_wall_upsample": ([P, D, I32, P, P, P, P, P, P, P, P, P, SZ, P], I),
        "near_wall_workspace_size": ([I, P, P, I32], SZ),
        "near_wall_correct_eval": ([I, P, P, P, D, I32, I32, I32, P, D, P, P, P, P, I, P, SZ, P], I),
        "near_wall_features_eval": ([P, P, P, D, P, P, P, P], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _bound = True
    return L


def _empty(nbytes, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ----------------------------------------------------------------------------
# entry points
# ----------------------------------------------------------------------------
def near_workspace_size(method, ves: Curves, trg: Targets, upsample: int) -> int:
    L = _bind()
    cs, ts = ves.struct(), trg.struct()
    return int(L.near_workspace_size(int(method), ctypes.byref(cs), ctypes.byref(ts), int(upsample)))


def near_correct_eval(method, ves: Curves, trg: Targets, trg_curve, upsample, blob, threshold, mu, du, dv,
                      used_fallback=None, ws=None, stream=None, curve_tol=None) -> None:
    L = _bind()
    cs, ts = ves.struct(), trg.struct()
    if ws is None:
        ws = _empty(near_workspace_size(method, ves, trg, upsample), du.device)
    _check(L.near_correct_eval(int(method), ctypes.byref(cs), ctypes.byref(ts), _ptr(trg_curve), int(upsample),
                               _ptr(blob), float(threshold), _ptr(curve_tol), float(mu), _ptr(du), _ptr(dv),
                               _ptr(used_fallback), _ptr(ws), ws.numel(), _stream(stream)))


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


def near_derivs_eval(curves: Curves, dtab, ws=None, stream=None) -> None:
    """dtab [n_nodes, 10] device float64: the density's node derivatives."""
    L = _bind()
    cs = curves.struct()
    if ws is None:
        ws = _empty(L.near_derivs_workspace_size(ctypes.byref(cs)), dtab.device)
    _check(L.near_derivs_eval(ctypes.byref(cs), _ptr(dtab), _ptr(ws), ws.numel(), _stream(stream)))


def near_features_eval(ves: Curves, trg: Targets, trg_curve, dtab, X, frame, stream=None) -> None:
    L = _bind()
    cs, ts = ves.struct(), trg.struct()
    _check(L.near_features_eval(ctypes.byref(cs), ctypes.byref(ts), _ptr(trg_curve), _ptr(dtab), _ptr(X),
                                _ptr(frame), _stream(stream)))


def near_train_targets(op, frame, du, dv, trg_curve, n_curves, u_ref, v_ref, mu, upsample, curve_scale, T,
                       weight_gain=WEIGHT_GAIN, stream=None) -> None:
    _check(_bind().near_train_targets(int(op), int(frame.shape[0]), _ptr(frame), _ptr(du), _ptr(dv),
                                      _ptr(trg_curve), int(n_curves), _ptr(u_ref), _ptr(v_ref), float(mu),
                                      int(upsample), float(weight_gain), _ptr(curve_scale), _ptr(T),
                                      _stream(stream)))


def near_mlp_train_workspace_size(batch: int) -> int:
    return int(_bind().near_mlp_train_workspace_size(int(batch)))


def near_mlp_train_step(batch, idx, X, T, params, m, v, step, lr, grad, loss, ws, stream=None) -> None:
    L = _bind()
    _check(L.near_mlp_train_step(int(batch), _ptr(idx), _ptr(X), _ptr(T), _ptr(params), _ptr(m), _ptr(v),
                                 int(step), float(lr), _ptr(grad), _ptr(loss), _ptr(ws), ws.numel(),
                                 _stream(stream)))


def near_mlp_forward(X, params, Y, stream=None) -> None:
    L = _bind()
    _check(L.near_mlp_forward(X.shape[0], _ptr(X), _ptr(params), _ptr(Y), _stream(stream)))


def near_feature_stats(X, params, stream=None) -> None:
    _check(_bind().near_feature_stats(int(X.shape[0]), _ptr(X), _ptr(params), _stream(stream)))


def near_calibrate(op, frame, du_pred, dv_pred, du, dv, mu, n_bins, bin_lo, bin_w, b_min, margin, bound,
                   bound_zero, count, count_margin=0.0, stream=None) -> None:
    _check(_bind().near_calibrate(int(op), int(frame.shape[0]), _ptr(frame), _ptr(du_pred), _ptr(dv_pred),
                                  _ptr(du), _ptr(dv), float(mu), int(n_bins), float(bin_lo), float(bin_w),
                                  float(b_min), float(margin), float(count_margin), _ptr(bound), _ptr(bound_zero),
                                  _ptr(count), _stream(stream)))


def near_mlp_blob_size() -> int:
    return int(_bind().near_mlp_blob_size())


def near_mlp_pack(params, bound, n_bins, bin_lo, bin_w, blob, bound_zero=None, b_min=B_MIN, upsample=8,
                  stream=None) -> None:
    L = _bind()
    _check(L.near_mlp_pack(_ptr(params), _ptr(bound), _ptr(bound_zero), int(n_bins), float(bin_lo), float(bin_w),
                           float(b_min), int(upsample), _ptr(blob), _stream(stream)))


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
                           ws=None, stream=None, curve_tol=None) -> None:
    """du, dv (device float64, [trg.n]) = (or +=) D_P - D_1 of the walls:
    by the refined walls (UPSAMPLE), the learned route (MLP) or per target
    (AUTO; trg_curve names each target's wall)."""
    L = _bind()
    cs, ts = walls.struct(), trg.struct()
    if ws is None:
        ws = _empty(near_wall_workspace_size(walls, trg, upsample, method), du.device)
    _check(L.near_wall_correct_eval(int(method), ctypes.byref(cs), ctypes.byref(ts), _ptr(trg_curve), float(d),
                                    int(img_lo), int(img_hi), int(upsample), _ptr(blob), float(threshold),
                                    _ptr(curve_tol), _ptr(du), _ptr(dv), _ptr(used_fallback), int(accumulate),
                                    _ptr(ws), ws.numel(), _stream(stream)))


def near_wall_features_eval(walls: Curves, trg: Targets, trg_curve, d, dtab, X, frame, stream=None) -> None:
    L = _bind()
    cs, ts = walls.struct(), trg.struct()
    _check(L.near_wall_features_eval(ctypes.byref(cs), ctypes.byref(ts), _ptr(trg_curve), float(d), _ptr(dtab),
                                     _ptr(X), _ptr(frame), _stream(stream)))


# ----------------------------------------------------------------------------
# parameters
# ----------------------------------------------------------------------------
def params_to_dict(p: np.ndarray) -> dict:
    p = np.asarray(p, dtype=np.float64)
    d = {"mu_in": p[0:NFEAT].copy(), "sd_in": p[NFEAT:2 * NFEAT].copy()}
    for k, shp in SHAPES.items():
        n = int(np.prod(shp))
        d[k] = p[OFF[k]:OFF[k] + n].reshape(shp).copy()
    return d


def dict_to_params(d: dict) -> np.ndarray:
    p = np.zeros(NPARAM)
    p[0:NFEAT] = d["mu_in"]
    p[NFEAT:2 * NFEAT] = d["sd_in"]
    for k, shp in SHAPES.items():
        n = int(np.prod(shp))
        p[OFF[k]:OFF[k] + n] = np.asarray(d[k]).reshape(-1)
    return p


def init_weights(seed=0, last_scale=0.01) -> np.ndarray:
    """He-normal hidden weights, the output layer scaled by last_scale, zero
    biases; the standardisation slots are left 0 / 1 (near_feature_stats
    fills them)."""
    rng = np.random.default_rng([seed, 2])
    d = {"mu_in": np.zeros(NFEAT), "sd_in": np.ones(NFEAT)}
    for k, shp in SHAPES.items():
        if k.startswith("W"):
            d[k] = rng.normal(size=shp) * math.sqrt(2.0 / shp[0]) * (last_scale if k == "W4" else 1.0)
        else:
            d[k] = np.zeros(shp)
    return dict_to_params(d)


# ----------------------------------------------------------------------------
# data
# ----------------------------------------------------------------------------
class _NearSet:
    """Features, frames, labels and training records of near targets (the
    common part of the vesicle and wall data sets)."""
    op = S2D_OP_SLP

    def _finish(self, labels, weight_gain):
        import torch
        dev = self.X.device
        self.T = self.curve_scale = None
        if labels:
            self.curve_scale = torch.zeros(max(self.n_curves, 1), dtype=torch.float32, device=dev)
            self.T = torch.empty((self.n, TSTRIDE), dtype=torch.float32, device=dev)
            near_train_targets(self.op, self.frame, self.du, self.dv, self.tc, self.n_curves, self.u_ref,
                               self.v_ref, self.mu, self.P, self.curve_scale, self.T, weight_gain)

    @property
    def b(self):
        return self.frame[:, 1]

    def curve_tolerance(self, rel):
        """[n_curves] device float64: rel times each curve's largest |u_ref|
        (per-curve tolerances for AUTO in the normalised error measure)."""
        return self.curve_scale.double() * float(rel)

    def scaled_errors(self, du_pred, dv_pred):
        """Per-target |pred - label| over the largest |u_ref| of the target's
        curve (the normalised error of the learned correction)."""
        import torch
        cs = self.curve_scale.double()[self.tc.long().clamp(0, self.n_curves - 1)]
        return torch.hypot(du_pred - self.du, dv_pred - self.dv) / cs


class NearData(_NearSet):
    """Device copy of a near-field data set of targets near closed curves:
    node derivatives, features, frames and (labels=True) the FP64 upsampled
    quadrature's Delta, the P-times upsampled single layer u_ref of each
    target's own curve (the error measure's scale) and the training
    records."""
    op = S2D_OP_SLP

    def __init__(self, curves, tx, ty, tc, mu=1.0, upsample=8, labels=True, device="cuda",
                 weight_gain=WEIGHT_GAIN):
        import torch
        self.curves = Curves(curves, device)
        self.trg = Targets(tx, ty, device=device)
        self.tc = torch.as_tensor(np.ascontiguousarray(tc, dtype=np.int32), device=device)
        self.n = self.trg.n
        self.n_curves = self.curves.n_curves
        self.mu = mu
        self.P = upsample
        f64 = dict(dtype=torch.float64, device=device)
        self.dtab = torch.empty((max(self.curves.n_nodes, 1), NDERIV), **f64)
        near_derivs_eval(self.curves, self.dtab)
        self.X = torch.empty((self.n, NFEAT), dtype=torch.float32, device=device)
        self.frame = torch.empty((self.n, NFRAME), **f64)
        near_features_eval(self.curves, self.trg, self.tc, self.dtab, self.X, self.frame)
        self.du = self.dv = self.u_ref = self.v_ref = None
        if labels:
            self.du = torch.empty(self.n, **f64)
            self.dv = torch.empty_like(self.du)
            near_correct_eval(S2D_NEAR_UPSAMPLE, self.curves, self.trg, self.tc, upsample, None, 0.0, mu,
                              self.du, self.dv)
            self.u_ref, self.v_ref = torch.empty_like(self.du), torch.empty_like(self.du)
            u1, v1 = torch.empty_like(self.du), torch.empty_like(self.du)
            near_upsampled_slp(self.curves, self.trg, self.tc, upsample, mu, self.u_ref, self.v_ref, u1, v1)
        self._finish(labels, weight_gain)

    def correct(self, method, blob, threshold, du, dv, used_fallback=None, ws=None, curve_tol=None):
        near_correct_eval(method, self.curves, self.trg, self.tc, self.P, blob, threshold, self.mu, du, dv,
                          used_fallback, ws, curve_tol=curve_tol)


class WallNearData(_NearSet):
    """Near-wall data set: targets near periodic walls (trg_curve naming each
    one's wall), node derivatives, features, frames and (labels=True) the
    refined-wall quadrature's Delta over images img_lo..img_hi of period d,
    the refined walls' double layer u_ref (the error measure's scale) and the
    training records."""
    op = S2D_OP_DLP

    def __init__(self, walls, d, tx, ty, tc, upsample=8, img=(-1, 1), labels=True, device="cuda",
                 weight_gain=WEIGHT_GAIN):
        import torch
        from . import S2D_FP64, stokes2d_dlp_eval
        self.curves = Curves(walls, device)
        self.trg = Targets(tx, ty, device=device)
        self.tc = torch.as_tensor(np.ascontiguousarray(tc, dtype=np.int32), device=device)
        self.n = self.trg.n
        self.n_curves = self.curves.n_curves
        self.d, self.img = float(d), img
        self.mu = 1.0
        self.P = upsample
        f64 = dict(dtype=torch.float64, device=device)
        self.dtab = torch.empty((max(self.curves.n_nodes, 1), NDERIV), **f64)
        near_derivs_eval(self.curves, self.dtab)
        self.X = torch.empty((self.n, NFEAT), dtype=torch.float32, device=device)
        self.frame = torch.empty((self.n, NFRAME), **f64)
        near_wall_features_eval(self.curves, self.trg, self.tc, self.d, self.dtab, self.X, self.frame)
        self.du = self.dv = self.u_ref = self.v_ref = None
        if labels:
            self.du = torch.empty(self.n, **f64)
            self.dv = torch.empty_like(self.du)
            near_wall_correct_eval(self.curves, self.trg, self.d, img[0], img[1], upsample, self.du, self.dv)
            # u_ref = D_1 + Delta = D_P, the corrected wall field
            self.u_ref, self.v_ref = torch.empty_like(self.du), torch.empty_like(self.du)
            stokes2d_dlp_eval(S2D_FP64, self.curves, self.trg, self.d, img[0], img[1], self.u_ref, self.v_ref)
            near_wall_correct_eval(self.curves, self.trg, self.d, img[0], img[1], upsample, self.u_ref,
                                   self.v_ref, accumulate=1)
        self._finish(labels, weight_gain)

    def correct(self, method, blob, threshold, du, dv, used_fallback=None, ws=None, curve_tol=None):
        near_wall_correct_eval(self.curves, self.trg, self.d, self.img[0], self.img[1], self.P, du, dv,
                               method=method, trg_curve=self.tc, blob=blob, threshold=threshold,
                               used_fallback=used_fallback, ws=ws, curve_tol=curve_tol)


# ----------------------------------------------------------------------------
# training and calibration
# ----------------------------------------------------------------------------
def train(data: _NearSet, steps=20000, batch=1024, lr=2e-3, lr_min=2e-5, b_train=0.04, seed=0, log=None,
          log_every=5000):
    """Trains the network on data.X -> data.T with the library's kernels
    (minibatches drawn with replacement from the targets with b >= b_train
    and a positive weight, cosine learning-rate decay from lr to lr_min).
    Returns (params tensor, list of (step, minibatch loss)) with the losses
    of the first step, every log_every-th step and the last."""
    import torch
    dev = data.X.device
    params = torch.as_tensor(init_weights(seed).astype(np.float32), device=dev)
    near_feature_stats(data.X, params)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    ws = _empty(near_mlp_train_workspace_size(batch), dev)
    pool = torch.nonzero((data.b >= b_train) & (data.T[:, 12] > 0)).view(-1).to(torch.int32)
    if pool.numel() == 0:
        raise ValueError("no training samples with b >= b_train")
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    chunk = 1000
    hist = []
    for s0 in range(0, steps, chunk):
        k = min(chunk, steps - s0)
        pick = torch.randint(0, pool.numel(), (k, batch), generator=gen).to(dev)
        idx_all = pool[pick.view(-1).long()].view(k, batch)
        for j in range(k):
            step = s0 + j + 1
            cur = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * (step - 1) / max(1, steps)))
            near_mlp_train_step(batch, idx_all[j], data.X, data.T, params, m, v, step, cur, grad, loss, ws)
            if step == 1 or step % log_every == 0 or step == steps:
                hist.append((step, float(loss.item())))
                if log:
                    log(f"step {step}: loss {hist[-1][1]:.3e}")
    return params, hist


def calibrate(data: _NearSet, params, margin=1.5, count_margin=2.0, b_min=B_MIN, n_bins=N_BINS, bin_lo=BIN_LO,
              bin_w=BIN_W):
    """Per-bin bounds on held-out data by the library's calibration kernel:
    the learned route's (BF16) largest error and the largest correction, each
    over scale F, times margin (1 + count_margin / sqrt(targets in the bin)),
    per bin of (log10 b, |s|, log10 |kappa h|).
    Returns (blob, bound, bound_zero, count) as device tensors ([N_BINS *
    CELL])."""
    import torch
    dev = data.X.device
    blob = torch.zeros(near_mlp_blob_size(), dtype=torch.uint8, device=dev)
    near_mlp_pack(params, None, 0, bin_lo, bin_w, blob, b_min=b_min, upsample=data.P)
    du = torch.empty_like(data.du)
    dv = torch.empty_like(data.dv)
    data.correct(S2D_NEAR_MLP, blob, 0.0, du, dv)
    bound = torch.zeros(n_bins * CELL, dtype=torch.float32, device=dev)
    bound0 = torch.zeros_like(bound)
    count = torch.zeros(n_bins * CELL, dtype=torch.int32, device=dev)
    near_calibrate(data.op, data.frame, du, dv, data.du, data.dv, data.mu, n_bins, bin_lo, bin_w, b_min, margin,
                   bound, bound0, count, count_margin)
    near_mlp_pack(params, bound, n_bins, bin_lo, bin_w, blob, bound_zero=bound0, b_min=b_min, upsample=data.P)
    return blob, bound, bound0, count
