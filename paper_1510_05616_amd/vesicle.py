"""Binding of the vesicle time-step entry points of libstokes2d
(include/stokes2d_vesicle.h): argument marshalling only, every step runs in
the library."""
from __future__ import annotations

import ctypes

from . import _check, _ptr, _stream, lib

_bound = False


class StepParams(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("dt", ctypes.c_double), ("kappa_b", ctypes.c_double),
                ("mu", ctypes.c_double), ("d", ctypes.c_double), ("img_lo", ctypes.c_int32),
                ("img_hi", ctypes.c_int32), ("L0", ctypes.c_void_p), ("u_resp_x", ctypes.c_void_p),
                ("u_resp_y", ctypes.c_void_p), ("tol", ctypes.c_double), ("restart", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("precond", ctypes.c_int32), ("nmax", ctypes.c_int32),
                ("near", ctypes.c_int32), ("near_P", ctypes.c_int32), ("near_band", ctypes.c_double),
                ("near_max", ctypes.c_int32), ("warm", ctypes.c_int32)]


def _bind():
    global _bound
    L = lib()
    if _bound:
        return L
    P, I, I32, I64, D, SZ = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                             ctypes.c_size_t)
    L.ves_geometry.argtypes = [I64, I32, P, P, P, P, P, P, P, P, P, P]
    L.ves_geometry.restype = I
    L.ves_forces.argtypes = [I64, I32, P, P, P, P, D, P, P, P, P, P]
    L.ves_forces.restype = I
    L.ves_measure.argtypes = [I64, I32, P, P, P, P, P, P]
    L.ves_measure.restype = I
    L.ves_step_workspace_size.argtypes = [I64, I32, P]
    L.ves_step_workspace_size.restype = SZ
    L.ves_step_apply.argtypes = [I64, I32, P, P, P, P, P, P, P, P, SZ, P]
    L.ves_step_apply.restype = I
    L.ves_step_solve.argtypes = [I64, I32, P, P, P, P, P, P, P, P, SZ, P]
    L.ves_step_solve.restype = I
    L.ves_area_correct.argtypes = [I64, I32, P, P, P, P, P]
    L.ves_area_correct.restype = I
    L.ves_reparameterize.argtypes = [I64, I32, P, P, P, P, P]
    L.ves_reparameterize.restype = I
    L.ves_time_step.argtypes = [I64, I32, P, P, P, P, P, P, I, P, P, P, P, P, SZ, P]
    L.ves_time_step.restype = I
    L.ves_total_force.argtypes = [I64, I32, P, P, P, P, D, P, P, P]
    L.ves_total_force.restype = I
    L.ves_response_workspace_size.argtypes = [P, I64, I32, I]
    L.ves_response_workspace_size.restype = SZ
    L.ves_channel_response.argtypes = [P, P, SZ, I64, I32, P, P, P, P, P, D, I, P, P, P, SZ, P]
    L.ves_channel_response.restype = I
    _bound = True
    return L


def params(mode=0, dt=1e-3, kappa_b=1.0, mu=1.0, d=0.0, img_lo=0, img_hi=0, L0=None, u_resp=None, tol=1e-12,
           restart=64, max_iter=2000, precond=None, nmax=0, near=0, near_P=8, near_band=5.0,
           near_max=1 << 20, warm=0) -> StepParams:
    """L0: device float64 [n_curves] or None; u_resp: (ux, uy) device tensors
    or None; nmax: largest curve size; precond (default: when nmax is given)
    selects the block-diagonal preconditioner; near = 1 turns on the close
    evaluation between vesicles (near_P-times upsampled quadrature for the
    nodes within near_band spacings of another vesicle, at most near_max
    such pairs); warm = 1 starts GMRES from the given solution (the z of
    step_solve, or the velocity uv and sigma of time_step).  The returned
    structure keeps the tensors it points to alive."""
    ux, uy = (None, None) if u_resp is None else u_resp
    precond = nmax > 0 if precond is None else precond
    p = StepParams(int(mode), float(dt), float(kappa_b), float(mu), float(d), int(img_lo), int(img_hi),
                   _ptr(L0), _ptr(ux), _ptr(uy), float(tol), int(restart), int(max_iter), int(bool(precond)),
                   int(nmax), int(near), int(near_P), float(near_band), int(near_max), int(bool(warm)))
    p._keep = (L0, ux, uy)
    return p


class Vesicles:
    """Device vesicle set: x, y, sigma ([n] float64 tensors, updated in place
    by a time step) and curve_off ([n_curves + 1] int32)."""

    def __init__(self, x, y, curve_off, sigma=None, device="cuda"):
        import torch
        f64 = dict(dtype=torch.float64, device=device)
        self.x = torch.as_tensor(x, **f64).clone().contiguous()
        self.y = torch.as_tensor(y, **f64).clone().contiguous()
        self.off = torch.as_tensor(curve_off, dtype=torch.int32, device=device).contiguous()
        self.n = int(self.x.shape[0])
        self.nc = int(self.off.shape[0]) - 1
        self.sigma = (torch.zeros(self.n, **f64) if sigma is None else
                      torch.as_tensor(sigma, **f64).clone().contiguous())
        self.device = device

    def _a(self):
        return (ctypes.c_int64(self.n), ctypes.c_int32(self.nc), _ptr(self.off), _ptr(self.x), _ptr(self.y))

    def geometry(self, stream=None):
        import torch
        out = [torch.empty(self.n, dtype=torch.float64, device=self.device) for _ in range(6)]
        _check(_bind().ves_geometry(*self._a(), *(_ptr(o) for o in out), _stream(stream)))
        return dict(zip(("speed", "w", "nx", "ny", "tx", "ty"), out))

    def forces(self, kappa_b, sigma=None, stream=None):
        import torch
        out = [torch.empty(self.n, dtype=torch.float64, device=self.device) for _ in range(4)]
        _check(_bind().ves_forces(*self._a(), _ptr(sigma), float(kappa_b), *(_ptr(o) for o in out),
                                  _stream(stream)))
        return out

    def total_force(self, kappa_b, stream=None):
        """f = f_b + f_sigma with the current tension."""
        import torch
        fx = torch.empty(self.n, dtype=torch.float64, device=self.device)
        fy = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(_bind().ves_total_force(*self._a(), _ptr(self.sigma), float(kappa_b), _ptr(fx), _ptr(fy),
                                       _stream(stream)))
        return fx, fy

    def channel_response(self, cell, fx, fy, p_drive, mode=0, ws=None, stream=None):
        """u_resp at the nodes for the force density (fx, fy), from a
        factored cell (paper_1510_05616_amd.cell.Cell)."""
        import torch
        if cell.ws is None:
            raise RuntimeError("factor() the cell first")
        L = _bind()
        cs = cell.struct()
        if ws is None:
            nb = int(L.ves_response_workspace_size(ctypes.byref(cs), self.n, self.nc, int(mode)))
            ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)
        ux = torch.empty(self.n, dtype=torch.float64, device=self.device)
        uy = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(L.ves_channel_response(ctypes.byref(cs), _ptr(cell.ws), cell.ws.numel(), self.n, self.nc,
                                      _ptr(self.off), _ptr(self.x), _ptr(self.y), _ptr(fx), _ptr(fy),
                                      float(p_drive), int(mode), _ptr(ux), _ptr(uy), _ptr(ws), ws.numel(),
                                      _stream(stream)))
        return ux, uy

    def measure(self, stream=None):
        import torch
        L = torch.empty(self.nc, dtype=torch.float64, device=self.device)
        A = torch.empty(self.nc, dtype=torch.float64, device=self.device)
        _check(_bind().ves_measure(*self._a(), _ptr(L), _ptr(A), _stream(stream)))
        return L, A

    def workspace(self, p: StepParams):
        import torch
        nb = int(_bind().ves_step_workspace_size(self.n, self.nc, ctypes.byref(p)))
        return torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)

    def step_apply(self, p: StepParams, z, with_rhs=True, ws=None, stream=None):
        import torch
        ws = self.workspace(p) if ws is None else ws
        out = torch.empty(3 * self.n, dtype=torch.float64, device=self.device)
        b = torch.empty(3 * self.n, dtype=torch.float64, device=self.device) if with_rhs else None
        _check(_bind().ves_step_apply(*self._a(), ctypes.byref(p), _ptr(z), _ptr(out), _ptr(b), _ptr(ws),
                                      ws.numel(), _stream(stream)))
        return out, b

    def step_solve(self, p: StepParams, ws=None, stream=None):
        import torch
        ws = self.workspace(p) if ws is None else ws
        z = torch.empty(3 * self.n, dtype=torch.float64, device=self.device)
        it, res = ctypes.c_int32(0), ctypes.c_double(0.0)
        _check(_bind().ves_step_solve(*self._a(), ctypes.byref(p), _ptr(z), ctypes.byref(it), ctypes.byref(res),
                                      _ptr(ws), ws.numel(), _stream(stream)))
        return z, int(it.value), float(res.value)

    def area_correct(self, A0, stream=None):
        _check(_bind().ves_area_correct(*self._a(), _ptr(A0), _stream(stream)))

    def reparameterize(self, with_sigma=True, stream=None):
        _check(_bind().ves_reparameterize(*self._a(), _ptr(self.sigma) if with_sigma else None,
                                          _stream(stream)))

    def time_step(self, p: StepParams, A0=None, reparam=True, ws=None, uv=None, stream=None):
        """One step in place; returns (iterations, relative residual)."""
        ws = self.workspace(p) if ws is None else ws
        u, v = (None, None) if uv is None else uv
        it, res = ctypes.c_int32(0), ctypes.c_double(0.0)
        _check(_bind().ves_time_step(*self._a(), _ptr(self.sigma), ctypes.byref(p), _ptr(A0), int(bool(reparam)),
                                     _ptr(u), _ptr(v), ctypes.byref(it), ctypes.byref(res), _ptr(ws), ws.numel(),
                                     _stream(stream)))
        return int(it.value), float(res.value)
