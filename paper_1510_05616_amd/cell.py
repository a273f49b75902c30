"""Binding of the periodization system of one channel cell (the
`stokes2d_cell_*` entry points of libstokes2d): assemble, factor and solve on
the GPU, and evaluate the represented flow with the layer-potential entry
points.  Argument marshalling only; the arithmetic runs in the library."""
from __future__ import annotations

import ctypes
import math
import types

import numpy as np

from . import (Curves, Targets, _Curves, _check, _dev_f64, _ptr, _stream, _workspace, lib,
               stokes2d_dlp_eval, stokes2d_dlp_pressure_eval, stokes2d_slp_eval, stokes2d_slp_pressure_eval)

RCOND = 1e-8


class _Cell(ctypes.Structure):
    _fields_ = [("walls", _Curves), ("n_side", ctypes.c_int32), ("side_y", ctypes.c_void_p),
                ("x_left", ctypes.c_double), ("n_proxy", ctypes.c_int32), ("proxy_cx", ctypes.c_double),
                ("proxy_cy", ctypes.c_double), ("proxy_r", ctypes.c_double), ("d", ctypes.c_double),
                ("mu", ctypes.c_double), ("lu_panel", ctypes.c_int32)]


_bound = False


def _bind():
    global _bound
    L = lib()
    if not _bound:
        P, I, SZ, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_double
        L.stokes2d_cell_workspace_size.argtypes = [P]
        L.stokes2d_cell_workspace_size.restype = SZ
        L.stokes2d_cell_assemble.argtypes = [P, P, P, P, P, P]
        L.stokes2d_cell_assemble.restype = I
        L.stokes2d_cell_factor.argtypes = [P, D, P, SZ, P]
        L.stokes2d_cell_factor.restype = I
        L.stokes2d_cell_solve.argtypes = [P, P, P, P, P, P, SZ, P]
        L.stokes2d_cell_solve.restype = I
        _bound = True
    return L


class Cell:
    """One period of a channel: wall curves (a CurveSet, or anything with x,
    y, nx, ny, w, kappa, curve_off), the K side-wall heights, period d, M
    proxy Stokeslets on the circle of radius proxy_r (default d) around the
    cell centre, viscosity mu; lu_panel: columns per LU panel (0: the widest
    the library calls allow).  Holds the factored system after factor()."""

    def __init__(self, walls, side_y, d, n_proxy, mu, x_left=0.0, proxy_r=None, device="cuda", lu_panel=0):
        self.walls = Curves(walls, device)
        self.side_y = _dev_f64(side_y, device)
        sy = np.asarray(side_y, dtype=np.float64)
        self.K = int(sy.shape[0])
        self.M = int(n_proxy)
        self.d, self.mu, self.x_left = float(d), float(mu), float(x_left)
        self.proxy_cx = self.x_left + 0.5 * self.d
        self.proxy_cy = 0.5 * (float(sy.min()) + float(sy.max()))
        self.proxy_r = self.d if proxy_r is None else float(proxy_r)
        self.device = device
        self.lu_panel = int(lu_panel)
        self.ws = None

    @property
    def n_wall(self):
        return self.walls.n_nodes

    def struct(self):
        return _Cell(self.walls.struct(), self.K, _ptr(self.side_y), self.x_left, self.M, self.proxy_cx,
                     self.proxy_cy, self.proxy_r, self.d, self.mu, self.lu_panel)

    def workspace_size(self) -> int:
        s = self.struct()
        return int(_bind().stokes2d_cell_workspace_size(ctypes.byref(s)))

    def proxy_points(self):
        th = 2 * math.pi * np.arange(self.M) / self.M
        return self.proxy_cx + self.proxy_r * np.cos(th), self.proxy_cy + self.proxy_r * np.sin(th)

    def assemble(self, stream=None):
        """The four blocks as (rows, cols) torch tensors (A, B, C, Q)."""
        import torch
        n, nc, mr = 2 * self.n_wall, 2 * self.M, 4 * self.K
        # column-major buffers = row-major (cols, rows) tensors, transposed on return
        A = torch.empty((n, n), dtype=torch.float64, device=self.device)
        B = torch.empty((nc, n), dtype=torch.float64, device=self.device)
        C = torch.empty((n, mr), dtype=torch.float64, device=self.device)
        Q = torch.empty((nc, mr), dtype=torch.float64, device=self.device)
        s = self.struct()
        _check(_bind().stokes2d_cell_assemble(ctypes.byref(s), _ptr(A), _ptr(B), _ptr(C), _ptr(Q),
                                              _stream(stream)))
        return A.t(), B.t(), C.t(), Q.t()

    def factor(self, rcond=RCOND, ws=None, stream=None):
        self.ws = _workspace(self.workspace_size(), self.device, ws)
        s = self.struct()
        _check(_bind().stokes2d_cell_factor(ctypes.byref(s), float(rcond), _ptr(self.ws), self.ws.numel(),
                                            _stream(stream)))

    def solve(self, v, g, tau=None, c=None, stream=None):
        """v [2N], g [4K] (device float64, interleaved); returns (tau [2N], c [2M])."""
        import torch
        if self.ws is None:
            raise RuntimeError("factor() the cell first")
        f64 = dict(dtype=torch.float64, device=self.device)
        tau = torch.empty(2 * self.n_wall, **f64) if tau is None else tau
        c = torch.empty(2 * self.M, **f64) if c is None else c
        s = self.struct()
        _check(_bind().stokes2d_cell_solve(ctypes.byref(s), _ptr(v), _ptr(g), _ptr(tau), _ptr(c), _ptr(self.ws),
                                           self.ws.numel(), _stream(stream)))
        return tau, c

    def flow(self, tau, c, X, Y, mode=0, stream=None):
        """Velocity (u, v) and pressure p of the representation at free
        points (X, Y): the wall double layer of tau over the images |n| <= 1
        plus the proxy Stokeslets of strength c."""
        import torch
        w = self.walls
        dens = types.SimpleNamespace(x=w.x, y=w.y, nx=w.nx, ny=w.ny, w=w.w, kappa=w.kappa,
                                     fx=tau[0::2].contiguous(), fy=tau[1::2].contiguous(), curve_off=w.curve_off)
        px, py = self.proxy_points()
        M = self.M
        prox = types.SimpleNamespace(x=px, y=py, nx=np.zeros(M), ny=np.zeros(M), w=np.ones(M), kappa=np.zeros(M),
                                     fx=c[0::2].contiguous(), fy=c[1::2].contiguous(),
                                     curve_off=np.array([0, M], np.int32))
        wc, pc = Curves(dens, self.device), Curves(prox, self.device)
        tg = Targets(X, Y, device=self.device)
        f64 = dict(dtype=torch.float64, device=self.device)
        n = tg.n
        u, v, p = torch.zeros(n, **f64), torch.zeros(n, **f64), torch.zeros(n, **f64)
        stokes2d_dlp_eval(mode, wc, tg, self.d, -1, 1, u, v, stream=stream)
        stokes2d_slp_eval(mode, pc, tg, self.d, 0, 0, self.mu, u, v, accumulate=1, stream=stream)
        stokes2d_dlp_pressure_eval(mode, wc, tg, self.d, -1, 1, self.mu, p, stream=stream)
        stokes2d_slp_pressure_eval(mode, pc, tg, self.d, 0, 0, p, accumulate=1, stream=stream)
        return u, v, p
