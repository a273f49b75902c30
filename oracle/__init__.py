"""FP64 CPU oracle for the periodic-channel Stokes layer potentials.

TEST INFRASTRUCTURE ONLY: imported by `tests/`, by `__graft_entry__.smoke()`
and by the CPU-baseline leg of `bench.py`, never by the library.  It shares no
code with the GPU path (`paper_1510_05616_amd`), and the GPU path never calls
it.

The pair sums and Kress's self quadrature are plain C (`stokes_oracle.c`,
OpenMP over targets, IEEE double, Neumaier summation); this module compiles
that file with gcc and marshals numpy arrays into it.  `near.py` holds the
numpy FP64 references for the near-field extension (FFT-upsampled trapezoid
quadrature, target features, and the MLP forward/backward pass); `els.py`
the dense assembly and Schur-complement solve of the periodization system of
an empty channel cell.

Pins (tests/test_oracle_*.py): Kress weights exact on cos(m t) and summing to
zero; the circle of constant density; the double-layer translation identity
(-c inside, 0 outside, -c/2 on the curve); reproduction of an exterior point
Stokeslet by Green's identity with spectral convergence; Stokeslet symmetry;
50-digit brute force on tiny curves; explicit image replication.  Pressures
and traction: the single-layer pressure of a circle of constant density in
closed form; the pressure form of Green's identity, with the traction data
taken from the oracle's own traction kernel; the traction equals the stress
of the single-layer velocity and pressure fields (finite differences).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stokes_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_lib = None

__all__ = ["build", "slp", "dlp", "slp_pressure", "dlp_pressure", "slp_traction", "kress_weights", "num_threads"]


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_slp.restype = ctypes.c_int
        lib.oracle_slp.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, P, P, P, P, P, P,
                                   ctypes.c_int64, P, P, P, P, ctypes.c_double,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_double, P, P]
        lib.oracle_dlp.restype = ctypes.c_int
        lib.oracle_dlp.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, P, P, P, P, P, P, P,
                                   ctypes.c_int64, P, P, P, P, ctypes.c_double,
                                   ctypes.c_int32, ctypes.c_int32, P, P]
        I64, I32, D = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.oracle_slp_pressure.restype = ctypes.c_int
        lib.oracle_slp_pressure.argtypes = [I64, P, P, P, P, P, I64, P, P, D, I32, I32, P]
        lib.oracle_dlp_pressure.restype = ctypes.c_int
        lib.oracle_dlp_pressure.argtypes = [I64, P, P, P, P, P, P, P, I64, P, P, D, I32, I32, D, P]
        lib.oracle_slp_traction.restype = ctypes.c_int
        lib.oracle_slp_traction.argtypes = [I64, P, P, P, P, P, I64, P, P, P, P, D, I32, I32, P, P]
        lib.oracle_kress_weights.argtypes = [ctypes.c_int, P]
        lib.oracle_kress_weights.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def slp(src, tx, ty, on_curve=None, on_node=None, d=0.0, img_lo=0, img_hi=0, mu=1.0):
    """Stokes single-layer potential of density src.fx, src.fy (weights src.w)
    at targets (tx, ty), summed over images img_lo..img_hi of period d.
    Targets with on_curve >= 0 are node on_node of that source curve and get
    Kress's product quadrature for their own curve (n = 0)."""
    lib = _load()
    arrs = [_f64(getattr(src, k)) for k in ("x", "y", "nx", "ny", "w", "fx", "fy")]
    off = _i32(src.curve_off)
    tx, ty = _f64(tx), _f64(ty)
    oc, on = _i32(on_curve), _i32(on_node)
    u = np.zeros(tx.shape[0])
    v = np.zeros(tx.shape[0])
    rc = lib.oracle_slp(arrs[0].shape[0], off.shape[0] - 1, _p(off), *[_p(a) for a in arrs],
                        tx.shape[0], _p(tx), _p(ty), _p(oc), _p(on), float(d),
                        int(img_lo), int(img_hi), float(mu), _p(u), _p(v))
    if rc != 0:
        raise ValueError("oracle_slp: invalid arguments")
    return u, v


def dlp(src, tx, ty, on_curve=None, on_node=None, d=0.0, img_lo=0, img_hi=0):
    """Stokes double-layer potential (principal value) of density src.fx,
    src.fy; targets with on_curve >= 0 use the Nystrom diagonal limit."""
    lib = _load()
    arrs = [_f64(getattr(src, k)) for k in ("x", "y", "nx", "ny", "w", "kappa", "fx", "fy")]
    off = _i32(src.curve_off)
    tx, ty = _f64(tx), _f64(ty)
    oc, on = _i32(on_curve), _i32(on_node)
    u = np.zeros(tx.shape[0])
    v = np.zeros(tx.shape[0])
    rc = lib.oracle_dlp(arrs[0].shape[0], off.shape[0] - 1, _p(off), *[_p(a) for a in arrs],
                        tx.shape[0], _p(tx), _p(ty), _p(oc), _p(on), float(d),
                        int(img_lo), int(img_hi), _p(u), _p(v))
    if rc != 0:
        raise ValueError("oracle_dlp: invalid arguments")
    return u, v


def slp_pressure(src, tx, ty, d=0.0, img_lo=0, img_hi=0):
    """Pressure of the single layer (density src.fx, src.fy, weights src.w) at
    free targets, summed over images img_lo..img_hi of period d."""
    lib = _load()
    x, y, w, fx, fy = (_f64(getattr(src, k)) for k in ("x", "y", "w", "fx", "fy"))
    tx, ty = _f64(tx), _f64(ty)
    p = np.zeros(tx.shape[0])
    if lib.oracle_slp_pressure(x.shape[0], _p(x), _p(y), _p(w), _p(fx), _p(fy), tx.shape[0], _p(tx), _p(ty),
                               float(d), int(img_lo), int(img_hi), _p(p)) != 0:
        raise ValueError("oracle_slp_pressure: invalid arguments")
    return p


def dlp_pressure(src, tx, ty, d=0.0, img_lo=0, img_hi=0, mu=1.0):
    """Pressure of the double layer (density src.fx, src.fy, source normals
    src.nx, src.ny, weights src.w) at free targets."""
    lib = _load()
    x, y, nx, ny, w, fx, fy = (_f64(getattr(src, k)) for k in ("x", "y", "nx", "ny", "w", "fx", "fy"))
    tx, ty = _f64(tx), _f64(ty)
    p = np.zeros(tx.shape[0])
    if lib.oracle_dlp_pressure(x.shape[0], _p(x), _p(y), _p(nx), _p(ny), _p(w), _p(fx), _p(fy), tx.shape[0],
                               _p(tx), _p(ty), float(d), int(img_lo), int(img_hi), float(mu), _p(p)) != 0:
        raise ValueError("oracle_dlp_pressure: invalid arguments")
    return p


def slp_traction(src, tx, ty, mx, my, d=0.0, img_lo=0, img_hi=0):
    """Traction of the single layer at free targets with unit normals (mx, my)."""
    lib = _load()
    x, y, w, fx, fy = (_f64(getattr(src, k)) for k in ("x", "y", "w", "fx", "fy"))
    tx, ty, mx, my = _f64(tx), _f64(ty), _f64(mx), _f64(my)
    ox, oy = np.zeros(tx.shape[0]), np.zeros(tx.shape[0])
    if lib.oracle_slp_traction(x.shape[0], _p(x), _p(y), _p(w), _p(fx), _p(fy), tx.shape[0], _p(tx), _p(ty),
                               _p(mx), _p(my), float(d), int(img_lo), int(img_hi), _p(ox), _p(oy)) != 0:
        raise ValueError("oracle_slp_traction: invalid arguments")
    return ox, oy


def kress_weights(N: int) -> np.ndarray:
    lib = _load()
    R = np.zeros(N)
    if lib.oracle_kress_weights(int(N), _p(R)) != 0:
        raise ValueError("N must be even and >= 2")
    return R


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def full_eval(prob, img_lo=-1, img_hi=1):
    """SLP(vesicles) + DLP(walls) at every target of a synthetic problem;
    returns (u_slp, v_slp, u_dlp, v_dlp)."""
    t = prob.trg
    us, vs = slp(prob.ves, t.x, t.y, t.ves_curve, t.ves_node, prob.d, img_lo, img_hi, prob.mu)
    ud, vd = dlp(prob.wall, t.x, t.y, t.wall_curve, t.wall_node, prob.d, img_lo, img_hi)
    return us, vs, ud, vd
