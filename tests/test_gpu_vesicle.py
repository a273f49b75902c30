"""GPU parity of the vesicle time step (include/stokes2d_vesicle.h) with the
FP64 oracle (oracle/vesicle.py): geometry, membrane forces, the step
operator and its right-hand side, the GMRES solve against the oracle's
dense solve, the area correction, the reparameterization and whole time
steps; at the 128k channel's vesicle set (1,000 x 96 nodes, images -1..1),
properties that hold at any size.

Tolerances (FP64).  Geometry, area correction: 1e-12 of the largest
magnitude.  The bending force applies D_s four times: rounding in mode k
grows like k^4 there, (N/2)^4 ~ 1e7 at N = 128, and the GPU's direct sums
and the oracle's FFTs round differently, so it is held to 1e-9 (measured
2e-10 to 3e-10); the operator with a smooth argument to 1e-10.  The
reparameterization evaluates interpolants at new parameters that depend on
the arc-length table; a tension with all modes present carries that
sensitivity: 1e-11 (measured 3e-12).  GMRES stops at a relative residual
of 1e-12; its solution is held to the oracle's dense solve through the
residual under the oracle's matrix (1e-10) and element-wise to 1e-7 of the
largest entry (the step matrix has condition numbers of 1e3-1e5 here)."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1510_05616_amd as s2d
    s2d.stokes2d_init(0)
    yield


def _set(sizes=(32, 64, 96, 128, 48), seed=0):
    """Ellipses of mixed node counts, random axes, angles and centres,
    spaced apart along x."""
    rng = np.random.default_rng(seed)
    xs, ys, off = [], [], [0]
    for i, N in enumerate(sizes):
        a = rng.uniform(0.3, 0.5)
        b = a * rng.uniform(0.4, 0.9)
        x, y = synth._ellipse(1.2 * i, rng.uniform(-0.2, 0.2), a, b, rng.uniform(0, math.pi), N)[:2]
        xs.append(x)
        ys.append(y)
        off.append(off[-1] + N)
    return np.concatenate(xs), np.concatenate(ys), np.array(off, np.int32)


def _rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def _np(t):
    return t.detach().cpu().numpy()


def test_geometry_and_forces():
    from oracle import vesicle as ov
    from paper_1510_05616_amd.vesicle import Vesicles
    import torch
    x, y, off = _set()
    n = x.shape[0]
    sig = np.cos(np.arange(n) * 0.37) + 0.2
    V = Vesicles(x, y, off)
    geo = V.geometry()
    g = ov.geometry(x, y, off)
    assert _rel(_np(geo["speed"]), g.sp) < 1e-12
    assert _rel(_np(geo["w"]), g.w) < 1e-12
    assert _rel(_np(geo["nx"]), g.nx) < 1e-12 and _rel(_np(geo["ny"]), g.ny) < 1e-12
    fb = V.forces(2.0, torch.as_tensor(sig, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    o = ov.forces(g, sig, 2.0)
    errs = [_rel(_np(a), b) for a, b in zip(fb, o)]
    print(f"forces rel errors {errs}", flush=True)
    assert max(errs[:2]) < 1e-9 and max(errs[2:]) < 1e-12
    L, A = V.measure()
    assert _rel(_np(L), ov.arc_lengths(g)) < 1e-12 and _rel(_np(A), ov.areas(x, y, off)) < 1e-12


@pytest.mark.parametrize("img", [(0, 0), (-1, 1)])
def test_step_operator_and_rhs(img):
    from oracle import vesicle as ov
    from paper_1510_05616_amd import vesicle as pv
    import torch
    x, y, off = _set(sizes=(32, 48, 64), seed=1)
    n = x.shape[0]
    d = 4.0
    g = ov.geometry(x, y, off)
    L0 = ov.arc_lengths(g) * np.array([1.002, 0.999, 1.0])
    rng = np.random.default_rng(2)
    urx, ury = rng.standard_normal(n), rng.standard_normal(n)
    f64 = dict(dtype=torch.float64, device="cuda")
    L0d = torch.as_tensor(L0, **f64)
    ur = (torch.as_tensor(urx, **f64), torch.as_tensor(ury, **f64))
    p = pv.params(dt=0.003, kappa_b=0.8, mu=0.7, d=d, img_lo=img[0], img_hi=img[1], L0=L0d, u_resp=ur)
    V = pv.Vesicles(x, y, off)
    # a smooth z (the operator's high modes are rounding-amplified k^4 times)
    al = np.concatenate([2 * math.pi * np.arange(off[c + 1] - off[c]) / (off[c + 1] - off[c]) for c in range(3)])
    z = np.concatenate([np.cos(al) + 0.3 * np.sin(3 * al), np.sin(2 * al) - 0.1, 0.5 * np.cos(al) + 1.0])
    out, b = V.step_apply(p, torch.as_tensor(z, **f64))
    torch.cuda.synchronize()
    S = ov.slp_matrix(g, d, img[0], img[1], 0.7)
    A = ov.step_system(g, S, 0.003, 0.8)
    bo = ov.step_rhs(g, S, 0.003, 0.8, L0, (urx, ury))
    e_op, e_b = _rel(_np(out), A @ z), _rel(_np(b), bo)
    print(f"img={img} operator {e_op:.2e} rhs {e_b:.2e}", flush=True)
    assert e_op < 1e-10 and e_b < 1e-10


def _close_set():
    """Three ellipses 0.05 apart along x (0.7 node spacings), the third's
    image at -d as close to the first: nodes near other vesicles and near
    images of them."""
    xs, ys, off = [], [], [0]
    for cx, cy, N in ((0.0, 0.0, 32), (0.95, 0.04, 48), (1.9, -0.03, 32)):
        x, y = synth._ellipse(cx, cy, 0.45, 0.3, 0.0, N)[:2]
        xs.append(x)
        ys.append(y)
        off.append(off[-1] + N)
    return np.concatenate(xs), np.concatenate(ys), np.array(off, np.int32), 2.85


def _near_oracle(g, d, img, band=5.0, P=8, mu=0.7):
    """The oracle's close-evaluation correction of S, and the pairs, checked
    to lie clear of the band's edge (decisions both sides must share)."""
    from oracle import vesicle as ov
    pairs = ov.near_pairs(g, d, img[0], img[1], band)
    for b2 in (band * (1 - 1e-9), band * (1 + 1e-9)):
        assert ov.near_pairs(g, d, img[0], img[1], b2) == pairs, "a node sits on the band's edge"
    return pairs, ov.near_slp_matrix(g, pairs, d, P, mu)


@pytest.mark.parametrize("img", [(0, 0), (-1, 1)])
def test_step_operator_with_close_evaluation(img):
    """The step operator and right-hand side with close evaluation between
    vesicles (8x upsampled, band 5 spacings) against the oracle's matrix
    with the same correction; the correction itself is far above the
    tolerance."""
    from oracle import vesicle as ov
    from paper_1510_05616_amd import vesicle as pv
    import torch
    x, y, off, d = _close_set()
    n = x.shape[0]
    g = ov.geometry(x, y, off)
    pairs, dS = _near_oracle(g, d, img)
    assert len(pairs) > 20 and (img == (0, 0) or any(k != 0 for _, _, k in pairs))
    L0 = ov.arc_lengths(g)
    f64 = dict(dtype=torch.float64, device="cuda")
    V = pv.Vesicles(x, y, off)
    al = np.concatenate([2 * math.pi * np.arange(off[c + 1] - off[c]) / (off[c + 1] - off[c]) for c in range(3)])
    z = np.concatenate([np.cos(al) + 0.3 * np.sin(3 * al), np.sin(2 * al) - 0.1, 0.5 * np.cos(al) + 1.0])
    kw = dict(dt=0.002, kappa_b=0.8, mu=0.7, d=d, img_lo=img[0], img_hi=img[1], L0=torch.as_tensor(L0, **f64),
              nmax=48, precond=False)
    out, b = V.step_apply(pv.params(near=1, near_P=8, near_band=5.0, near_max=4096, **kw), torch.as_tensor(z, **f64))
    out0, b0 = V.step_apply(pv.params(**kw), torch.as_tensor(z, **f64))
    torch.cuda.synchronize()
    S = ov.slp_matrix(g, d, img[0], img[1], 0.7) + dS
    A = ov.step_system(g, S, 0.002, 0.8)
    bo = ov.step_rhs(g, S, 0.002, 0.8, L0)
    e_op, e_b = _rel(_np(out), A @ z), _rel(_np(b), bo)
    c_op, c_b = _rel(_np(out0), A @ z), _rel(_np(b0), bo)
    print(f"img={img} pairs {len(pairs)}: operator {e_op:.2e} rhs {e_b:.2e} (without the correction "
          f"{c_op:.2e}, {c_b:.2e})", flush=True)
    assert e_op < 1e-10 and e_b < 1e-10
    assert c_op > 1e-6 and c_b > 1e-6
    # a capacity below the pair count is an error, not a silent truncation
    import paper_1510_05616_amd as s2d
    with pytest.raises(s2d.S2DError):
        V.step_apply(pv.params(near=1, near_P=8, near_band=5.0, near_max=len(pairs) - 1, **kw),
                     torch.as_tensor(z, **f64))


def test_time_steps_with_close_evaluation_match_the_oracle():
    """Three time steps of the close set with close evaluation (images
    -1..1; the pairs are found anew at every step) against the oracle's
    steps with the same correction."""
    from oracle import vesicle as ov
    from paper_1510_05616_amd import vesicle as pv
    import torch
    x, y, off, d = _close_set()
    g = ov.geometry(x, y, off)
    L0, A0 = ov.arc_lengths(g), ov.areas(x, y, off)
    f64 = dict(dtype=torch.float64, device="cuda")
    p = pv.params(mode=0, dt=0.002, kappa_b=1.0, mu=0.7, d=d, img_lo=-1, img_hi=1, L0=torch.as_tensor(L0, **f64),
                  tol=1e-13, restart=64, max_iter=4000, nmax=48, near=1, near_P=8, near_band=5.0, near_max=4096)
    V = pv.Vesicles(x, y, off)
    A0d = torch.as_tensor(A0, **f64)
    xo, yo, so = x.copy(), y.copy(), np.zeros_like(x)
    for k in range(3):
        _near_oracle(ov.geometry(xo, yo, off), d, (-1, 1))
        it, res = V.time_step(p, A0=A0d, reparam=True)
        xo, yo, so, _, _ = ov.time_step(xo, yo, so, off, 0.002, 1.0, 0.7, L0=L0, A0=A0, d=d, img_lo=-1, img_hi=1,
                                        near=(8, 5.0))
        torch.cuda.synchronize()
        ex = max(_rel(_np(V.x), xo), _rel(_np(V.y), yo))
        es = _rel(_np(V.sigma), so)
        print(f"close set step {k}: {it} iterations, residual {res:.1e}, x {ex:.2e}, sigma {es:.2e}", flush=True)
        assert res <= 1e-13 and ex < 1e-11 and es < 1e-7


def test_refined_fp32c_solve_matches_dense_solve():
    # FP32C corrections with FP64 residuals reach the FP64 tolerance
    from oracle import vesicle as ov
    from paper_1510_05616_amd import vesicle as pv
    import torch
    x, y, off = _set(sizes=(32, 48, 64), seed=3)
    g = ov.geometry(x, y, off)
    L0 = ov.arc_lengths(g) * np.array([1.001, 1.0, 0.998])
    f64 = dict(dtype=torch.float64, device="cuda")
    p = pv.params(mode=1, dt=0.002, kappa_b=1.0, mu=1.0, L0=torch.as_tensor(L0, **f64), tol=1e-12, nmax=64)
    V = pv.Vesicles(x, y, off)
    z, it, res = V.step_solve(p)
    torch.cuda.synchronize()
    S = ov.slp_matrix(g, 0.0, 0, 0, 1.0)
    A = ov.step_system(g, S, 0.002, 1.0)
    b = ov.step_rhs(g, S, 0.002, 1.0, L0)
    zo = np.linalg.solve(A, b)
    zg = _np(z)
    r_or = np.linalg.norm(A @ zg - b) / np.linalg.norm(b)
    print(f"refined FP32C: {it} GMRES iterations, residual {res:.2e}, under the oracle's matrix {r_or:.2e}, "
          f"vs dense {_rel(zg, zo):.2e}", flush=True)
    assert res <= 1e-12 and r_or < 1e-10 and _rel(zg, zo) < 1e-7


@pytest.mark.parametrize("precond", [True, False])
def test_gmres_solve_matches_dense_solve(precond):
    from oracle import vesicle as ov
    from paper_1510_05616_amd import vesicle as pv
    import torch
    x, y, off = _set(sizes=(32, 48, 64), seed=3)
    g = ov.geometry(x, y, off)
    L0 = ov.arc_lengths(g) * np.array([1.001, 1.0, 0.998])
    f64 = dict(dtype=torch.float64, device="cuda")
    # without the preconditioner GMRES needs thousands of iterations
    # (condition number 1e5): it is run to 1e-8 only
    tol = 1e-12 if precond else 1e-8
    p = pv.params(dt=0.002, kappa_b=1.0, mu=1.0, L0=torch.as_tensor(L0, **f64), tol=tol, restart=64,
                  max_iter=8000, precond=precond, nmax=64)
    V = pv.Vesicles(x, y, off)
    z, it, res = V.step_solve(p)
    torch.cuda.synchronize()
    S = ov.slp_matrix(g, 0.0, 0, 0, 1.0)
    A = ov.step_system(g, S, 0.002, 1.0)
    b = ov.step_rhs(g, S, 0.002, 1.0, L0)
    zo = np.linalg.solve(A, b)
    zg = _np(z)
    r_or = np.linalg.norm(A @ zg - b) / np.linalg.norm(b)
    print(f"precond={precond}: GMRES {it} iterations, residual {res:.2e}, under the oracle's matrix {r_or:.2e}, "
          f"vs dense {_rel(zg, zo):.2e}, cond {np.linalg.cond(A):.2e}", flush=True)
    assert res <= tol and r_or < 100 * tol and _rel(zg, zo) < 1e5 * tol


def test_area_correction_and_reparameterization():
    from oracle import vesicle as ov
    from paper_1510_05616_amd.vesicle import Vesicles
    import torch
    # curves in a stretched parameter (non-uniform nodes), then scaled
    sizes = (32, 64, 96)
    xs, ys, off = [], [], [0]
    for i, N in enumerate(sizes):
        al = 2 * math.pi * np.arange(N) / N
        t = al + 0.2 * np.sin(al + i)
        xs.append(1.5 * i + 0.5 * np.cos(t) + 0.05 * np.cos(3 * t))
        ys.append(0.3 * np.sin(t))
        off.append(off[-1] + N)
    x, y, off = np.concatenate(xs), np.concatenate(ys), np.array(off, np.int32)
    sig = np.sin(np.arange(x.shape[0]) * 0.2)
    A0 = ov.areas(x, y, off) * np.array([1.01, 0.99, 1.005])
    V = Vesicles(x, y, off, sigma=sig)
    V.area_correct(torch.as_tensor(A0, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    xo, yo, _ = ov.area_correct(x, y, off, A0)
    assert _rel(_np(V.x), xo) < 1e-13 and _rel(_np(V.y), yo) < 1e-12
    V.reparameterize()
    torch.cuda.synchronize()
    xr, yr, sr = ov.reparameterize(xo, yo, sig, off)
    errs = (_rel(_np(V.x), xr), _rel(_np(V.y), yr), _rel(_np(V.sigma), sr))
    print(f"reparameterization rel errors {errs}", flush=True)
    assert max(errs) < 1e-11


@pytest.mark.parametrize("img,mode", [((0, 0), 0), ((-1, 1), 0), ((-1, 1), 1)])
def test_time_steps_match_the_oracle(img, mode):
    from oracle import vesicle as ov
    from paper_1510_05616_amd import vesicle as pv
    import torch
    x, y, off = _set(sizes=(32, 32, 48), seed=4)
    d = 4.0
    g = ov.geometry(x, y, off)
    L0, A0 = ov.arc_lengths(g), ov.areas(x, y, off)
    f64 = dict(dtype=torch.float64, device="cuda")
    # FP32C (mode 1): refined to 1e-12 (FP64 residuals)
    tol = 1e-13 if mode == 0 else 1e-12
    p = pv.params(mode=mode, dt=0.005, kappa_b=1.0, mu=1.0, d=d, img_lo=img[0], img_hi=img[1],
                  L0=torch.as_tensor(L0, **f64), tol=tol, restart=64, max_iter=4000, nmax=48)
    V = pv.Vesicles(x, y, off)
    A0d = torch.as_tensor(A0, **f64)
    xo, yo, so = x.copy(), y.copy(), np.zeros_like(x)
    for k in range(3):
        it, res = V.time_step(p, A0=A0d, reparam=True)
        xo, yo, so, _, _ = ov.time_step(xo, yo, so, off, 0.005, 1.0, 1.0, L0=L0, A0=A0, d=d, img_lo=img[0],
                                        img_hi=img[1])
        torch.cuda.synchronize()
        ex = max(_rel(_np(V.x), xo), _rel(_np(V.y), yo))
        es = _rel(_np(V.sigma), so)
        print(f"img={img} mode={mode} step {k}: {it} iterations, residual {res:.1e}, x {ex:.2e}, sigma {es:.2e}",
              flush=True)
        assert res <= tol and ex < 1e-11 and es < 1e-7


@pytest.mark.parametrize("mode", [0, 1])
def test_warm_started_steps_match_the_oracle_in_fewer_iterations(mode):
    """GMRES started from the previous step's velocity and the current
    tension (warm = 1) reaches the same tolerance, so the steps still match
    the oracle's dense solves, and needs fewer iterations than from zero."""
    from oracle import vesicle as ov
    from paper_1510_05616_amd import vesicle as pv
    import torch
    x, y, off = _set(sizes=(32, 32, 48), seed=4)
    d = 4.0
    g = ov.geometry(x, y, off)
    L0, A0 = ov.arc_lengths(g), ov.areas(x, y, off)
    f64 = dict(dtype=torch.float64, device="cuda")
    tol = 1e-13 if mode == 0 else 1e-12
    kw = dict(mode=mode, dt=0.005, kappa_b=1.0, mu=1.0, d=d, img_lo=-1, img_hi=1, L0=torch.as_tensor(L0, **f64),
              tol=tol, restart=64, max_iter=4000, nmax=48)
    cold, warm = pv.params(**kw), pv.params(warm=1, **kw)
    A0d = torch.as_tensor(A0, **f64)
    Vc, Vw = pv.Vesicles(x, y, off), pv.Vesicles(x, y, off)
    n = Vw.n
    uc, vc = torch.zeros(n, **f64), torch.zeros(n, **f64)
    uw, vw = torch.zeros(n, **f64), torch.zeros(n, **f64)
    xo, yo, so = x.copy(), y.copy(), np.zeros_like(x)
    saved = 0
    for k in range(4):
        itc, rc = Vc.time_step(cold, A0=A0d, reparam=True, uv=(uc, vc))
        itw, rw = Vw.time_step(warm, A0=A0d, reparam=True, uv=(uw, vw))
        xo, yo, so, _, _ = ov.time_step(xo, yo, so, off, 0.005, 1.0, 1.0, L0=L0, A0=A0, d=d, img_lo=-1, img_hi=1)
        torch.cuda.synchronize()
        ex = max(_rel(_np(Vw.x), xo), _rel(_np(Vw.y), yo))
        es = _rel(_np(Vw.sigma), so)
        print(f"mode={mode} step {k}: cold {itc} iterations ({rc:.1e}), warm {itw} ({rw:.1e}), "
              f"x {ex:.2e}, sigma {es:.2e}", flush=True)
        assert rw <= tol and ex < 1e-11 and es < 1e-7
        if k > 0:
            saved += itc - itw
    assert saved > 0


def test_invalid_curves_and_empty_set():
    from paper_1510_05616_amd.vesicle import Vesicles
    import torch
    x, y, off = _set(sizes=(32, 32), seed=5)
    # an odd curve between two good ones
    xo, yo = synth._ellipse(5.0, 0.0, 0.4, 0.2, 0.0, 7)[:2]
    x2 = np.concatenate([x[:32], xo, x[32:]])
    y2 = np.concatenate([y[:32], yo, y[32:]])
    off2 = np.array([0, 32, 39, 71], np.int32)
    V = Vesicles(x2, y2, off2)
    fb = V.forces(1.0)
    torch.cuda.synchronize()
    f = _np(fb[0])
    assert np.all(np.isnan(f[32:39])) and np.all(np.isfinite(f[:32])) and np.all(np.isfinite(f[39:]))
    E = Vesicles(np.zeros(0), np.zeros(0), np.array([0], np.int32))
    E.area_correct(torch.zeros(0, dtype=torch.float64, device="cuda"))
    E.reparameterize()


def test_channel_vesicle_set_one_step():
    # the 128k channel's 1,000 vesicles x 96 nodes, images -1..1 (d = 64 pi):
    # one step in FP64 converges, the step's constraint rows hold, the areas
    # are restored, and the forces of a sample of curves match the oracle
    from oracle import vesicle as ov
    from paper_1510_05616_amd import vesicle as pv
    import torch
    prob = synth.make_config(3)
    ves = prob.ves
    x, y, off = ves.x, ves.y, ves.curve_off
    f64 = dict(dtype=torch.float64, device="cuda")
    V = pv.Vesicles(x, y, off)
    L0, A0 = V.measure()
    p = pv.params(dt=1e-3, kappa_b=1.0, mu=prob.mu, d=prob.d, img_lo=-1, img_hi=1, L0=L0, tol=1e-10,
                  restart=64, max_iter=500, nmax=96)
    fb = V.forces(1.0)
    torch.cuda.synchronize()
    for c in (0, 417, 999):
        # the oracle on coordinates relative to the curve's first node (the
        # forces do not depend on the origin; the channel's x reaches 200,
        # whose rounding D_s^4 would amplify to 1e-8 in the oracle itself)
        s = slice(off[c], off[c + 1])
        g = ov.geometry(x[s] - x[s][0], y[s] - y[s][0], np.array([0, s.stop - s.start]))
        o = ov.forces(g, np.zeros(s.stop - s.start), 1.0)
        assert _rel(_np(fb[0])[s], o[0]) < 1e-9 and _rel(_np(fb[1])[s], o[1]) < 1e-9
    ws = V.workspace(p)
    z, it, res = V.step_solve(p, ws=ws)
    out, b = V.step_apply(p, z, ws=ws)
    torch.cuda.synchronize()
    r = np.linalg.norm(_np(out) - _np(b)) / np.linalg.norm(_np(b))
    print(f"config 3 vesicles: {it} GMRES iterations, residual {res:.2e} (recomputed {r:.2e})", flush=True)
    assert res <= 1e-10 and r < 2e-10
    # the step without reparameterization restores the areas exactly; the
    # reparameterization (step 9, after the area correction of step 8)
    # resamples at piecewise-linearly placed parameters and moves them slightly
    it2, res2 = V.time_step(p, A0=A0, reparam=False)
    L1, A1 = V.measure()
    torch.cuda.synchronize()
    assert it2 == it and res2 == res                    # the same solve, bit for bit
    assert _rel(_np(A1), _np(A0)) < 1e-12
    V.reparameterize()
    L2, A2 = V.measure()
    torch.cuda.synchronize()
    dA = np.abs(_np(A2) / _np(A0) - 1).max()
    print(f"length change {np.abs(_np(L1) / _np(L0) - 1).max():.2e}, area change by the reparameterization "
          f"{dA:.2e}", flush=True)
    assert dA < 1e-7
    assert np.isfinite(_np(V.x)).all() and np.isfinite(_np(V.sigma)).all()


# ---------------------------------------------------------------------------
# in the channel: Algorithm 1 with the response (steps 2-9)
# ---------------------------------------------------------------------------
def _channel_setup():
    walls, sy, d = synth.make_channel(256, 16)
    x1, y1 = synth._ellipse(math.pi, 0.1, 0.3, 0.15, 0.3, 32)[:2]
    x2, y2 = synth._ellipse(1.5, -0.3, 0.25, 0.15, -0.4, 32)[:2]
    return walls, sy, d, np.r_[x1, x2], np.r_[y1, y2], np.array([0, 32, 64], np.int32)


def test_total_force_and_channel_response():
    from oracle import vesicle as ov
    from paper_1510_05616_amd import vesicle as pv
    from paper_1510_05616_amd.cell import Cell
    import torch
    walls, sy, d, x, y, off = _channel_setup()
    mu, pd, M = 0.7, 0.9, 64
    sig = 0.3 * np.cos(np.arange(64) * 2 * math.pi / 32) + 1.0
    V = pv.Vesicles(x, y, off, sigma=sig)
    fx, fy = V.total_force(1.0)
    g = ov.geometry(x, y, off)
    o = ov.forces(g, sig, 1.0)
    ofx, ofy = o[0] + o[2], o[1] + o[3]
    torch.cuda.synchronize()
    assert _rel(_np(fx), ofx) < 1e-9 and _rel(_np(fy), ofy) < 1e-9
    cell = Cell(walls, sy, d, M, mu)
    cell.factor()
    u_o = ov.channel_response(walls, sy, d, M, mu, x, y, off, ofx, ofy, pd)[0]
    # FP32C: the data v, g carry the FP32C sums' ~1e-7; the cell system's
    # solve amplifies it (measured 7e-6 on u_resp)
    for mode, tol in ((0, 1e-9), (1, 2e-5)):
        ux, uy = V.channel_response(cell, fx, fy, pd, mode=mode)
        torch.cuda.synchronize()
        e = max(_rel(_np(ux), u_o[:, 0]), _rel(_np(uy), u_o[:, 1]))
        print(f"mode={mode} response rel error {e:.2e}", flush=True)
        assert e < tol


def test_channel_time_steps_match_the_oracle():
    # two steps of Algorithm 1 in the channel: forces with the current
    # tension, the channel's response, the preconditioned step, update, area
    # correction, reparameterization
    from oracle import vesicle as ov
    from paper_1510_05616_amd import vesicle as pv
    from paper_1510_05616_amd.cell import Cell
    import torch
    walls, sy, d, x, y, off = _channel_setup()
    mu, pd, M, dt, kb = 0.7, 0.9, 64, 0.005, 1.0
    g = ov.geometry(x, y, off)
    L0, A0 = ov.arc_lengths(g), ov.areas(x, y, off)
    f64 = dict(dtype=torch.float64, device="cuda")
    cell = Cell(walls, sy, d, M, mu)
    cell.factor()
    V = pv.Vesicles(x, y, off)
    L0d, A0d = torch.as_tensor(L0, **f64), torch.as_tensor(A0, **f64)
    xo, yo, so = x.copy(), y.copy(), np.zeros(64)
    for k in range(2):
        fx, fy = V.total_force(kb)
        ur = V.channel_response(cell, fx, fy, pd)
        p = pv.params(dt=dt, kappa_b=kb, mu=mu, d=d, img_lo=-1, img_hi=1, L0=L0d, u_resp=ur, tol=1e-13,
                      nmax=32)
        it, res = V.time_step(p, A0=A0d)
        go = ov.geometry(xo, yo, off)
        o = ov.forces(go, so, kb)
        uo = ov.channel_response(walls, sy, d, M, mu, xo, yo, off, o[0] + o[2], o[1] + o[3], pd)[0]
        xo, yo, so, _, _ = ov.time_step(xo, yo, so, off, dt, kb, mu, L0=L0, A0=A0, u_resp=(uo[:, 0], uo[:, 1]),
                                        d=d, img_lo=-1, img_hi=1)
        torch.cuda.synchronize()
        ex = max(_rel(_np(V.x), xo), _rel(_np(V.y), yo))
        es = _rel(_np(V.sigma), so)
        print(f"channel step {k}: {it} iterations, residual {res:.1e}, x {ex:.2e}, sigma {es:.2e}", flush=True)
        assert res <= 1e-13 and ex < 1e-11 and es < 1e-8


def _gpu_relax(dt, t_end, corrections):
    from oracle import vesicle as ov
    from paper_1510_05616_amd import vesicle as pv
    import torch
    x, y = synth._ellipse(0.0, 0.0, 1.0, 0.4, 0.2, 32)[:2]
    off = np.array([0, 32], np.int32)
    V = pv.Vesicles(x, y, off)
    L0, A0 = V.measure()
    p = pv.params(dt=dt, kappa_b=1.0, mu=1.0, L0=L0 if corrections else None, tol=1e-13, nmax=32)
    ws = V.workspace(p)
    for _ in range(int(round(t_end / dt))):
        V.time_step(p, A0=A0 if corrections else None, reparam=False, ws=ws)
    L1, A1 = V.measure()
    torch.cuda.synchronize()
    return (_np(V.x), _np(V.y), abs(float(_np(L1)[0] / _np(L0)[0]) - 1), abs(float(_np(A1)[0] / _np(A0)[0]) - 1))


@pytest.mark.parametrize("corrections", [True, False])
def test_table4_convergence_orders_on_the_gpu(corrections):
    # Table 4's experiment with the GPU time step (the oracle's pin of the
    # same orders is in test_oracle_vesicle): t = 0.1, dt = 0.01 / M
    Ms = (2, 4, 8)
    ref = _gpu_relax(0.01 / 64, 0.1, corrections)
    out = {M: _gpu_relax(0.01 / M, 0.1, corrections) for M in Ms}
    eL = [out[M][2] for M in Ms]
    ex = [np.abs(np.r_[out[M][0] - ref[0], out[M][1] - ref[1]]).max() for M in Ms]
    rL = [eL[i] / eL[i + 1] for i in range(2)]
    rx = [ex[i] / ex[i + 1] for i in range(2)]
    print(f"GPU corrections={corrections}: L errors {eL} ratios {rL}; x ratios {rx}", flush=True)
    assert all(1.6 < r < 2.5 for r in rx), rx
    if corrections:
        assert all(3.5 < r < 5.5 for r in rL), rL
        assert max(out[M][3] for M in Ms) < 1e-12
    else:
        assert all(1.5 < r < 2.5 for r in rL), rL
