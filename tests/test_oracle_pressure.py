"""Pins of the oracle's pressure and traction sums (CPU, no GPU) against facts
that the mathematics fixes, independent of the formulas' transcription:

  * single-layer pressure of a circle of constant density c (closed form):
    p = R (c . x) / |x|^2 outside, 0 inside (x from the centre);
  * Green's identity for a Stokeslet outside a curve, in velocity and in
    pressure: S[t] - D[u] = u and Q[t] - P[u] = p inside, 0 outside, with the
    traction data t taken from the oracle's own traction sum (a one-node
    source at the Stokeslet), converging spectrally in N;
  * the traction sum equals the stress -p m + mu (grad u + grad u^T) m of the
    single-layer velocity and pressure fields (central differences);
  * each velocity/pressure pair solves the Stokes equations,
    mu Lap u = grad p (finite differences), for both layers;
  * image sums equal explicitly replicated sources.
"""
import numpy as np
import pytest

import synth
from synth import CurveSet


def _with_density(c, fx, fy):
    return CurveSet(c.x, c.y, c.nx, c.ny, c.w, c.kappa, np.asarray(fx, float), np.asarray(fy, float),
                    c.curve_off)


def _point(z, F):
    """A one-node 'curve' with unit weight: a point force F at z."""
    return CurveSet(np.array([z[0]]), np.array([z[1]]), np.zeros(1), np.zeros(1), np.ones(1), np.zeros(1),
                    np.array([F[0]]), np.array([F[1]]), np.array([0, 1], np.int32))


def _random_density(c, seed, K=6):
    rng = np.random.default_rng(seed)
    N = c.x.shape[0]
    th = 2 * np.pi * np.arange(N) / N
    f = []
    for _ in range(2):
        v = np.zeros(N)
        for k in range(1, K + 1):
            v += k ** -2.0 * (rng.normal() * np.cos(k * th) + rng.normal() * np.sin(k * th))
        f.append(v + rng.normal())
    return _with_density(c, f[0], f[1])


@pytest.mark.parametrize("R,N", [(0.7, 64), (1.3, 128)])
def test_slp_pressure_of_a_circle(oracle_lib, R, N):
    ctr = np.array([0.3, -0.2])
    c = synth.ellipse_curve(R, R, N, center=tuple(ctr), phi=0.4)
    cv = np.array([0.8, -1.1])
    c = _with_density(c, np.full(N, cv[0]), np.full(N, cv[1]))
    ang = np.array([0.1, 1.7, 3.0, 4.4])
    for rho, inside in ((0.4 * R, True), (0.6 * R, True), (1.8 * R, False), (3.0 * R, False)):
        X = ctr[0] + rho * np.cos(ang)
        Y = ctr[1] + rho * np.sin(ang)
        p = oracle_lib.slp_pressure(c, X, Y)
        exact = np.zeros_like(X) if inside else R * ((X - ctr[0]) * cv[0] + (Y - ctr[1]) * cv[1]) / rho ** 2
        assert np.abs(p - exact).max() < 1e-12, (rho, p, exact)


def _green(oracle_lib, N, z, F, mu, X, Y):
    c = synth.ellipse_curve(0.3, 0.17, N, phi=0.2)
    pt = _point(z, F)
    # traction of the Stokeslet flow on the curve, from the oracle's traction
    # sum with the curve's outward normals as target normals
    tx, ty = oracle_lib.slp_traction(pt, c.x, c.y, c.nx, c.ny)
    ux, uy = oracle_lib.slp(pt, c.x, c.y, mu=mu)
    cs, cd = _with_density(c, tx, ty), _with_density(c, ux, uy)
    su, sv = oracle_lib.slp(cs, X, Y, mu=mu)
    du, dv = oracle_lib.dlp(cd, X, Y)
    sp = oracle_lib.slp_pressure(cs, X, Y)
    dp = oracle_lib.dlp_pressure(cd, X, Y, mu=mu)
    return su - du, sv - dv, sp - dp


def test_green_identity_for_velocity_and_pressure(oracle_lib):
    z, F, mu = np.array([0.6, 0.25]), np.array([0.7, -0.4]), 0.8
    Xi, Yi = np.array([0.05, -0.08, 0.1]), np.array([0.02, 0.0, 0.03])
    Xo, Yo = np.array([0.9, -0.6]), np.array([0.0, 0.3])
    eu, ev = oracle_lib.slp(_point(z, F), Xi, Yi, mu=mu)
    ep = oracle_lib.slp_pressure(_point(z, F), Xi, Yi)
    # the Stokeslet pressure itself: (1/2 pi) (x - z) . F / |x - z|^2
    rx, ry = Xi - z[0], Yi - z[1]
    assert np.allclose(ep, (rx * F[0] + ry * F[1]) / (rx * rx + ry * ry) / (2 * np.pi), rtol=1e-14, atol=0)
    errs = []
    for N in (16, 32, 64, 128):
        gu, gv, gp = _green(oracle_lib, N, z, F, mu, Xi, Yi)
        errs.append((max(np.abs(gu - eu).max(), np.abs(gv - ev).max()), np.abs(gp - ep).max()))
    assert errs[-1][0] < 1e-13 and errs[-1][1] < 1e-12, errs
    assert errs[1][0] < errs[0][0] / 50 and errs[1][1] < errs[0][1] / 50, errs
    gu, gv, gp = _green(oracle_lib, 128, z, F, mu, Xo, Yo)
    assert np.abs(gu).max() < 1e-13 and np.abs(gv).max() < 1e-13 and np.abs(gp).max() < 1e-12


def test_traction_is_the_stress_of_the_single_layer_fields(oracle_lib):
    mu = 1.7
    c = _random_density(synth.ellipse_curve(0.3, 0.17, 256, center=(0.1, 0.05), phi=0.5), seed=3)
    rng = np.random.default_rng(4)
    ang = rng.uniform(0, 2 * np.pi, 6)
    X = 0.1 + 0.55 * np.cos(ang)
    Y = 0.05 + 0.45 * np.sin(ang)
    th = rng.uniform(0, 2 * np.pi, 6)
    mx, my = np.cos(th), np.sin(th)
    h = 1e-5
    g = np.zeros((6, 2, 2))                          # g[:, i, j] = d u_i / d x_j
    for j, (ex, ey) in enumerate(((h, 0.0), (0.0, h))):
        up, vp = oracle_lib.slp(c, X + ex, Y + ey, mu=mu)
        um, vm = oracle_lib.slp(c, X - ex, Y - ey, mu=mu)
        g[:, 0, j] = (up - um) / (2 * h)
        g[:, 1, j] = (vp - vm) / (2 * h)
    p = oracle_lib.slp_pressure(c, X, Y)
    m = np.stack([mx, my], 1)
    e = g + np.transpose(g, (0, 2, 1))
    t_fd = -p[:, None] * m + mu * np.einsum("kij,kj->ki", e, m)
    tx, ty = oracle_lib.slp_traction(c, X, Y, mx, my)
    t = np.stack([tx, ty], 1)
    assert np.abs(t - t_fd).max() < 1e-6 * np.abs(t).max(), (t, t_fd)


@pytest.mark.parametrize("layer", ["single", "double"])
def test_velocity_and_pressure_solve_stokes(oracle_lib, layer):
    mu = 0.6
    c = _random_density(synth.ellipse_curve(0.3, 0.17, 256, center=(0.0, 0.0), phi=0.2), seed=7)
    X = np.array([0.7, -0.2, 0.05, 0.9])
    Y = np.array([0.1, 0.5, -0.45, -0.4])
    if layer == "single":
        vel = lambda x, y: oracle_lib.slp(c, x, y, mu=mu)
        prs = lambda x, y: oracle_lib.slp_pressure(c, x, y)
    else:
        vel = lambda x, y: oracle_lib.dlp(c, x, y)
        prs = lambda x, y: oracle_lib.dlp_pressure(c, x, y, mu=mu)
    h = 2e-3
    u0 = np.stack(vel(X, Y), 1)
    lap = -4 * u0
    for ex, ey in ((h, 0), (-h, 0), (0, h), (0, -h)):
        lap = lap + np.stack(vel(X + ex, Y + ey), 1)
    lap /= h * h
    k = 1e-5
    gp = np.stack([(prs(X + k, Y) - prs(X - k, Y)) / (2 * k), (prs(X, Y + k) - prs(X, Y - k)) / (2 * k)], 1)
    assert np.abs(mu * lap - gp).max() < 2e-4 * np.abs(gp).max(), (mu * lap, gp)
    # a sign or factor slip in the pressure would break the balance by O(1)
    assert np.abs(gp).max() > 1e-3


def test_pressure_and_traction_image_sums_are_replications(oracle_lib):
    rng = np.random.default_rng(12)
    c = _random_density(synth.ellipse_curve(0.3, 0.17, 32, center=(0.5, 0.0), phi=0.3), seed=12)
    d, lo, hi = 2.5, -2, 1
    X, Y = rng.uniform(-1, 1, 7), rng.uniform(-1, 1, 7)
    th = rng.uniform(0, 2 * np.pi, 7)
    mx, my = np.cos(th), np.sin(th)
    rep = CurveSet(*(np.concatenate([getattr(c, a) + (n * d if a == "x" else 0.0) for n in range(lo, hi + 1)])
                     for a in ("x", "y", "nx", "ny", "w", "kappa", "fx", "fy")),
                   curve_off=np.array([0, 32 * (hi - lo + 1)], np.int32))
    for img, ref in ((lambda: oracle_lib.slp_pressure(c, X, Y, d, lo, hi), lambda: oracle_lib.slp_pressure(rep, X, Y)),
                     (lambda: oracle_lib.dlp_pressure(c, X, Y, d, lo, hi, 1.3),
                      lambda: oracle_lib.dlp_pressure(rep, X, Y, mu=1.3))):
        a, b = img(), ref()
        assert np.abs(a - b).max() < 1e-13 * max(1.0, np.abs(b).max())
    a = oracle_lib.slp_traction(c, X, Y, mx, my, d, lo, hi)
    b = oracle_lib.slp_traction(rep, X, Y, mx, my)
    assert max(np.abs(a[0] - b[0]).max(), np.abs(a[1] - b[1]).max()) < 1e-13 * max(1.0, np.abs(b[0]).max())
