"""Pins of the FP64 oracle against facts fixed by the mathematics.

None of these tests re-types the oracle's formulas: each compares the oracle
with a closed form, an identity of Stokes flow, or a second oracle evaluation
of a transformed problem.
  * Kress weights integrate log(4 sin^2((t_i - t)/2)) cos(m t) exactly
    (closed form -2 pi cos(m t_i) / m, and 0 for m = 0).
  * Circle of radius R, constant density c: on-curve single layer equals
    (R / (4 mu)) (1 - 2 ln R) c.
  * Double layer of a rigid motion (translation, rotation) with outward
    normals: -u inside, 0 outside, -u/2 on the curve (principal value plus the
    diagonal limit), from the jump relation (Section 2.1, Eq. (JR)).
  * Green's identity for the Stokeslet of an exterior point: S[t] - D[u] = u
    inside, 0 outside, u/2 on the curve, converging spectrally in N.
  * Stokeslet symmetry S(x, y) = S(y, x), S_ij = S_ji.
  * The image sum equals explicitly replicated sources.
  * Translation and rotation covariance; linearity in the density.
"""
import math

import numpy as np
import pytest

import synth
from synth import CurveSet


def _stokeslet(xx, yy, zx, zy, F, mu):
    rx, ry = xx - zx, yy - zy
    q = rx * rx + ry * ry
    rf = rx * F[0] + ry * F[1]
    c = 1.0 / (4.0 * np.pi * mu)
    return c * (-0.5 * np.log(q) * F[0] + rx * rf / q), c * (-0.5 * np.log(q) * F[1] + ry * rf / q)


def _with_density(c, fx, fy):
    return CurveSet(c.x, c.y, c.nx, c.ny, c.w, c.kappa, np.asarray(fx, float),
                    np.asarray(fy, float), c.curve_off)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N", [8, 16, 32, 64, 96])
def test_kress_weights_exact_on_trig(oracle_lib, N):
    R = oracle_lib.kress_weights(N)
    t = 2 * np.pi * np.arange(N) / N
    idx = (np.arange(N)[:, None] - np.arange(N)[None, :]) % N
    W = R[idx]                                # W[i, k] = R_{(i - k) mod N}
    assert abs(R.sum()) < 1e-13
    for m in range(1, N // 2 + 1):
        for fn in (np.cos, np.sin):
            if fn is np.sin and m == N // 2:
                continue                      # sin(N/2 t) vanishes at the nodes
            lhs = W @ fn(m * t)
            rhs = -(2 * np.pi / m) * fn(m * t)
            assert np.abs(lhs - rhs).max() < 1e-12 * max(1.0, np.abs(rhs).max()), (N, m)


@pytest.mark.parametrize("R,mu,N", [(0.7, 0.7, 64), (1.3, 1.0, 32), (0.25, 2.0, 128)])
def test_circle_constant_density(oracle_lib, R, mu, N):
    c = synth.ellipse_curve(R, R, N, center=(0.3, -0.2), phi=0.4)
    cv = np.array([0.8, -1.1])
    c = _with_density(c, np.full(N, cv[0]), np.full(N, cv[1]))
    oc = np.zeros(N, np.int32)
    on = np.arange(N, dtype=np.int32)
    u, v = oracle_lib.slp(c, c.x, c.y, oc, on, mu=mu)
    exact = (R / (4 * mu)) * (1 - 2 * math.log(R)) * cv
    assert np.abs(u - exact[0]).max() < 1e-14 * 10
    assert np.abs(v - exact[1]).max() < 1e-14 * 10


@pytest.mark.parametrize("motion", ["translation", "rotation"])
def test_dlp_rigid_motion_identity(oracle_lib, motion):
    a, b, N = 0.3, 0.17, 128
    c = synth.ellipse_curve(a, b, N, center=(0.2, 0.1), phi=0.3)
    if motion == "translation":
        ux, uy = np.full(N, 0.9), np.full(N, -0.4)
        rigid = lambda X, Y: (np.full_like(X, 0.9), np.full_like(Y, -0.4))
    else:
        om = 0.7
        ux, uy = -om * c.y, om * c.x
        rigid = lambda X, Y: (-om * Y, om * X)
    cd = _with_density(c, ux, uy)
    Xi = np.array([0.2, 0.3, 0.1, 0.15]); Yi = np.array([0.1, 0.12, 0.05, 0.08])
    Xo = np.array([0.9, -0.5, 0.2]); Yo = np.array([0.1, 0.0, 0.6])
    u, v = oracle_lib.dlp(cd, Xi, Yi)
    ex, ey = rigid(Xi, Yi)
    assert np.abs(u + ex).max() < 1e-12 and np.abs(v + ey).max() < 1e-12
    u, v = oracle_lib.dlp(cd, Xo, Yo)
    assert np.abs(u).max() < 1e-12 and np.abs(v).max() < 1e-12
    oc = np.zeros(N, np.int32); on = np.arange(N, dtype=np.int32)
    u, v = oracle_lib.dlp(cd, c.x, c.y, oc, on)
    assert np.abs(u + 0.5 * ux).max() < 1e-12 and np.abs(v + 0.5 * uy).max() < 1e-12


def _green_parts(oracle_lib, N, z, F, mu, X, Y, on_curve=False):
    c = synth.ellipse_curve(0.3, 0.17, N, phi=0.2)
    rx, ry = c.x - z[0], c.y - z[1]
    q = rx * rx + ry * ry
    rn = rx * c.nx + ry * c.ny
    rF = rx * F[0] + ry * F[1]
    # traction of the Stokeslet flow on the curve (Section 2.1, Eq. (K)),
    # r = y - z, target normal n_y
    tx = -(1 / np.pi) * rx * rF * rn / q ** 2
    ty = -(1 / np.pi) * ry * rF * rn / q ** 2
    ux, uy = _stokeslet(c.x, c.y, z[0], z[1], F, mu)
    cs, cd = _with_density(c, tx, ty), _with_density(c, ux, uy)
    if on_curve:
        oc = np.zeros(N, np.int32); on = np.arange(N, dtype=np.int32)
        su, sv = oracle_lib.slp(cs, c.x, c.y, oc, on, mu=mu)
        du, dv = oracle_lib.dlp(cd, c.x, c.y, oc, on)
        return su - du, sv - dv, 0.5 * ux, 0.5 * uy
    su, sv = oracle_lib.slp(cs, X, Y, mu=mu)
    du, dv = oracle_lib.dlp(cd, X, Y)
    return su - du, sv - dv, None, None


def test_green_reproduction_spectral(oracle_lib):
    z, F, mu = np.array([0.6, 0.25]), np.array([0.7, -0.4]), 0.8
    Xi, Yi = np.array([0.05, -0.08, 0.1]), np.array([0.02, 0.0, 0.03])
    Xo, Yo = np.array([0.9, -0.6]), np.array([0.0, 0.3])
    ex, ey = _stokeslet(Xi, Yi, z[0], z[1], F, mu)
    errs_in, errs_on = [], []
    for N in (16, 32, 64, 128):
        gu, gv, _, _ = _green_parts(oracle_lib, N, z, F, mu, Xi, Yi)
        errs_in.append(max(np.abs(gu - ex).max(), np.abs(gv - ey).max()))
        gu, gv, hu, hv = _green_parts(oracle_lib, N, z, F, mu, None, None, on_curve=True)
        errs_on.append(max(np.abs(gu - hu).max(), np.abs(gv - hv).max()))
    # spectral: each doubling gains several digits until round-off
    assert errs_in[-1] < 1e-14 and errs_on[-1] < 1e-14
    assert errs_in[1] < errs_in[0] / 50 and errs_on[1] < errs_on[0] / 50
    assert errs_in[2] < 1e-10 and errs_on[2] < 1e-12
    gu, gv, _, _ = _green_parts(oracle_lib, 128, z, F, mu, Xo, Yo)
    assert np.abs(gu).max() < 1e-14 and np.abs(gv).max() < 1e-14


def test_stokeslet_symmetry(oracle_lib):
    rng = np.random.default_rng(11)
    for _ in range(5):
        p, q = rng.normal(size=2), rng.normal(size=2)
        S_xy = np.zeros((2, 2)); S_yx = np.zeros((2, 2))
        for k in range(2):
            f = np.zeros(2); f[k] = 1.0
            src = CurveSet(np.array([q[0]]), np.array([q[1]]), np.zeros(1), np.zeros(1),
                           np.ones(1), np.zeros(1), np.array([f[0]]), np.array([f[1]]),
                           np.array([0, 1], np.int32))
            u, v = oracle_lib.slp(src, np.array([p[0]]), np.array([p[1]]), mu=1.3)
            S_xy[:, k] = [u[0], v[0]]
            src = CurveSet(np.array([p[0]]), np.array([p[1]]), np.zeros(1), np.zeros(1),
                           np.ones(1), np.zeros(1), np.array([f[0]]), np.array([f[1]]),
                           np.array([0, 1], np.int32))
            u, v = oracle_lib.slp(src, np.array([q[0]]), np.array([q[1]]), mu=1.3)
            S_yx[:, k] = [u[0], v[0]]
        assert np.allclose(S_xy, S_yx, rtol=0, atol=1e-15)
        assert abs(S_xy[0, 1] - S_xy[1, 0]) < 1e-15


def _replicate(cs, d):
    parts = []
    for n in (-1, 0, 1):
        for c in range(cs.n_curves):
            s = slice(cs.curve_off[c], cs.curve_off[c + 1])
            parts.append((cs.x[s] + n * d, cs.y[s], cs.nx[s], cs.ny[s], cs.w[s],
                          cs.kappa[s], cs.fx[s], cs.fy[s]))
    return synth.concat_curves(parts)


def test_image_sum_equals_replicated_sources(oracle_lib):
    p = synth.make_config(1)
    t = p.trg
    rep_v = _replicate(p.ves, p.d)
    rep_w = _replicate(p.wall, p.d)
    shift_v = p.ves.n_curves          # the n = 0 copies follow the n = -1 copies
    shift_w = p.wall.n_curves
    u1, v1 = oracle_lib.slp(p.ves, t.x, t.y, t.ves_curve, t.ves_node, p.d, -1, 1, p.mu)
    oc = np.where(t.ves_curve >= 0, t.ves_curve + shift_v, -1).astype(np.int32)
    on = np.where(t.ves_node >= 0, t.ves_node + p.ves.n_nodes, -1).astype(np.int32)
    u2, v2 = oracle_lib.slp(rep_v, t.x, t.y, oc, on, 0.0, 0, 0, p.mu)
    sc = max(np.abs(u1).max(), np.abs(v1).max())
    assert max(np.abs(u1 - u2).max(), np.abs(v1 - v2).max()) < 1e-13 * sc
    u1, v1 = oracle_lib.dlp(p.wall, t.x, t.y, t.wall_curve, t.wall_node, p.d, -1, 1)
    oc = np.where(t.wall_curve >= 0, t.wall_curve + shift_w, -1).astype(np.int32)
    on = np.where(t.wall_node >= 0, t.wall_node + p.wall.n_nodes, -1).astype(np.int32)
    u2, v2 = oracle_lib.dlp(rep_w, t.x, t.y, oc, on, 0.0, 0, 0)
    sc = max(np.abs(u1).max(), np.abs(v1).max())
    assert max(np.abs(u1 - u2).max(), np.abs(v1 - v2).max()) < 1e-13 * sc


def test_single_images_sum_to_range(oracle_lib):
    p = synth.make_config(1)
    t = p.trg
    tot = oracle_lib.slp(p.ves, t.x, t.y, t.ves_curve, t.ves_node, p.d, -1, 1, p.mu)
    parts = [oracle_lib.slp(p.ves, t.x, t.y, t.ves_curve, t.ves_node, p.d, n, n, p.mu)
             for n in (-1, 0, 1)]
    sc = np.abs(tot[0]).max()
    assert np.abs(tot[0] - sum(q[0] for q in parts)).max() < 1e-13 * sc


def _rotate(cs, phi, shift):
    c, s = math.cos(phi), math.sin(phi)
    R = lambda u, v: (c * u - s * v, s * u + c * v)
    x, y = R(cs.x, cs.y)
    nx, ny = R(cs.nx, cs.ny)
    fx, fy = R(cs.fx, cs.fy)
    return CurveSet(x + shift[0], y + shift[1], nx, ny, cs.w, cs.kappa, fx, fy, cs.curve_off)


def test_translation_rotation_covariance(oracle_lib):
    p = synth.make_config(1)
    t = p.trg
    phi, sh = 0.7, (1.3, -0.4)
    c, s = math.cos(phi), math.sin(phi)
    tx, ty = c * t.x - s * t.y + sh[0], s * t.x + c * t.y + sh[1]
    for fn, src, oc, on in ((oracle_lib.slp, p.ves, t.ves_curve, t.ves_node),
                            (oracle_lib.dlp, p.wall, t.wall_curve, t.wall_node)):
        kw = dict(mu=p.mu) if fn is oracle_lib.slp else {}
        u, v = fn(src, t.x, t.y, oc, on, 0.0, 0, 0, **kw)
        ur, vr = fn(_rotate(src, phi, sh), tx, ty, oc, on, 0.0, 0, 0, **kw)
        sc = max(np.abs(u).max(), np.abs(v).max())
        assert np.abs(ur - (c * u - s * v)).max() < 1e-12 * sc
        assert np.abs(vr - (s * u + c * v)).max() < 1e-12 * sc


def test_linearity_in_density(oracle_lib):
    p = synth.make_config(1)
    t = p.trg
    rng = np.random.default_rng(3)
    g1, g2 = rng.normal(size=(2, p.ves.n_nodes))
    a, b = 0.7, -1.9
    s1 = _with_density(p.ves, g1, g2)
    s2 = _with_density(p.ves, g2, -g1)
    s12 = _with_density(p.ves, a * g1 + b * g2, a * g2 - b * g1)
    args = (t.x, t.y, t.ves_curve, t.ves_node, p.d, -1, 1, p.mu)
    u1, v1 = oracle_lib.slp(s1, *args)
    u2, v2 = oracle_lib.slp(s2, *args)
    u, v = oracle_lib.slp(s12, *args)
    sc = np.abs(u).max()
    assert np.abs(u - (a * u1 + b * u2)).max() < 1e-13 * sc
    assert np.abs(v - (a * v1 + b * v2)).max() < 1e-13 * sc


def test_bad_arguments(oracle_lib):
    c = synth.ellipse_curve(0.3, 0.2, 7, fx=np.cos, fy=np.sin)
    oc = np.zeros(7, np.int32); on = np.arange(7, dtype=np.int32)
    with pytest.raises(ValueError):
        oracle_lib.slp(c, c.x, c.y, oc, on)           # odd N with self targets
    c = synth.ellipse_curve(0.3, 0.2, 8, fx=np.cos, fy=np.sin)
    oc = np.zeros(8, np.int32); on = np.arange(8, dtype=np.int32) + 1
    with pytest.raises(ValueError):
        oracle_lib.slp(c, c.x, c.y, oc, on)           # on_node outside its curve
