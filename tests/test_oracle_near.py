"""Pins of the near-field references in oracle/near.py against closed forms:
trigonometric interpolation is exact on band-limited data (including the
split Nyquist mode), the upsampled ellipse and its speed equal the closed
form, upsampled quadrature converges to the integral computed from the closed
form curve, the target features reconstruct the target and the density
window, the tanh GELU stays within 1e-3 of x Phi(x), the MLP gradient equals
central finite differences, and one Adam step from rest moves each weight by
lr against the sign of its gradient."""
import math

import numpy as np
import pytest
from scipy.special import erf

import synth
from oracle import near


def test_upsample_exact_on_trig_polynomials():
    for N in (16, 32, 64):
        t = 2 * np.pi * np.arange(N) / N
        f = lambda s: 0.3 + np.cos(3 * s) - 0.5 * np.sin(5 * s) + 0.25 * np.cos((N // 2 - 1) * s)
        for P in (1, 2, 8):
            M = P * N
            tf = 2 * np.pi * np.arange(M) / M
            assert np.abs(near.upsample_periodic(f(t), P) - f(tf)).max() < 1e-13


def test_upsample_nyquist_split():
    N, P = 16, 4
    t = 2 * np.pi * np.arange(N) / N
    tf = 2 * np.pi * np.arange(N * P) / (N * P)
    # the samples of cos(N/2 t) interpolate to cos(N/2 t) itself
    assert np.abs(near.upsample_periodic(np.cos(N // 2 * t), P) - np.cos(N // 2 * tf)).max() < 1e-13


def test_spectral_derivative():
    N = 32
    t = 2 * np.pi * np.arange(N) / N
    f = np.sin(2 * t) + 0.4 * np.cos(7 * t)
    df = 2 * np.cos(2 * t) - 2.8 * np.sin(7 * t)
    assert np.abs(near.spectral_derivative(f) - df).max() < 1e-12


def test_upsampled_ellipse_matches_closed_form():
    a, b, N, P, phi = 0.35, 0.15, 64, 8, 0.4
    c = synth.ellipse_curve(a, b, N, center=(0.2, -0.1), phi=phi, fx=lambda t: np.cos(2 * t),
                            fy=lambda t: np.sin(3 * t))
    xu, yu, wu, fxu, fyu = near.upsample_curve(c.x, c.y, c.fx, c.fy, P)
    fine = synth.ellipse_curve(a, b, N * P, center=(0.2, -0.1), phi=phi, fx=lambda t: np.cos(2 * t),
                               fy=lambda t: np.sin(3 * t))
    for u, v in ((xu, fine.x), (yu, fine.y), (wu, fine.w), (fxu, fine.fx), (fyu, fine.fy)):
        assert np.abs(u - v).max() < 1e-13


def test_label_is_zero_without_upsampling():
    c = synth.make_curve(0.8, 64, K=8, seed=3)
    tx, ty = c.x[:5] + 0.01, c.y[:5] + 0.02
    du, dv = near.near_label(c.x, c.y, c.fx, c.fy, c.w, tx, ty, P=1)
    assert np.abs(du).max() < 1e-15 and np.abs(dv).max() < 1e-15   # weights re-derived spectrally


def test_upsampled_quadrature_converges_to_the_integral():
    # band-limited density and an ellipse: the fine-node trapezoid of the
    # closed-form data is the integral to round-off
    a, b, N = 0.3, 0.17, 64
    fxf = lambda t: np.cos(t) + 0.3 * np.sin(5 * t)
    fyf = lambda t: 0.5 * np.sin(2 * t) - 0.2 * np.cos(6 * t)
    c = synth.ellipse_curve(a, b, N, fx=fxf, fy=fyf)
    truth = synth.ellipse_curve(a, b, 32768, fx=fxf, fy=fyf)
    h = c.w.sum() / N
    k = np.arange(0, N, 7)
    errs = {}
    for delta in (0.5, 1.0, 2.0):
        tx = c.x[k] + delta * h * c.nx[k]
        ty = c.y[k] + delta * h * c.ny[k]
        ut, vt = near.slp_trap(truth.x, truth.y, truth.w, truth.fx, truth.fy, tx, ty)
        sc = np.hypot(ut, vt).max()
        for P in (1, 8, 32):
            xu, yu, wu, fu, gu = near.upsample_curve(c.x, c.y, c.fx, c.fy, P)
            u, v = near.slp_trap(xu, yu, wu, fu, gu, tx, ty)
            errs[(delta, P)] = np.hypot(u - ut, v - vt).max() / sc
    assert errs[(0.5, 32)] < 1e-12 and errs[(1.0, 32)] < 1e-12
    assert errs[(0.5, 8)] < 1e-8 and errs[(2.0, 8)] < 1e-12
    assert errs[(0.5, 1)] > 1e-4 > errs[(0.5, 8)] * 1e3


def test_features_reconstruct_target_and_window():
    c = synth.make_curve(0.75, 64, K=8, seed=5, phi=0.3)
    rng = np.random.default_rng(1)
    N = 64
    h = c.w.sum() / N
    for _ in range(40):
        th = rng.uniform(0, 2 * np.pi)
        k = int(th / (2 * np.pi) * N) % N
        delta = h * 10 ** rng.uniform(np.log10(0.05), np.log10(5))
        px = np.interp(th, 2 * np.pi * np.arange(N + 1) / N, np.append(c.x, c.x[0])) + delta * c.nx[k]
        py = np.interp(th, 2 * np.pi * np.arange(N + 1) / N, np.append(c.y, c.y[0])) + delta * c.ny[k]
        f, t0, n0, hh, F = near.features_one(c.x, c.y, c.nx, c.ny, c.kappa, c.w, c.fx, c.fy, px, py)
        assert abs(hh - h) < 1e-15
        d2 = (px - c.x) ** 2 + (py - c.y) ** 2
        ks = int(np.argmin(d2))
        assert abs(f[2] - math.log(math.sqrt(d2[ks]) / h)) < 1e-12   # log distance to the nearest node
        # the target is x_k0 + h (s t0 + n_off n0) for the node k0 whose frame it uses
        k0 = [j for j in range(N) if abs(-c.ny[j] - t0[0]) < 1e-15 and abs(c.nx[j] - t0[1]) < 1e-15][0]
        assert k0 in (ks, (ks - 1) % N) and f[0] >= 0.0 or k0 == (ks - 1) % N
        assert abs(c.x[k0] + h * (f[0] * t0[0] + f[1] * n0[0]) - px) < 1e-13
        assert abs(c.y[k0] + h * (f[0] * t0[1] + f[1] * n0[1]) - py) < 1e-13
        # the density window k0-3 .. k0+4 comes back from (f_t, f_n) * F
        idx = [(k0 + j) % N for j in range(-3, 5)]
        fx = (f[4:12] * t0[0] + f[12:20] * n0[0]) * F
        fy = (f[4:12] * t0[1] + f[12:20] * n0[1]) * F
        assert np.abs(fx - c.fx[idx]).max() < 1e-13 and np.abs(fy - c.fy[idx]).max() < 1e-13
        assert abs(np.hypot(f[4:12], f[12:20]).max() - 1.0) < 1e-14
        assert abs(f[3] - c.kappa[k0] * h) < 1e-15


def test_gelu_tanh_form_close_to_exact_gelu():
    z = np.linspace(-6, 6, 2001)
    exact = z * 0.5 * (1 + erf(z / math.sqrt(2)))
    assert np.abs(near.gelu(z) - exact).max() < 1e-3
    # and its derivative matches a central difference of itself
    e = 1e-6
    fd = (near.gelu(z + e) - near.gelu(z - e)) / (2 * e)
    assert np.abs(near.gelu_grad(z) - fd).max() < 1e-8


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = near.init_params(seed=4, mu_in=rng.normal(size=20) * 0.1, sd_in=1 + rng.random(20))
    X = rng.normal(size=(7, 20))
    T = rng.normal(size=(7, 2))
    L, g = near.mlp_loss_grad(p, X, T)
    eps = 1e-6
    for name in ("W1", "b1", "W2", "b3", "W4", "b4"):
        flat = p[name].reshape(-1)
        for j in rng.choice(flat.size, min(6, flat.size), replace=False):
            old = flat[j]
            flat[j] = old + eps
            Lp, _ = near.mlp_loss_grad(p, X, T)
            flat[j] = old - eps
            Lm, _ = near.mlp_loss_grad(p, X, T)
            flat[j] = old
            fd = (Lp - Lm) / (2 * eps)
            gj = g[name].reshape(-1)[j]
            assert abs(fd - gj) <= 1e-7 * max(1.0, abs(fd)), (name, j, fd, gj)


def test_adam_first_step():
    p = {"W": np.array([1.0, -2.0, 0.5])}
    g = {"W": np.array([0.3, -4.0, 1e-3])}
    st = {}
    near.adam_step(p, g, st, lr=0.01)
    assert np.allclose(p["W"], [1.0 - 0.01, -2.0 + 0.01, 0.5 - 0.01 * 1e-3 / (1e-3 + 1e-8)], atol=1e-12)


def test_wall_upsampling_is_the_wall():
    # the channel wall y = +-h(x) is known in closed form: the upsampled nodes,
    # weights (d / PN) sqrt(1 + h'^2) and normals lie on it
    from oracle import near as onear
    walls, sy, d = synth.make_channel(96, 8)
    h, hp, _ = synth.wall_profile("sin1")
    for c, sg in ((0, 1.0), (1, -1.0)):
        s = slice(walls.curve_off[c], walls.curve_off[c + 1])
        xu, yu, nxu, nyu, wu, _, _ = onear.wall_upsample(walls.x[s], walls.y[s], walls.nx[s], walls.ny[s],
                                                         walls.fx[s], walls.fy[s], d, 8)
        sq = np.sqrt(1 + hp(xu) ** 2)
        assert np.abs(xu[::8] - walls.x[s]).max() < 1e-13
        assert np.abs(yu - sg * h(xu)).max() < 1e-13
        assert np.abs(wu - (d / xu.shape[0]) * sq).max() < 1e-14
        # both walls: n_x = -h' / sqrt(1 + h'^2) (normals point out of the fluid)
        assert np.abs(nxu + hp(xu) / sq).max() < 1e-12 and np.abs(nyu - sg / sq).max() < 1e-12


def test_wall_correction_converges_to_the_integral(oracle_lib):
    # a target 0.3 wall spacings inside the fluid above the lower wall: the
    # plain trapezoid double layer is off by more than 1e-3 of the field, the
    # 8x-upsampled one agrees with the 32x one far better
    from oracle import near as onear
    walls, sy, d = synth.make_channel(128, 8)
    n = walls.n_nodes
    th = 2 * np.pi * np.arange(n // 2) / (n // 2)
    fx = np.concatenate([np.cos(th) + 0.3 * np.sin(2 * th), 0.5 * np.cos(3 * th)])
    fy = np.concatenate([np.sin(th), np.cos(th) - 0.2 * np.sin(4 * th)])
    ws = synth.CurveSet(walls.x, walls.y, walls.nx, walls.ny, walls.w, walls.kappa, fx, fy, walls.curve_off)

    def upsampled(P):
        parts = []
        for c in range(2):
            s_ = slice(ws.curve_off[c], ws.curve_off[c + 1])
            x, y, nx, ny, w, ux, uy = onear.wall_upsample(ws.x[s_], ws.y[s_], ws.nx[s_], ws.ny[s_], ws.fx[s_],
                                                          ws.fy[s_], d, P)
            parts.append((x, y, nx, ny, w, np.zeros_like(x), ux, uy))
        return synth.concat_curves(parts)

    i = n // 2 + 40                                  # a lower-wall node (normal points down)
    tx, ty = np.array([ws.x[i]]), np.array([ws.y[i] + 0.3 * ws.w[i]])
    vals = {P: oracle_lib.dlp(upsampled(P) if P > 1 else ws, tx, ty, None, None, d, -1, 1) for P in (1, 8, 32)}
    ref = np.hypot(*vals[32])[0]
    e1 = np.hypot(vals[1][0] - vals[32][0], vals[1][1] - vals[32][1])[0] / ref
    e8 = np.hypot(vals[8][0] - vals[32][0], vals[8][1] - vals[32][1])[0] / ref
    assert e1 > 1e-3 and e8 < 1e-3 * e1, (e1, e8)


def test_wall_features_reconstruct_target_and_window():
    # from the features and the frame, the target is node K0 (unrolled over
    # the period) plus h (s t0 + n_off n0), also for targets across the
    # period boundary; the window is the wall density in the local frame
    import math
    from oracle import near as onear
    walls, sy, d = synth.make_channel(64, 4)
    w = synth.wall_densities(walls, 3)
    rng = np.random.default_rng(4)
    N = 64
    s = slice(0, N)                     # the upper wall, x from 0 to d
    h = w.w[s].sum() / N
    for px, py in ((0.01, 0.9), (d - 0.02, 0.95), (-0.05, 0.92), (d + 0.03, 0.9), (2.0, 1.1)):
        f, t0, n0, one, F = onear.wall_features_one(w.x[s], w.y[s], w.nx[s], w.ny[s], w.kappa[s], w.w[s],
                                                    w.fx[s], w.fy[s], d, px, py)
        assert one == 1.0
        # candidate K0 positions: the node whose unrolled position + offsets gives p
        ox, oy = h * (f[0] * t0[0] + f[1] * n0[0]), h * (f[0] * t0[1] + f[1] * n0[1])
        qx, qy = px - ox, py - oy
        K = np.arange(-N, 2 * N)
        X = w.x[s][K % N] + d * np.floor_divide(K, N)
        j = int(np.argmin((X - qx) ** 2 + (w.y[s][K % N] - qy) ** 2))
        assert math.hypot(X[j] - qx, w.y[s][K[j] % N] - qy) < 1e-12
        k0 = int(K[j])
        # k0 is the nearest node or its predecessor
        d2 = (X - px) ** 2 + (w.y[s][K % N] - py) ** 2
        assert k0 in (int(K[np.argmin(d2)]), int(K[np.argmin(d2)]) - 1)
        win = [(k0 + jj) % N for jj in range(-3, 5)]
        ft = (w.fx[s][win] * t0[0] + w.fy[s][win] * t0[1]) / F
        assert np.abs(f[4:12] - ft).max() < 1e-14
        assert abs(f[2] - math.log(math.sqrt(d2.min()) / h)) < 1e-12
