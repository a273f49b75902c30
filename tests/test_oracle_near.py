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


def _lattice_flat(s, b, pmax, op, P=8, T=60.0):
    """Brute force: the P-refined minus the plain trapezoid sum on the line y = 0
    (nodes at the integers), density tau^p / p!, target (s, b), summed
    directly with a smooth cutoff that vanishes well inside [-T, T] (the two
    rules agree to rounding on the smooth far part)."""
    from scipy.special import erfc

    def rule(step):
        tau = np.arange(-T, T + step / 2, step)
        win = 0.5 * erfc((np.abs(tau) - 0.5 * T) / (0.06 * T))
        a, q = s - tau, (s - tau) ** 2 + b * b
        if op == "slp":
            K = np.array([[-0.5 * np.log(q) + a * a / q, a * b / q], [a * b / q, -0.5 * np.log(q) + b * b / q]])
        else:
            K = np.array([[b * a * a / q ** 2, a * b * b / q ** 2], [a * b * b / q ** 2, b ** 3 / q ** 2]])
        return np.stack([(K * (tau ** p / math.factorial(p) * win * step)).sum(-1) for p in range(pmax + 1)], 0)
    return rule(1.0 / P) - rule(1.0)


@pytest.mark.parametrize("op", ["slp", "dlp"])
def test_flat_coefficients_match_lattice_sums(op):
    pts = [(0.0, 0.05), (0.3, 0.05), (-0.4, 0.2), (0.1, 0.5), (0.45, 1.0), (-0.5, 2.0), (0.25, 3.0)]
    for sv, bv in pts:
        ref = _lattice_flat(sv, bv, 4, op)
        fn = near.flat_coeffs_slp if op == "slp" else near.flat_coeffs_dlp
        got = fn(np.array([sv]), np.array([bv]))[0]
        scale = max(np.abs(ref).max(), 1e-300)
        assert np.abs(got - ref).max() <= 1e-8 * max(scale, 1.0), (op, sv, bv, np.abs(got - ref).max(), scale)


def test_flat_dlp_is_the_straight_wall_correction():
    """On a straight periodic wall with equispaced nodes the double-layer
    correction of the 8x refined wall (the oracle's wall upsampling and pair
    sums over images -1..1) is the flat closed form contracted with the
    density's node derivatives, up to the derivatives past p = 4 and the
    ends of the summed image range."""
    import oracle
    N, d = 128, 2 * np.pi
    xs = d * np.arange(N) / N
    h = d / N
    rng = np.random.default_rng(3)
    dens = [sum(rng.normal() * np.cos(k * xs + rng.uniform(0, 6.3)) / k ** 2 for k in range(1, 5)) for _ in range(2)]
    parts = [(xs, np.full(N, 1.0), np.zeros(N), np.ones(N), np.full(N, h), np.zeros(N), dens[0], dens[1])]
    walls = synth.concat_curves(parts)
    xu, yu, nxu, nyu, wu, fxu, fyu = near.wall_upsample(walls.x, walls.y, walls.nx, walls.ny, walls.fx, walls.fy,
                                                        d, 8)
    fine = synth.concat_curves([(xu, yu, nxu, nyu, wu, np.zeros_like(xu), fxu, fyu)])
    # targets below the wall (normal +y points away from them), several offsets and phases
    px = np.array([xs[40] + 0.3 * h, xs[41] - 0.2 * h, xs[70], xs[10] + 0.45 * h, xs[90] - 0.1 * h])
    py = 1.0 - np.array([0.05, 0.2, 0.5, 1.0, 2.0]) * h
    # 81 periods: the truncated image sum's end terms (a kernel decaying like
    # 1 / r^2, 40 periods away) fall below the tolerance
    uf, vf = oracle.dlp(fine, px, py, d=d, img_lo=-40, img_hi=40)
    uc, vc = oracle.dlp(walls, px, py, d=d, img_lo=-40, img_hi=40)
    X, frames, dd = near.wall_features(walls, d, px, py, np.zeros(len(px), np.int32))
    yf = near.flat_predict(frames, dd, op="dlp")
    du, dv = near.frame_to_velocity(yf, frames, 1.0 / np.pi)
    err = np.hypot(du - (uf - uc), dv - (vf - vc))
    assert err.max() <= 5e-9 * max(np.hypot(uf, vf).max(), 1.0), err
    assert np.hypot(uf - uc, vf - vc).max() > 1e-4          # the correction itself is not small


def test_node_derivatives_exact_on_trig_polynomials():
    N = 32
    t = 2 * np.pi * np.arange(N) / N
    f = 0.3 + np.cos(3 * t) - 2.0 * np.sin(5 * t) + 0.7 * np.cos(16 * t)
    D = near.node_derivatives(f, 4)
    h = 2 * np.pi / N
    # exact derivatives of the interpolant: the Nyquist term cos(16 t) keeps its even derivatives
    ex = [f,
          -3 * np.sin(3 * t) - 10 * np.cos(5 * t),
          -9 * np.cos(3 * t) + 50 * np.sin(5 * t) - 0.7 * 256 * np.cos(16 * t),
          27 * np.sin(3 * t) + 250 * np.cos(5 * t),
          81 * np.cos(3 * t) - 1250 * np.sin(5 * t) + 0.7 * 16 ** 4 * np.cos(16 * t)]
    for p in range(5):
        assert np.abs(D[p] - ex[p] * h ** p).max() < 1e-12 * max(1.0, np.abs(ex[p] * h ** p).max()), p


def test_features_reconstruct_target_and_frame():
    cs, tx, ty, tc, dh = synth.make_near_dataset(200, 9, per_curve=200, sizes=(96,))
    c = cs
    N = 96
    X, frames, dd = near.features(c, tx, ty)
    for i in range(200):
        px, py = tx[i], ty[i]
        d2 = (px - c.x) ** 2 + (py - c.y) ** 2
        ks = int(np.argmin(d2))
        sv, b, t0, t1, nf0, nf1, hl, F, sg = frames[i]
        assert hl == c.w[ks] and abs(t0 + c.ny[ks]) == 0.0 and abs(t1 - c.nx[ks]) == 0.0 and sg == 1.0
        assert b >= 0.0 and abs(abs(nf0) - abs(c.nx[ks])) == 0.0
        # the target is x_k* + hl (s t + b n_f)
        assert abs(c.x[ks] + hl * (sv * t0 + b * nf0) - px) < 1e-13
        assert abs(c.y[ks] + hl * (sv * t1 + b * nf1) - py) < 1e-13
        assert X[i, 0] == sv and X[i, 1] == b and abs(X[i, 2] - math.log(math.sqrt(d2[ks]) / hl)) < 1e-12
        # the neighbours come back from their frame coordinates
        for q, j in enumerate((-2, -1, 1, 2)):
            k = (ks + j) % N
            gx = c.x[ks] + hl * (X[i, 4 + 2 * q] * t0 + X[i, 5 + 2 * q] * nf0)
            gy = c.y[ks] + hl * (X[i, 4 + 2 * q] * t1 + X[i, 5 + 2 * q] * nf1)
            assert abs(gx - c.x[k]) < 1e-13 and abs(gy - c.y[k]) < 1e-13
        Q = np.exp(-2 * np.pi * (b + 1j * sv))
        assert abs(X[i, 12] - Q.real) < 1e-15 and abs(X[i, 13] - Q.imag) < 1e-15
        # d_0 is the density at k* in the frame, F the sum of |d| over p and components
        assert abs(dd[i, 0, 0] * t0 + dd[i, 0, 1] * nf0 - c.fx[ks]) < 1e-13
        assert abs(dd[i, 0, 0] * t1 + dd[i, 0, 1] * nf1 - c.fy[ks]) < 1e-13
        assert F == np.abs(dd[i]).sum()


def test_flat_prediction_captures_most_of_the_label():
    """The closed-form straight-line coefficients account for the bulk of
    the upsampled correction near a curved vesicle (the rest is what the
    network learns): within 20 % (median 5 %) where the correction is large.
    A dropped term or a wrong sign in the closed form misses by O(1)."""
    cs, tx, ty, tc, dh = synth.make_near_dataset(200, 4, per_curve=200, sizes=(64,))
    one = synth.concat_curves([(cs.x, cs.y, cs.nx, cs.ny, cs.w, cs.kappa, cs.fx, cs.fy)])
    X, frames, dd = near.features(one, tx, ty)
    du, dv = near.near_label(one.x, one.y, one.fx, one.fy, one.w, tx, ty)
    y = near.velocity_to_frame(du, dv, frames, frames[:, 6] / (4 * np.pi))
    yf = near.flat_predict(frames, dd)
    big = np.hypot(*y.T) > 0.1 * np.hypot(*y.T).max()
    assert big.sum() >= 10
    rel = np.hypot(*(y - yf).T)[big] / np.hypot(*y.T)[big]
    assert rel.max() < 0.2 and np.median(rel) < 0.05, (rel.max(), np.median(rel))


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
    nf = near.N_FEAT
    p = near.init_params(seed=4, mu_in=rng.normal(size=nf) * 0.1, sd_in=1 + rng.random(nf))
    X = rng.normal(size=(7, nf))
    X[:, 1] = rng.uniform(0.05, 1.0, 7)              # the envelope's normal offset
    dd = rng.normal(size=(7, near.N_DERIV, 2))
    R = rng.normal(size=(7, 2))
    wt = rng.uniform(0.5, 2.0, 7)
    L, g = near.mlp_loss_grad(p, X, dd, R, wt)
    eps = 1e-6
    for name in ("W1", "b1", "W2", "b3", "W4", "b4"):
        flat = p[name].reshape(-1)
        for j in rng.choice(flat.size, min(6, flat.size), replace=False):
            old = flat[j]
            flat[j] = old + eps
            Lp, _ = near.mlp_loss_grad(p, X, dd, R, wt)
            flat[j] = old - eps
            Lm, _ = near.mlp_loss_grad(p, X, dd, R, wt)
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


def test_wall_features_reconstruct_target_across_periods():
    walls, sy, d = synth.make_channel(64, 8)
    for c in (0, 1):
        s = slice(walls.curve_off[c], walls.curve_off[c + 1])
        x, y, nx, ny = walls.x[s], walls.y[s], walls.nx[s], walls.ny[s]
        for k in (0, 1, 31, 62, 63):        # 0, 63: next to the period boundary
            for off in (-0.4, 0.3):
                # a point in the fluid half a spacing from the wall beside node k
                h = walls.w[s][k]
                px = x[k] + off * h * (-ny[k]) - 0.5 * h * nx[k]
                py = y[k] + off * h * nx[k] - 0.5 * h * ny[k]
                X, frames, dd = near.wall_features(walls, d, np.array([px]), np.array([py]), np.array([c]))
                sv, b, t0, t1, nf0, nf1, hl, F, sg = frames[0]
                # the frame's tangent follows the node order: (-n_y, n_x) or its opposite
                orient = t0 * -ny[k] + t1 * nx[k]
                assert abs(abs(orient) - 1.0) < 1e-14
                assert b > 0 and abs(b - 0.5) < 1e-9 and abs(sv - orient * off) < 1e-9
                assert nf0 * nx[k] + nf1 * ny[k] < 0 and sg == -1.0      # the frame normal points into the fluid
                assert np.abs(X[0, 4:12:2] - [-2, -1, 1, 2]).max() < 0.05   # neighbours along the tangent
