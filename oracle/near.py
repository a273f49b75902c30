"""FP64 numpy references for the near-field extension.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Spectral upsampling of a closed curve sampled at N equispaced parameter
  nodes (the paper represents vesicle curves in a Fourier basis, Section 1 and
  Appendix C): FFT, zero-pad to P*N modes with the Nyquist mode split evenly
  between +N/2 and -N/2, inverse FFT; the speed |x'(t)| comes from the
  spectral derivative, and the fine trapezoid weights are (2 pi / (P N)) |x'|.
* The near-field label of a target: Delta = u_P(x) - u_1(x), the single
  layer of one curve evaluated with the P-times upsampled trapezoid rule minus
  the plain N-node trapezoid rule (no images, no self term).  The paper
  notes that the trapezoid rule loses accuracy for targets near a curve
  (Section 5 footnote, and the error band of its serpentine-channel figure in
  Section 5.1).
* Spectral upsampling of one period of a periodic channel wall (the same
  trigonometric interpolation applied to the wall's periodic parts), for the
  near-wall correction of the double layer: Delta = D_P - D_1 with both sums
  over the whole wall and its images, the close evaluation the paper names as
  future work for the walls (Section 5 footnote; Section 6).
* Target features and the MLP (3 hidden layers of width 64, tanh-form GELU)
  forward and backward passes, written out plainly.
"""
from __future__ import annotations

import math

import numpy as np

N_FEAT = 20
WINDOW = (-3, 4)          # the 8 nodes k0-3 .. k0+4 around the target's interval


def upsample_periodic(v: np.ndarray, P: int) -> np.ndarray:
    """Trigonometric interpolation of the N-periodic samples v onto P*N
    equispaced nodes (N even), Nyquist mode split in half."""
    N = v.shape[0]
    if P == 1:
        return v.copy()
    M = P * N
    V = np.fft.fft(v)
    W = np.zeros(M, dtype=complex)
    h = N // 2
    W[:h] = V[:h]
    W[M - h + 1:] = V[h + 1:]
    W[h] = 0.5 * V[h]
    W[M - h] = 0.5 * V[h]
    return np.real(np.fft.ifft(W)) * P


def spectral_derivative(v: np.ndarray) -> np.ndarray:
    """d/dt of the trigonometric interpolant of N-periodic samples v on
    t_k = 2 pi k / N; the Nyquist mode (a cosine at the nodes) has zero
    derivative at the nodes."""
    N = v.shape[0]
    V = np.fft.fft(v)
    m = np.fft.fftfreq(N, d=1.0 / N)
    m[N // 2] = 0.0
    return np.real(np.fft.ifft(1j * m * V))


def upsample_curve(x, y, fx, fy, P: int):
    """Returns (xu, yu, wu, fxu, fyu) on P*N nodes."""
    xu, yu = upsample_periodic(x, P), upsample_periodic(y, P)
    fxu, fyu = upsample_periodic(fx, P), upsample_periodic(fy, P)
    dx, dy = spectral_derivative(xu), spectral_derivative(yu)
    M = xu.shape[0]
    wu = (2.0 * np.pi / M) * np.hypot(dx, dy)
    return xu, yu, wu, fxu, fyu


def slp_trap(xs, ys, ws, fxs, fys, tx, ty, mu=1.0):
    """Plain trapezoid single layer of one curve at free targets (numpy)."""
    rx = tx[:, None] - xs[None, :]
    ry = ty[:, None] - ys[None, :]
    q = rx * rx + ry * ry
    gx, gy = ws * fxs, ws * fys
    rg = (rx * gx + ry * gy) / q
    lq = np.log(q)
    u = (-0.5 * lq * gx + rx * rg).sum(1)
    v = (-0.5 * lq * gy + ry * rg).sum(1)
    return u / (4 * np.pi * mu), v / (4 * np.pi * mu)


def near_label(x, y, fx, fy, w, tx, ty, P=8, mu=1.0):
    """Delta = u_P - u_1 at targets (tx, ty) for one curve."""
    xu, yu, wu, fxu, fyu = upsample_curve(x, y, fx, fy, P)
    u1, v1 = slp_trap(x, y, w, fx, fy, tx, ty, mu)
    uP, vP = slp_trap(xu, yu, wu, fxu, fyu, tx, ty, mu)
    return uP - u1, vP - v1


# ----------------------------------------------------------------------------
# walls: spectral upsampling of one period of a periodic wall
# ----------------------------------------------------------------------------
def wall_upsample(x, y, nx, ny, fx, fy, d, P):
    """One period of a wall with N nodes equispaced in its parameter t in
    [0, 2 pi), advancing by d (or -d) in x per period: the periodic parts
    x - s d t / (2 pi) (s = +-1) and y, and the density, interpolated onto P N
    nodes (trigonometric interpolation, Nyquist mode split evenly); the speed
    |x'(t)| from spectral derivatives, weights (2 pi / (P N)) |x'|, unit
    normals perpendicular to the tangent and oriented like the given ones.
    Returns (x, y, nx, ny, w, fx, fy) on P N nodes."""
    N = x.shape[0]
    s = 1.0 if x[1] > x[0] else -1.0
    t = 2 * np.pi * np.arange(N) / N
    xp = x - s * d * t / (2 * np.pi)
    M = P * N
    tf = 2 * np.pi * np.arange(M) / M
    xu = upsample_periodic(xp, P) + s * d * tf / (2 * np.pi)
    yu = upsample_periodic(y, P)
    dx = spectral_derivative(upsample_periodic(xp, P)) + s * d / (2 * np.pi)
    dy = spectral_derivative(yu)
    sp = np.hypot(dx, dy)
    # orientation of the given normals relative to the left normal (-y', x')
    tx0 = spectral_derivative(xp)[0] + s * d / (2 * np.pi)
    ty0 = spectral_derivative(y)[0]
    o = 1.0 if (-ty0 * nx[0] + tx0 * ny[0]) > 0 else -1.0
    return (xu, yu, o * -dy / sp, o * dx / sp, (2 * np.pi / M) * sp,
            upsample_periodic(fx, P), upsample_periodic(fy, P))


# ----------------------------------------------------------------------------
# features
# ----------------------------------------------------------------------------
def features_one(x, y, nx, ny, kappa, w, fx, fy, px, py):
    """Feature vector (20) of target p relative to one curve, plus the frame
    (t0, n0), the length unit h = (sum w) / N and the density scale F.

    k* is the nearest node (smallest index on ties); k0 = k* if the target's
    tangential offset from k* is >= 0, else k* - 1, so the target lies over
    the interval [k0, k0+1).  Features: [s, n_off, dist, kappa h,
    f_t(k0-3..k0+4) / F, f_n(k0-3..k0+4) / F] with s, n_off the tangential
    and normal offsets from node k0 in units of h, dist = ln(|p - x_k*| / h),
    t0 = (-n_y, n_x) at k0 and F the largest density norm in the window (1 if
    zero)."""
    N = x.shape[0]
    h = w.sum() / N
    d2 = (px - x) ** 2 + (py - y) ** 2
    ks = int(np.argmin(d2))
    ts = np.array([-ny[ks], nx[ks]])
    if (px - x[ks]) * ts[0] + (py - y[ks]) * ts[1] >= 0.0:
        k0 = ks
    else:
        k0 = (ks - 1) % N
    t0 = np.array([-ny[k0], nx[k0]])
    n0 = np.array([nx[k0], ny[k0]])
    ox, oy = px - x[k0], py - y[k0]
    s = (ox * t0[0] + oy * t0[1]) / h
    no = (ox * n0[0] + oy * n0[1]) / h
    dist = math.log(math.sqrt(d2[ks]) / h)
    idx = [(k0 + j) % N for j in range(WINDOW[0], WINDOW[1] + 1)]
    ft = np.array([fx[j] * t0[0] + fy[j] * t0[1] for j in idx])
    fn = np.array([fx[j] * n0[0] + fy[j] * n0[1] for j in idx])
    F = max(np.hypot(ft, fn).max(), 0.0)
    if F == 0.0:
        F = 1.0
    feat = np.concatenate([[s, no, dist, kappa[k0] * h], ft / F, fn / F])
    return feat, t0, n0, h, F


def features(curve, px, py):
    out = np.zeros((len(px), N_FEAT))
    frames = np.zeros((len(px), 6))       # t0x, t0y, n0x, n0y, h, F
    for i in range(len(px)):
        f, t0, n0, h, F = features_one(curve.x, curve.y, curve.nx, curve.ny, curve.kappa, curve.w,
                                       curve.fx, curve.fy, px[i], py[i])
        out[i] = f
        frames[i] = [t0[0], t0[1], n0[0], n0[1], h, F]
    return out, frames


def label_to_frame(du, dv, frames, mu=1.0):
    """Scaled label in the local frame: (Delta . t0, Delta . n0) * 4 pi mu / (h F)."""
    sc = 4 * np.pi * mu / (frames[:, 4] * frames[:, 5])
    return np.stack([(du * frames[:, 0] + dv * frames[:, 1]) * sc,
                     (du * frames[:, 2] + dv * frames[:, 3]) * sc], 1)


def frame_to_velocity(yt, frames, mu=1.0):
    sc = frames[:, 4] * frames[:, 5] / (4 * np.pi * mu)
    du = (yt[:, 0] * frames[:, 0] + yt[:, 1] * frames[:, 2]) * sc
    dv = (yt[:, 0] * frames[:, 1] + yt[:, 1] * frames[:, 3]) * sc
    return du, dv


# ----------------------------------------------------------------------------
# walls: features of targets near a periodic wall (the learned correction of
# the walls' double layer)
# ----------------------------------------------------------------------------
def wall_features_one(x, y, nx, ny, kappa, w, fx, fy, d, px, py):
    """Feature vector (20) of target p relative to one period of a wall
    (N nodes advancing by s d in x, s = +-1 from its first two nodes), with
    the frame (t0, n0), the scale length 1 and the density scale F.  The
    wall is unrolled over three periods: node K in [-N, 2N) sits at
    (x_{K mod N} + s d floor(K / N), y_{K mod N}).  K* is the nearest
    unrolled node (smallest K on ties), K0 = K* or K* - 1 as for closed
    curves, and the window holds the densities of K0-3 .. K0+4; s, n_off
    and dist as for closed curves (units h = sum w / N), kappa of node
    K0 mod N."""
    N = x.shape[0]
    sg = 1.0 if x[1] > x[0] else -1.0
    h = w.sum() / N
    K = np.arange(-N, 2 * N)
    kk = K % N
    X = x[kk] + sg * d * np.floor_divide(K, N)
    Y = y[kk]
    d2 = (px - X) ** 2 + (py - Y) ** 2
    i = int(np.argmin(d2))
    ks = K[i]
    ts = np.array([-ny[ks % N], nx[ks % N]])
    k0 = ks if (px - X[i]) * ts[0] + (py - Y[i]) * ts[1] >= 0.0 else ks - 1
    m0 = k0 % N
    t0 = np.array([-ny[m0], nx[m0]])
    n0 = np.array([nx[m0], ny[m0]])
    ox, oy = px - (x[m0] + sg * d * (k0 // N)), py - y[m0]
    s = (ox * t0[0] + oy * t0[1]) / h
    no = (ox * n0[0] + oy * n0[1]) / h
    dist = math.log(math.sqrt(d2[i]) / h)
    idx = [(k0 + j) % N for j in range(WINDOW[0], WINDOW[1] + 1)]
    ft = np.array([fx[j] * t0[0] + fy[j] * t0[1] for j in idx])
    fn = np.array([fx[j] * n0[0] + fy[j] * n0[1] for j in idx])
    F = max(np.hypot(ft, fn).max(), 0.0)
    if F == 0.0:
        F = 1.0
    feat = np.concatenate([[s, no, dist, kappa[m0] * h], ft / F, fn / F])
    return feat, t0, n0, 1.0, F


def wall_features(walls, d, px, py, tc):
    """Features and frames (t0, n0, 1, F) of targets (px, py) relative to
    wall curve tc[i] of `walls`."""
    out = np.zeros((len(px), N_FEAT))
    frames = np.zeros((len(px), 6))
    for i in range(len(px)):
        s = slice(walls.curve_off[tc[i]], walls.curve_off[tc[i] + 1])
        f, t0, n0, h, F = wall_features_one(walls.x[s], walls.y[s], walls.nx[s], walls.ny[s], walls.kappa[s],
                                            walls.w[s], walls.fx[s], walls.fy[s], d, px[i], py[i])
        out[i] = f
        frames[i] = [t0[0], t0[1], n0[0], n0[1], h, F]
    return out, frames


# ----------------------------------------------------------------------------
# MLP: x (n, 20) -> standardise -> [64 GELU] x 3 -> 2
# ----------------------------------------------------------------------------
SQRT_2_OVER_PI = math.sqrt(2.0 / math.pi)


def gelu(z):
    """tanh form of GELU (Hendrycks and Gimpel)."""
    return 0.5 * z * (1.0 + np.tanh(SQRT_2_OVER_PI * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    u = SQRT_2_OVER_PI * (z + 0.044715 * z ** 3)
    th = np.tanh(u)
    du = SQRT_2_OVER_PI * (1.0 + 3 * 0.044715 * z ** 2)
    return 0.5 * (1.0 + th) + 0.5 * z * (1.0 - th ** 2) * du


def mlp_forward(params, X):
    """params: dict with mu_in (20), sd_in (20), W1 (20,64), b1, W2 (64,64), b2,
    W3 (64,64), b3, W4 (64,2), b4.  Returns (Y, cache)."""
    x0 = (X - params["mu_in"]) / params["sd_in"]
    z1 = x0 @ params["W1"] + params["b1"]
    h1 = gelu(z1)
    z2 = h1 @ params["W2"] + params["b2"]
    h2 = gelu(z2)
    z3 = h2 @ params["W3"] + params["b3"]
    h3 = gelu(z3)
    Y = h3 @ params["W4"] + params["b4"]
    return Y, (x0, z1, h1, z2, h2, z3, h3)


def mlp_loss_grad(params, X, T):
    """Mean squared error over the batch, L = (1 / (2 n)) sum ||Y - T||^2,
    and its gradient with respect to every weight and bias."""
    n = X.shape[0]
    Y, (x0, z1, h1, z2, h2, z3, h3) = mlp_forward(params, X)
    R = Y - T
    L = 0.5 * (R * R).sum() / n
    dY = R / n
    g = {}
    g["W4"] = h3.T @ dY
    g["b4"] = dY.sum(0)
    d3 = (dY @ params["W4"].T) * gelu_grad(z3)
    g["W3"] = h2.T @ d3
    g["b3"] = d3.sum(0)
    d2 = (d3 @ params["W3"].T) * gelu_grad(z2)
    g["W2"] = h1.T @ d2
    g["b2"] = d2.sum(0)
    d1 = (d2 @ params["W2"].T) * gelu_grad(z1)
    g["W1"] = x0.T @ d1
    g["b1"] = d1.sum(0)
    return L, g


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) of every trainable entry in place;
    state holds m, v per name and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k, gk in grads.items():
        m = state.setdefault("m_" + k, np.zeros_like(gk))
        v = state.setdefault("v_" + k, np.zeros_like(gk))
        m[...] = beta1 * m + (1 - beta1) * gk
        v[...] = beta2 * v + (1 - beta2) * gk * gk
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)


PARAM_SHAPES = [("W1", (N_FEAT, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
                ("W3", (64, 64)), ("b3", (64,)), ("W4", (64, 2)), ("b4", (2,))]


def init_params(seed=0, mu_in=None, sd_in=None):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in PARAM_SHAPES:
        if name.startswith("W"):
            p[name] = rng.normal(size=shp) * math.sqrt(2.0 / shp[0])
        else:
            p[name] = np.zeros(shp)
    p["mu_in"] = np.zeros(N_FEAT) if mu_in is None else np.asarray(mu_in, float)
    p["sd_in"] = np.ones(N_FEAT) if sd_in is None else np.asarray(sd_in, float)
    return p
