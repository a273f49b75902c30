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
* The learned correction's representation: the density's node derivatives,
  geometry features of the target, the closed-form correction coefficients
  of a straight line (Poisson summation), and the MLP (3 hidden layers of
  width 64, tanh-form GELU, 20 outputs contracted with the density
  derivatives) forward and backward passes, written out plainly.
"""
from __future__ import annotations

import math

import numpy as np

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
# the learned correction's representation
# ----------------------------------------------------------------------------
# Delta is linear in the density, and the trapezoid rules see the density only
# through its trigonometric interpolant; near the target's nearest node k*
# the interpolant is summarised by its derivatives there.  With the frame
# (t, n) of node k* (n turned towards the target), the local node spacing
# hl = w_k* and lengths in units of hl, the correction is written
#   Delta = (hl / 4 pi mu) sum_{p=0..4} (Cflat_p(s, b) + env(b) dC_p) d_p
# (single layer; the double layer has 1/pi in place of hl / 4 pi mu), where
# d_p are the density's derivatives at k* in per-node units, in the frame,
# Cflat_p the 2 x 2 coefficients of a straight line with equispaced nodes
# (closed form below), env(b) = exp(-2 pi b) the decay of the plain rule's
# aliasing error with the normal offset b, and dC_p the network's output
# (20 numbers) from geometry-only features.
N_FEAT = 14
N_DERIV = 5                # density derivatives p = 0..4
N_OUT = 4 * N_DERIV        # dC[p][out][in]
FRAME = 9                  # s, b, tx, ty, nfx, nfy, hl, F, sg (n_f = sg n: the normal towards the target)


def node_derivatives(f: np.ndarray, pmax: int = N_DERIV - 1) -> np.ndarray:
    """[pmax + 1, N]: (2 pi / N)^p d^p/dt^p of the trigonometric interpolant
    of the N-periodic samples f (N even, Nyquist mode split evenly, so its
    odd derivatives vanish at the nodes), evaluated at the nodes."""
    N = f.shape[0]
    F = np.fft.fft(f)
    m = np.fft.fftfreq(N, d=1.0 / N)
    out = np.zeros((pmax + 1, N))
    for p in range(pmax + 1):
        mm = m.copy()
        if p % 2 == 1:
            mm[N // 2] = 0.0
        out[p] = np.real(np.fft.ifft(F * (1j * mm) ** p)) * (2 * np.pi / N) ** p
    return out


def _polylogs(Q, kmax, L):
    """Li_0 .. Li_kmax at complex Q, |Q| < 1: Li_0 = Q / (1 - Q), Li_1 =
    -log(1 - Q), the others by their series truncated after L terms."""
    out = [Q / (1 - Q), -np.log(1 - Q)]
    acc = [np.zeros_like(Q) for _ in range(kmax - 1)]
    ql = np.ones_like(Q)
    for l in range(1, L + 1):
        ql = ql * Q
        for k in range(2, kmax + 1):
            acc[k - 2] = acc[k - 2] + ql / float(l) ** k
    return out + acc


def flat_coeffs_slp(s, b, P=8, pmax=N_DERIV - 1, L_coarse=64, L_fine=16):
    """Cflat[..., p, out, in] of the single layer (no 1/4 pi mu): the P-times
    refined trapezoid rule minus the plain one on the line y = 0 with nodes
    at the integers, density tau^p / p! (component `in`), target (s, b),
    b > 0, weight 1 per node.  By Poisson summation the error of the rule of
    spacing D for an integrand g is sum_{l != 0} g^(2 pi l / D); the Fourier
    transforms of -1/2 log q + a^2/q, a b/q and -1/2 log q + b^2/q (a = s -
    tau, q = a^2 + b^2) are e^{-i w s - b|w|} times pi/|w| - pi b,
    i pi b sgn(w) and pi/|w| + pi b; multiplying by tau^p is (i d/dw)^p, and
    the sums over l are polylogarithms of Q = exp(-2 pi (b + i s) / D)."""
    s = np.asarray(s, float)
    b = np.asarray(b, float)
    z = b + 1j * s
    C = np.zeros(s.shape + (pmax + 1, 2, 2))
    for D, L, sign in ((1.0 / P, L_fine, 1.0), (1.0, L_coarse, -1.0)):
        c = 2 * np.pi / D
        Q = np.exp(-c * z)
        Li = _polylogs(Q, pmax + 1, L)
        for p in range(pmax + 1):
            S1 = 0
            for j in range(p + 1):
                S1 = S1 + math.comb(p, j) * (-z) ** (p - j) * (-1) ** j * math.factorial(j) * c ** (-(j + 1)) * Li[j + 1]
            S1 = np.pi * S1
            S0 = (-z) ** p * Li[0]
            ip = 1j ** p
            f = 2.0 / math.factorial(p)
            C[..., p, 0, 0] += sign * f * np.real(ip * (S1 - np.pi * b * S0))
            C[..., p, 1, 1] += sign * f * np.real(ip * (S1 + np.pi * b * S0))
            e = sign * f * np.real(ip * 1j * np.pi * b * S0)
            C[..., p, 0, 1] += e
            C[..., p, 1, 0] += e
    return C


def flat_coeffs_dlp(s, b, P=8, pmax=N_DERIV - 1):
    """Cflat[..., p, out, in] of the double layer (no 1/pi) on the same line,
    source normal towards the target: the kernel b r r^T / q^2 has the
    transforms e^{-i w s - b|w|} times (pi/2)(1 - b|w|), i (pi/2) b w and
    (pi/2)(1 + b|w|) (TT, TN, NN), polynomial in w, so the sums over l are
    Li_0(Q) = Q / (1 - Q) and Li_-1(Q) = Q / (1 - Q)^2 in closed form."""
    s = np.asarray(s, float)
    b = np.asarray(b, float)
    z = b + 1j * s
    C = np.zeros(s.shape + (pmax + 1, 2, 2))
    for D, sign in ((1.0 / P, 1.0), (1.0, -1.0)):
        c = 2 * np.pi / D
        Q = np.exp(-c * z)
        L0 = Q / (1 - Q)
        Lm1 = Q / (1 - Q) ** 2
        for p in range(pmax + 1):
            # sum_l d^p/dw^p [e^{-wz} (alpha + beta w)] at w = c l
            #   = alpha (-z)^p L0 + beta ((-z)^p c Lm1 + p (-z)^(p-1) L0)
            zp = (-z) ** p
            zp1 = p * (-z) ** (p - 1) if p > 0 else 0.0
            base = zp * L0                       # alpha = 1
            lin = zp * c * Lm1 + zp1 * L0        # beta = 1
            ip = 1j ** p
            f = 2.0 / math.factorial(p)
            C[..., p, 0, 0] += sign * f * np.real(ip * (np.pi / 2) * (base - b * lin))
            C[..., p, 1, 1] += sign * f * np.real(ip * (np.pi / 2) * (base + b * lin))
            e = sign * f * np.real(ip * 1j * (np.pi / 2) * b * lin)
            C[..., p, 0, 1] += e
            C[..., p, 1, 0] += e
    return C


def _frame_features(px, py, X, Y, NX, NY, kap, hl, nbr):
    """Geometry features and frame of a target p whose nearest node is at
    (X, Y) with unit normal (NX, NY), curvature kap, spacing hl, and the
    positions nbr[j] = (x, y) of the nodes k* - 2, k* - 1, k* + 1, k* + 2.
    The tangent t points the way the node index grows (the density
    derivatives are taken along it): t = +-(-n_y, n_x), the sign from the
    nodes k* - 1 and k* + 1."""
    (xm, ym), (xp, yp) = nbr[1], nbr[2]
    st = 1.0 if (xp - xm) * -NY + (yp - ym) * NX >= 0.0 else -1.0
    tx, ty = -st * NY, st * NX
    ox, oy = px - X, py - Y
    sv = (ox * tx + oy * ty) / hl
    nv = (ox * NX + oy * NY) / hl
    sg = 1.0 if nv >= 0.0 else -1.0            # the frame's normal points towards the target
    nfx, nfy = sg * NX, sg * NY
    b = sg * nv
    feat = [sv, b, math.log(math.hypot(ox, oy) / hl), sg * kap * hl]
    for gx, gy in nbr:
        feat += [((gx - X) * tx + (gy - Y) * ty) / hl, ((gx - X) * nfx + (gy - Y) * nfy) / hl]
    Q = np.exp(-2 * np.pi * (b + 1j * sv))
    feat += [Q.real, Q.imag]
    return np.array(feat), (sv, b, tx, ty, nfx, nfy, hl), sg


def features_one(x, y, nx, ny, kappa, w, px, py):
    """Geometry features (14), frame, sign of the normal offset and the
    nearest node k* (smallest index on ties) of a target near one closed
    curve: [s, b, ln(|p - x_k*| / hl), sg kappa hl, the nodes k* +- 1, +- 2 in
    the frame (units hl), Re Q, Im Q] with s, b the tangential and (unsigned)
    normal offsets from x_k* in units of hl = w_k*, sg the sign of the normal
    offset along n_k* and Q = exp(-2 pi (b + i s))."""
    N = x.shape[0]
    d2 = (px - x) ** 2 + (py - y) ** 2
    ks = int(np.argmin(d2))
    nbr = [(x[(ks + j) % N], y[(ks + j) % N]) for j in (-2, -1, 1, 2)]
    feat, fr, sg = _frame_features(px, py, x[ks], y[ks], nx[ks], ny[ks], kappa[ks], w[ks], nbr)
    return feat, fr, sg, ks


def head_data(D, ks, fr):
    """d[p][in] in the frame (in = t, n_f) from the node-derivative table D
    ([pmax + 1, N] per component: (Dx, Dy)), and the scale F = sum |d| over
    p and both components (1 if zero; the unit of the calibrated bounds)."""
    Dx, Dy = D
    tx, ty, nfx, nfy = fr[2], fr[3], fr[4], fr[5]
    d = np.stack([Dx[:, ks] * tx + Dy[:, ks] * ty, Dx[:, ks] * nfx + Dy[:, ks] * nfy], 1)
    F = np.abs(d).sum()
    return d, (F if F > 0 else 1.0)


def features(curve, px, py):
    """Features (n, 14), frames (n, FRAME) and head data d (n, 5, 2) of targets
    near one closed curve."""
    Dx, Dy = node_derivatives(curve.fx), node_derivatives(curve.fy)
    X = np.zeros((len(px), N_FEAT))
    frames = np.zeros((len(px), FRAME))
    dd = np.zeros((len(px), N_DERIV, 2))
    for i in range(len(px)):
        f, fr, sg, ks = features_one(curve.x, curve.y, curve.nx, curve.ny, curve.kappa, curve.w, px[i], py[i])
        d, F = head_data((Dx, Dy), ks, fr)
        X[i] = f
        dd[i] = d
        frames[i] = [fr[0], fr[1], fr[2], fr[3], fr[4], fr[5], fr[6], F, sg]
    return X, frames, dd


def frame_to_velocity(yf, frames, scale):
    """(n, 2) frame components (units scale: hl / 4 pi mu per target for the
    single layer, 1 / pi for the double layer) to velocity (du, dv)."""
    du = (yf[:, 0] * frames[:, 2] + yf[:, 1] * frames[:, 4]) * scale
    dv = (yf[:, 0] * frames[:, 3] + yf[:, 1] * frames[:, 5]) * scale
    return du, dv


def velocity_to_frame(du, dv, frames, scale):
    return np.stack([(du * frames[:, 2] + dv * frames[:, 3]) / scale,
                     (du * frames[:, 4] + dv * frames[:, 5]) / scale], 1)





def flat_predict(frames, dd, op="slp", P=8):
    """sum_p Cflat_p d_p in the frame (n, 2).  The double layer's kernel is
    odd in the source normal: its coefficients take the sign sg of the normal
    offset (flat_coeffs_dlp has the source normal towards the target)."""
    if op == "slp":
        C = flat_coeffs_slp(frames[:, 0], frames[:, 1], P=P)
    else:
        C = flat_coeffs_dlp(frames[:, 0], frames[:, 1], P=P) * frames[:, 8][:, None, None, None]
    return np.einsum('npoi,npi->no', C, dd)


# ----------------------------------------------------------------------------
# walls: features of targets near a periodic wall (the learned correction of
# the walls' double layer)
# ----------------------------------------------------------------------------
def wall_features_one(x, y, nx, ny, kappa, w, d, px, py):
    """As features_one for one period of a wall (N nodes advancing by sg d
    in x, sg = +-1 from its first two nodes), unrolled over three periods:
    node K in [-N, 2N) at (x_{K mod N} + sg d floor(K / N), y_{K mod N});
    k* is the nearest unrolled node (smallest K on ties), its neighbours are
    unrolled nodes too.  Returns (features, frame, sign, K*)."""
    N = x.shape[0]
    sgd = 1.0 if x[1] > x[0] else -1.0
    K = np.arange(-N, 2 * N)
    kk = K % N
    X = x[kk] + sgd * d * np.floor_divide(K, N)
    Y = y[kk]
    d2 = (px - X) ** 2 + (py - Y) ** 2
    i = int(np.argmin(d2))
    ks = int(K[i])
    m = ks % N

    def node(Kj):
        return x[Kj % N] + sgd * d * (Kj // N), y[Kj % N]
    nbr = [node(ks + j) for j in (-2, -1, 1, 2)]
    feat, fr, sg = _frame_features(px, py, X[i], Y[i], nx[m], ny[m], kappa[m], w[m], nbr)
    return feat, fr, sg, ks


def wall_features(walls, d, px, py, tc):
    """Features, frames and head data of targets (px, py) near wall curve
    tc[i] of `walls`."""
    X = np.zeros((len(px), N_FEAT))
    frames = np.zeros((len(px), FRAME))
    dd = np.zeros((len(px), N_DERIV, 2))
    cache = {}
    for i in range(len(px)):
        c = int(tc[i])
        s = slice(walls.curve_off[c], walls.curve_off[c + 1])
        if c not in cache:
            cache[c] = (node_derivatives(walls.fx[s]), node_derivatives(walls.fy[s]))
        f, fr, sg, ks = wall_features_one(walls.x[s], walls.y[s], walls.nx[s], walls.ny[s], walls.kappa[s],
                                          walls.w[s], d, px[i], py[i])
        N = walls.curve_off[c + 1] - walls.curve_off[c]
        dv, F = head_data(cache[c], ks % N, fr)
        X[i] = f
        dd[i] = dv
        frames[i] = [fr[0], fr[1], fr[2], fr[3], fr[4], fr[5], fr[6], F, sg]
    return X, frames, dd


# ----------------------------------------------------------------------------
# MLP: x (n, 14) -> standardise -> [64 GELU] x 3 -> 20 = dC[p][out][in]
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
    """params: dict with mu_in (14), sd_in (14), W1 (14,64), b1, W2 (64,64), b2,
    W3 (64,64), b3, W4 (64,20), b4.  Returns (Y (n, 20), cache)."""
    x0 = (X - params["mu_in"]) / params["sd_in"]
    z1 = x0 @ params["W1"] + params["b1"]
    h1 = gelu(z1)
    z2 = h1 @ params["W2"] + params["b2"]
    h2 = gelu(z2)
    z3 = h2 @ params["W3"] + params["b3"]
    h3 = gelu(z3)
    Y = h3 @ params["W4"] + params["b4"]
    return Y, (x0, z1, h1, z2, h2, z3, h3)


def envelope(X):
    """exp(-2 pi b), b = X[:, 1] (the unsigned normal offset in units hl)."""
    return np.exp(-2 * np.pi * X[:, 1])


def head(Y, X, dd):
    """The network's part of the correction in the frame: env(b) sum_p dC_p d_p,
    dC = Y reshaped to [p][out][in]."""
    C = Y.reshape(-1, N_DERIV, 2, 2)
    return envelope(X)[:, None] * np.einsum('npoi,npi->no', C, dd)


def mlp_loss_grad(params, X, dd, R, wt):
    """Loss L = (1 / (2 n)) sum_i wt_i^2 |head_i - R_i|^2 (R: the frame
    residual of the flat prediction, wt: the per-sample weight) and its
    gradient with respect to every weight and bias."""
    n = X.shape[0]
    Y, (x0, z1, h1, z2, h2, z3, h3) = mlp_forward(params, X)
    E = (head(Y, X, dd) - R) * wt[:, None]
    L = 0.5 * (E * E).sum() / n
    # dL/dY[p][o][i] = wt E_o env d_p,i / n
    g_out = (wt[:, None] * E) / n                                       # (n, 2)
    env = envelope(X)
    dY = (env[:, None, None, None] * g_out[:, None, :, None] * dd[:, :, None, :]).reshape(n, N_OUT)
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
                ("W3", (64, 64)), ("b3", (64,)), ("W4", (64, N_OUT)), ("b4", (N_OUT,))]


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
