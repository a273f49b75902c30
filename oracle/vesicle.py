"""FP64 numpy reference for the vesicle time step (Algorithm 1, steps 2 and
6-9): membrane forces, the semi-implicit step system with the arc-length
correction, the position update, the area correction and the
reparameterization.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): tests, the smoke check and
the benchmark's CPU baseline may call it; the product path never does.

Curves are closed, counter-clockwise, with N (even) nodes x_j = x(alpha_j)
equispaced in a parameter alpha_j = 2 pi j / N.  Conventions (both sides of
every parity test use them):
  * D_alpha is the spectral derivative of the trigonometric interpolant
    (the Nyquist mode's derivative is zero at the nodes);
  * D_s = diag(1 / |x_alpha|) D_alpha, the arc-length derivative (Section
    3.1), with |x_alpha| from D_alpha of the node coordinates; higher
    derivatives apply D_s repeatedly (x_ssss = D_s D_s D_s D_s x);
  * the trapezoid weights are w_j = (2 pi / N) |x_alpha|_j, the outward
    normal (y_alpha, -x_alpha) / |x_alpha|.
Vectors of unknowns are stacked as [u_x (all nodes); u_y; sigma].
"""
from __future__ import annotations

import math
from types import SimpleNamespace

import numpy as np

from .near import spectral_derivative


# ---------------------------------------------------------------------------
# geometry and derivatives, per curve
# ---------------------------------------------------------------------------
def _curves(off):
    return [slice(int(off[c]), int(off[c + 1])) for c in range(len(off) - 1)]


def d_alpha(v, off):
    """Spectral alpha-derivative of the per-curve periodic samples v."""
    out = np.empty_like(v, dtype=float)
    for s in _curves(off):
        out[s] = spectral_derivative(v[s])
    return out


def geometry(x, y, off):
    """Curve set with the quantities the layer potentials and D_s need:
    x, y, speed |x_alpha|, weights, unit outward normals, curve offsets."""
    xa, ya = d_alpha(x, off), d_alpha(y, off)
    sp = np.hypot(xa, ya)
    w = np.empty_like(sp)
    for s in _curves(off):
        w[s] = (2 * math.pi / (s.stop - s.start)) * sp[s]
    return SimpleNamespace(x=x, y=y, sp=sp, w=w, nx=ya / sp, ny=-xa / sp, kappa=np.zeros_like(x),
                           curve_off=np.asarray(off, np.int32))


def d_s(v, g):
    """Arc-length derivative D_s v = D_alpha v / |x_alpha| (Section 3.2)."""
    return d_alpha(v, g.curve_off) / g.sp


def forces(g, sigma, kappa_b):
    """Bending force f_b = -kappa_B x_ssss and tension force
    f_sigma = (sigma x_s)_s (Section 3.1; Algorithm 1, step 2).  Returns
    (fbx, fby, fsx, fsy)."""
    xs, ys = d_s(g.x, g), d_s(g.y, g)
    x4, y4 = g.x, g.y
    for _ in range(4):
        x4, y4 = d_s(x4, g), d_s(y4, g)
    return -kappa_b * x4, -kappa_b * y4, d_s(sigma * xs, g), d_s(sigma * ys, g)


def arc_lengths(g):
    """Perimeter of every curve, sum of its trapezoid weights."""
    return np.array([g.w[s].sum() for s in _curves(g.curve_off)])


def areas(x, y, off):
    """Enclosed area of every curve, A = integral of x y_alpha d alpha
    (Appendix B), by the trapezoid rule in alpha."""
    ya = d_alpha(y, off)
    return np.array([(2 * math.pi / (s.stop - s.start)) * np.dot(x[s], ya[s]) for s in _curves(off)])


# ---------------------------------------------------------------------------
# the step system (Eq. (tsteplinsys) with Eq. (ALC))
# ---------------------------------------------------------------------------
def slp_matrix(g, d, img_lo, img_hi, mu):
    """S^near_{gamma,gamma} as a dense (2n x 2n) matrix over all nodes of all
    curves, stacked [x components; y components]: column j is the oracle's
    single layer (Kress product quadrature on the own curve at n = 0) of the
    unit density e_j, at every node."""
    import oracle
    n = g.x.shape[0]
    oc = np.empty(n, np.int32)
    for c, s in enumerate(_curves(g.curve_off)):
        oc[s] = c
    on = np.arange(n, dtype=np.int32)
    S = np.zeros((2 * n, 2 * n))
    for comp in range(2):
        for j in range(n):
            fx, fy = np.zeros(n), np.zeros(n)
            (fx if comp == 0 else fy)[j] = 1.0
            src = SimpleNamespace(x=g.x, y=g.y, nx=g.nx, ny=g.ny, w=g.w, fx=fx, fy=fy, curve_off=g.curve_off)
            u, v = oracle.slp(src, g.x, g.y, oc, on, d, img_lo, img_hi, mu)
            S[:n, comp * n + j] = u
            S[n:, comp * n + j] = v
    return S


def near_pairs(g, d, img_lo, img_hi, band):
    """The vesicle-vesicle interactions that take close evaluation (Section
    3.2, the paragraph on suspensions): every (node i, curve c, image k) with
    c other than the node's own curve or k != 0, for which the node moved to
    (x_i - k d, y_i) lies closer than band h_c to a node of c, h_c the largest
    trapezoid weight on c.  The squared distance is formed as the sum of two
    rounded squares, and (band h_c)^2 as the square of the rounded product.
    Returns [(i, c, k)] ordered by node, then curve, then image."""
    curves = _curves(g.curve_off)
    n = g.x.shape[0]
    own = np.empty(n, np.int64)
    for c, s in enumerate(curves):
        own[s] = c
    out = []
    for i in range(n):
        for c, s in enumerate(curves):
            R = band * g.w[s].max()
            R2 = R * R
            for k in range(img_lo, img_hi + 1):
                if c == own[i] and k == 0:
                    continue
                dx = (g.x[i] - k * d) - g.x[s]
                dy = g.y[i] - g.y[s]
                if (dx * dx + dy * dy).min() < R2:
                    out.append((i, c, k))
    return out


def near_slp_matrix(g, pairs, d, P, mu):
    """The close-evaluation correction of S^near_{gamma,gamma} as a dense
    (2n x 2n) matrix: for a pair (i, c, k), rows i and n + i gain the map from
    the density on curve c to u_P - u_1 at (x_i - k d, y_i), the P-times
    upsampled quadrature of c's single layer less its trapezoid rule
    (oracle.near.near_label), column by column for unit densities."""
    from .near import near_label
    curves = _curves(g.curve_off)
    n = g.x.shape[0]
    dS = np.zeros((2 * n, 2 * n))
    for i, c, k in pairs:
        s = curves[c]
        N = s.stop - s.start
        tx, ty = np.array([g.x[i] - k * d]), np.array([g.y[i]])
        for comp in range(2):
            for j in range(N):
                f = np.zeros(N)
                f[j] = 1.0
                fx, fy = (f, np.zeros(N)) if comp == 0 else (np.zeros(N), f)
                du, dv = near_label(g.x[s], g.y[s], fx, fy, g.w[s], tx, ty, P, mu)
                dS[i, comp * n + s.start + j] += du[0]
                dS[n + i, comp * n + s.start + j] += dv[0]
    return dS


def ds_matrix(g):
    """D_s as a dense (n x n) block-diagonal matrix."""
    n = g.x.shape[0]
    D = np.zeros((n, n))
    for s in _curves(g.curve_off):
        m = s.stop - s.start
        for j in range(m):
            e = np.zeros(m)
            e[j] = 1.0
            D[s, s.start + j] = spectral_derivative(e)
    return D / g.sp[:, None]


def step_system(g, S, dt, kappa_b):
    """The matrix of Eq. (tsteplinsys): unknowns [u_x; u_y; sigma],
        rows 1-2:  u + dt kappa_B S D_s^4 u - S D_s(sigma x_s)
        row 3:     x_s . D_s u
    with D_s and x_s from the current shape."""
    n = g.x.shape[0]
    D = ds_matrix(g)
    D4 = np.linalg.matrix_power(D, 4)
    Z = np.zeros((n, n))
    xs, ys = D @ g.x, D @ g.y
    D4b = np.block([[D4, Z], [Z, D4]])
    T = np.vstack([D @ np.diag(xs), D @ np.diag(ys)])              # sigma -> (sigma x_s)_s
    top = np.hstack([np.eye(2 * n) + dt * kappa_b * S @ D4b, -S @ T])
    bot = np.hstack([np.diag(xs) @ D, np.diag(ys) @ D, Z])
    return np.vstack([top, bot])


def step_rhs(g, S, dt, kappa_b, L0, u_resp=None):
    """Right-hand side of Eq. (tsteplinsys): [-kappa_B S x_ssss + u_resp;
    (L0 - L_k) / (dt L_k) per curve] (Eq. (ALC)); L0 = None gives the plain
    constraint x_s . u_s = 0."""
    n = g.x.shape[0]
    fbx, fby, _, _ = forces(g, np.zeros(n), kappa_b)
    r = S @ np.concatenate([fbx, fby])
    if u_resp is not None:
        r = r + np.concatenate([u_resp[0], u_resp[1]])
    alc = np.zeros(n)
    if L0 is not None:
        Lk = arc_lengths(g)
        for c, s in enumerate(_curves(g.curve_off)):
            alc[s] = (L0[c] - Lk[c]) / (dt * Lk[c])
    return np.concatenate([r, alc])


# ---------------------------------------------------------------------------
# corrections
# ---------------------------------------------------------------------------
def area_correct(x, y, off, A0):
    """Appendix B: x <- x + c (y_alpha, -x_alpha) per curve, c the root
    nearest zero of
      int x y_a - c int x x_aa + c int y_a^2 - c^2 int y_a x_aa = A0."""
    xa, ya = d_alpha(x, off), d_alpha(y, off)
    xaa = d_alpha(xa, off)
    xn, yn = x.copy(), y.copy()
    cs = []
    for c_i, s in enumerate(_curves(off)):
        h = 2 * math.pi / (s.stop - s.start)
        qa = -h * np.dot(ya[s], xaa[s])
        qb = h * (np.dot(ya[s], ya[s]) - np.dot(x[s], xaa[s]))
        qc = h * np.dot(x[s], ya[s]) - A0[c_i]
        if qa == 0.0:
            c = -qc / qb
        else:
            disc = math.sqrt(qb * qb - 4 * qa * qc)
            r1, r2 = (-qb + disc) / (2 * qa), (-qb - disc) / (2 * qa)
            c = r1 if abs(r1) <= abs(r2) else r2
        xn[s] = x[s] + c * ya[s]
        yn[s] = y[s] - c * xa[s]
        cs.append(c)
    return xn, yn, np.array(cs)


def arclength_table(x, y):
    """s_j = s(2 pi j / N), j = 0..N, of one curve from the Fourier series of
    |x_alpha| integrated term by term (Appendix C); s_N = s(2 pi)."""
    N = x.shape[0]
    sp = np.hypot(spectral_derivative(x), spectral_derivative(y))
    C = np.fft.fft(sp) / N
    k = np.arange(1, N // 2)
    al = 2 * math.pi * np.arange(N + 1) / N
    # real form of sum_{k != 0} C_k / (ik) (e^{ik alpha} - 1); the Nyquist
    # term is C_{N/2} sin(N alpha / 2) / (N / 2), zero at the nodes
    s = C[0].real * al
    for kk in k:
        s = s + 2 * np.real(C[kk] / (1j * kk) * (np.exp(1j * kk * al) - 1.0))
    return s


def trig_eval(v, alpha):
    """The trigonometric interpolant of the N-periodic samples v (Nyquist
    mode split evenly) at arbitrary parameters alpha."""
    N = v.shape[0]
    V = np.fft.fft(v) / N
    h = N // 2
    out = np.full(alpha.shape, V[0].real)
    for k in range(1, h):
        out = out + 2 * np.real(V[k] * np.exp(1j * k * alpha))
    return out + V[h].real * np.cos(h * alpha)


def reparam_alpha(s):
    """Algorithm 2: parameters alpha*_k whose arc lengths are k L / N, by
    linear interpolation in the table s_0..s_N."""
    N = s.shape[0] - 1
    L = s[N]
    a = np.zeros(N)
    j = 0
    for k in range(1, N):
        t = L * k / N
        while not (s[j] <= t < s[j + 1]):
            j += 1
        a[k] = 2 * math.pi / N * (j + (t - s[j]) / (s[j + 1] - s[j]))
    return a


def reparameterize(x, y, sigma, off):
    """Appendix C: every curve's nodes moved to the parameters alpha* of
    Algorithm 2 by Fourier interpolation; the tension is interpolated the
    same way."""
    xn, yn, sn = x.copy(), y.copy(), sigma.copy()
    for s in _curves(off):
        a = reparam_alpha(arclength_table(x[s], y[s]))
        xn[s], yn[s], sn[s] = trig_eval(x[s], a), trig_eval(y[s], a), trig_eval(sigma[s], a)
    return xn, yn, sn


# ---------------------------------------------------------------------------
# one time step
# ---------------------------------------------------------------------------
def time_step(x, y, sigma, off, dt, kappa_b, mu, L0=None, A0=None, u_resp=None, d=0.0, img_lo=0, img_hi=0,
              reparam=True, near=None):
    """Steps 6-9 of Algorithm 1 for all curves: solve Eq. (tsteplinsys)
    (constraint per Eq. (ALC) when L0 is given) exactly, x <- x + dt u,
    area correction to A0 (when given), reparameterization (when asked).
    near = (P, band): S with the close-evaluation correction of the pairs
    near_pairs(.., band) (near_slp_matrix, P-times upsampled).
    Returns (x, y, sigma, u, v) with sigma = sigma^{k+1}."""
    g = geometry(x, y, off)
    S = slp_matrix(g, d, img_lo, img_hi, mu)
    if near is not None:
        S = S + near_slp_matrix(g, near_pairs(g, d, img_lo, img_hi, near[1]), d, near[0], mu)
    A = step_system(g, S, dt, kappa_b)
    b = step_rhs(g, S, dt, kappa_b, L0, u_resp)
    z = np.linalg.solve(A, b)
    n = x.shape[0]
    u, v, sig = z[:n], z[n:2 * n], z[2 * n:]
    xn, yn = x + dt * u, y + dt * v
    if A0 is not None:
        xn, yn, _ = area_correct(xn, yn, off, A0)
    if reparam:
        xn, yn, sig = reparameterize(xn, yn, sig, off)
    return xn, yn, sig, u, v


def bending_energy(x, y, off, kappa_b=1.0):
    """(kappa_B / 2) int kappa^2 ds per curve, kappa = x_s x y_ss."""
    g = geometry(x, y, off)
    xs, ys = d_s(x, g), d_s(y, g)
    xss, yss = d_s(xs, g), d_s(ys, g)
    k = xs * yss - ys * xss
    return np.array([0.5 * kappa_b * np.dot(k[s] ** 2, g.w[s]) for s in _curves(off)])


# ---------------------------------------------------------------------------
# the channel's response to the vesicles (Algorithm 1, steps 3-5)
# ---------------------------------------------------------------------------
def _vesicle_source(x, y, off, fx, fy):
    g = geometry(x, y, off)
    return SimpleNamespace(x=x, y=y, nx=g.nx, ny=g.ny, w=g.w, kappa=g.kappa, fx=fx, fy=fy,
                           curve_off=np.asarray(off, np.int32))


def channel_response(walls, side_y, d, M, mu, x, y, off, fx, fy, p_drive, x_left=0.0, radius=None, tx=None,
                     ty=None):
    """Steps 3-5 of Algorithm 1 for vesicles with force density f:
      v_U, v_D = -S^near f on the walls (Eq. (vesU)),
      g_u = -S_{gamma-d} f|_R + S_{gamma+d} f|_L,
      g_T = -T(S_{gamma-d} f, Q_{gamma-d} f)|_R + T(S_{gamma+d} f, Q_{gamma+d} f)|_L + p_drive n
    (Eq. (vesgT), n = (1, 0); p_drive is the pressure drop p(L) - p(R) per
    period), the cell system (Eq. (bsys)) for tau and c, and
    u_resp = D^near tau + sum_m c_m phi_m (Eq. (urep)) at the vesicle nodes,
    or at the points (tx, ty) when given.  Returns (u_resp (n, 2), p_resp
    (n,), tau, c, (px, py))."""
    import oracle
    from . import els
    src = _vesicle_source(x, y, off, fx, fy)
    A, B, C, Q, (px, py) = els.assemble(walls, side_y, d, M, mu, x_left, radius)
    vx, vy = oracle.slp(src, walls.x, walls.y, None, None, d, -1, 1, mu)
    v = -np.stack([vx, vy], 1).reshape(-1)
    K = len(side_y)
    xl = np.full(K, x_left)
    xr = xl + d
    ones, zeros = np.ones(K), np.zeros(K)
    rx, ry = oracle.slp(src, xr, side_y, None, None, d, -1, -1, mu)
    lx, ly = oracle.slp(src, xl, side_y, None, None, d, 1, 1, mu)
    gu = np.stack([lx - rx, ly - ry], 1).reshape(-1)
    trx, try_ = oracle.slp_traction(src, xr, side_y, ones, zeros, d, -1, -1)
    tlx, tly = oracle.slp_traction(src, xl, side_y, ones, zeros, d, 1, 1)
    gt = np.stack([tlx - trx + p_drive, tly - try_], 1).reshape(-1)
    tau, c = els.solve(A, B, C, Q, v, np.concatenate([gu, gt]))
    X = x if tx is None else tx
    Y = y if ty is None else ty
    u, p = els.field(walls, tau, px, py, c, d, mu, X, Y)
    return u, p, tau, c, (px, py)


def imposed_field(x, y, off, fx, fy, d, mu, tx, ty):
    """The vesicles' imposed flow S^near f and pressure Q^near f (images
    -1..1, Eq. (utotrep)) at free points."""
    import oracle
    src = _vesicle_source(x, y, off, fx, fy)
    u, v = oracle.slp(src, tx, ty, None, None, d, -1, 1, mu)
    p = oracle.slp_pressure(src, tx, ty, d, -1, 1)
    return np.stack([u, v], 1), p
