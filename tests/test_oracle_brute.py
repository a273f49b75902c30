"""Brute-force pins of the FP64 oracle at 50 significant digits.

The discrete operators the oracle evaluates are finite sums whose terms have
plain definitions.  Here each sum is evaluated term by term in mpmath with 50
digits on tiny curves (4 to 16 nodes), starting from the same FP64 input
arrays, and compared with the oracle's double-precision result:

  * single layer (Section 2.1, Eq. (S)) over the source nodes and their
    images n = -1, 0, 1 (Section 3.1, Eq. (utotrep)), own curve skipped at
    n = 0 for on-curve targets;
  * Kress's product quadrature for the own curve of an on-curve target
    (Section 3.2 cites it; weights R_m built here from their cosine series
    R_m = -(4 pi / N) sum_{p=1}^{N/2-1} cos(2 pi p m / N) / p
          - (4 pi / N^2) cos(pi m));
  * double layer (Eq. (D), summed as Eq. (Dnr)) with the Nystrom diagonal
    limit -(kappa / 2 pi) (t . tau) t w at the target's own node
    (Section 2.3).

Agreement to 1e-14 relative (max over targets of the error norm over the
max velocity norm) leaves room only for double rounding in the oracle; a
dropped image, a missed or extra exclusion, a wrong Kress weight or a
transposed diagonal fails by orders of magnitude.

The Adam update (Kingma and Ba) is pinned at t >= 2 by its closed form under
a constant gradient: both moment estimates are exactly unbiased, so every
step moves each entry by lr * g / (|g| + eps).
"""
import numpy as np
import pytest

mpmath = pytest.importorskip("mpmath")
from mpmath import mp, mpf  # noqa: E402

import synth  # noqa: E402
from synth import CurveSet  # noqa: E402

DPS = 50


def _mp(a):
    return [mpf(float(v)) for v in np.asarray(a, dtype=np.float64)]


def _kress_R(N):
    """Kress's log-quadrature weights R_m, m = 0..N-1, from the cosine series."""
    R = []
    for m in range(N):
        s = mpf(0)
        for p in range(1, N // 2):
            s += mp.cos(2 * mp.pi * p * m / N) / p
        R.append(-(4 * mp.pi / N) * s - (4 * mp.pi / (N * N)) * mp.cos(mp.pi * m))
    return R


def _slp_brute(src, tx, ty, on_curve, on_node, d, images, mu):
    x, y, nx, ny, w, fx, fy = (_mp(getattr(src, k)) for k in ("x", "y", "nx", "ny", "w", "fx", "fy"))
    off = [int(v) for v in src.curve_off]
    D, MU = mpf(float(d)), mpf(float(mu))
    out = []
    for i in range(len(tx)):
        px, py = mpf(float(tx[i])), mpf(float(ty[i]))
        c = int(on_curve[i]) if on_curve is not None else -1
        ux = uy = mpf(0)
        for n in images:
            for j in range(len(x)):
                if n == 0 and c >= 0 and off[c] <= j < off[c + 1]:
                    continue
                rx, ry = px - x[j] - n * D, py - y[j]
                q = rx * rx + ry * ry
                gx, gy = w[j] * fx[j], w[j] * fy[j]
                rg = (rx * gx + ry * gy) / q
                ux += -mp.log(q) / 2 * gx + rx * rg
                uy += -mp.log(q) / 2 * gy + ry * rg
        if c >= 0 and 0 in images:
            a, b = off[c], off[c + 1]
            N = b - a
            R = _kress_R(N)
            ii = int(on_node[i]) - a
            for k in range(N):
                sk = w[a + k] * N / (2 * mp.pi)
                phx, phy = fx[a + k] * sk, fy[a + k] * sk
                m = (ii - k) % N
                if k == ii:
                    Lt = -mp.log(w[a + ii] * N / (2 * mp.pi))
                    tvx, tvy = -ny[a + ii], nx[a + ii]
                    Txx, Txy, Tyy = tvx * tvx, tvx * tvy, tvy * tvy
                else:
                    rx, ry = x[a + ii] - x[a + k], y[a + ii] - y[a + k]
                    q = rx * rx + ry * ry
                    Lt = -mp.log(q / (4 * mp.sin(mp.pi * (ii - k) / N) ** 2)) / 2
                    Txx, Txy, Tyy = rx * rx / q, rx * ry / q, ry * ry / q
                h = 2 * mp.pi / N
                sc = -R[m] / 2 + h * Lt
                ux += sc * phx + h * (Txx * phx + Txy * phy)
                uy += sc * phy + h * (Txy * phx + Tyy * phy)
        pref = 1 / (4 * mp.pi * MU)
        out.append((ux * pref, uy * pref))
    return out


def _dlp_brute(src, tx, ty, on_curve, on_node, d, images):
    x, y, nx, ny, w, kap, fx, fy = (_mp(getattr(src, k)) for k in
                                    ("x", "y", "nx", "ny", "w", "kappa", "fx", "fy"))
    D = mpf(float(d))
    out = []
    for i in range(len(tx)):
        px, py = mpf(float(tx[i])), mpf(float(ty[i]))
        own = int(on_node[i]) if on_curve is not None and on_curve[i] >= 0 else -1
        ux = uy = mpf(0)
        for n in images:
            for j in range(len(x)):
                if n == 0 and j == own:
                    tvx, tvy = -ny[j], nx[j]
                    tt = tvx * fx[j] + tvy * fy[j]
                    c = -kap[j] * w[j] / 2            # times 1/pi below: -(kappa / 2 pi)
                    ux += c * tt * tvx
                    uy += c * tt * tvy
                    continue
                rx, ry = px - x[j] - n * D, py - y[j]
                q = rx * rx + ry * ry
                rn = rx * w[j] * nx[j] + ry * w[j] * ny[j]
                rt = rx * fx[j] + ry * fy[j]
                ux += rx * rn * rt / (q * q)
                uy += ry * rn * rt / (q * q)
        out.append((ux / mp.pi, uy / mp.pi))
    return out


def _rel(gu, gv, ref):
    ru = np.array([float(a) for a, _ in ref])
    rv = np.array([float(b) for _, b in ref])
    err = np.hypot(np.asarray(gu) - ru, np.asarray(gv) - rv).max()
    return err / np.hypot(ru, rv).max()


def _two_vesicles(N1, N2, seed):
    rng = np.random.default_rng(seed)
    parts = []
    for N, c, ab, phi in ((N1, (0.4, 0.15), (0.35, 0.2), 0.3), (N2, (1.5, -0.2), (0.3, 0.18), -0.7)):
        x, y, nx, ny, w, kap, t = synth._ellipse(c[0], c[1], ab[0], ab[1], phi, N)
        fx = rng.normal(size=N)
        fy = rng.normal(size=N)
        parts.append((x, y, nx, ny, w, kap, fx, fy))
    return synth.concat_curves(parts)


@pytest.mark.parametrize("N1,N2", [(4, 6), (8, 12), (16, 10)])
def test_slp_matches_50_digit_sum(oracle_lib, N1, N2):
    mp.dps = DPS
    ves = _two_vesicles(N1, N2, seed=N1 * 31 + N2)
    d = 2.3
    # every node (own curve by Kress) plus free points, one of them close to
    # a node of a neighbouring image
    fxp = np.array([0.9, -0.6, 1.0, 0.41 + d])
    fyp = np.array([0.6, 0.1, -0.5, 0.351])
    tx = np.r_[ves.x, fxp]
    ty = np.r_[ves.y, fyp]
    n = ves.n_nodes
    oc = np.r_[np.repeat(np.arange(2), np.diff(ves.curve_off)), -np.ones(4)].astype(np.int32)
    on = np.r_[np.arange(n), -np.ones(4)].astype(np.int32)
    for lo, hi in ((-1, 1), (0, 0), (1, 1)):
        u, v = oracle_lib.slp(ves, tx, ty, oc, on, d, lo, hi, 0.8)
        ref = _slp_brute(ves, tx, ty, oc, on, d, list(range(lo, hi + 1)), 0.8)
        assert _rel(u, v, ref) < 1e-14, (lo, hi, _rel(u, v, ref))


@pytest.mark.parametrize("N", [4, 8, 16])
def test_kress_self_term_matches_50_digit_sum(oracle_lib, N):
    """One curve, every node a target, image 0 only: the whole result is
    the Kress product quadrature."""
    mp.dps = DPS
    ves = _two_vesicles(N, 4, seed=N)
    one = CurveSet(*(getattr(ves, k)[:N] for k in ("x", "y", "nx", "ny", "w", "kappa", "fx", "fy")),
                   curve_off=np.array([0, N], np.int32))
    tx, ty = one.x.copy(), one.y.copy()
    oc = np.zeros(N, np.int32)
    on = np.arange(N, dtype=np.int32)
    u, v = oracle_lib.slp(one, tx, ty, oc, on, 0.0, 0, 0, 1.0)
    ref = _slp_brute(one, tx, ty, oc, on, 0.0, [0], 1.0)
    assert _rel(u, v, ref) < 1e-14


def test_kress_weights_match_cosine_series(oracle_lib):
    mp.dps = DPS
    for N in (4, 6, 8, 16):
        R = oracle_lib.kress_weights(N)
        Rm = [float(r) for r in _kress_R(N)]
        assert np.abs(R - Rm).max() < 1e-15 * max(1.0, np.abs(Rm).max()), N


@pytest.mark.parametrize("N", [8, 16])
def test_dlp_with_diagonal_matches_50_digit_sum(oracle_lib, N):
    mp.dps = DPS
    rng = np.random.default_rng(N)
    h, hp, hpp = synth.wall_profile("sin1")
    d = 2 * np.pi
    parts = []
    for upper in (True, False):
        x, y, nx, ny, w, kap, th = synth._wall(h, hp, hpp, d, N, upper)
        parts.append((x, y, nx, ny, w, kap, rng.normal(size=N), rng.normal(size=N)))
    walls = synth.concat_curves(parts)
    fx = np.array([0.3, 3.0, 6.0])
    fy = np.array([0.2, -0.4, 0.7])
    tx = np.r_[walls.x, fx]
    ty = np.r_[walls.y, fy]
    n = walls.n_nodes
    oc = np.r_[np.repeat(np.arange(2), N), -np.ones(3)].astype(np.int32)
    on = np.r_[np.arange(n), -np.ones(3)].astype(np.int32)
    for lo, hi in ((-1, 1), (0, 0), (-1, -1)):
        u, v = oracle_lib.dlp(walls, tx, ty, oc, on, d, lo, hi)
        ref = _dlp_brute(walls, tx, ty, oc, on, d, list(range(lo, hi + 1)))
        assert _rel(u, v, ref) < 1e-14, (lo, hi, _rel(u, v, ref))


def test_dlp_vesicle_curves_match_50_digit_sum(oracle_lib):
    """Closed curves as double-layer sources (free and on-curve targets)."""
    mp.dps = DPS
    ves = _two_vesicles(6, 8, seed=5)
    tx = np.r_[ves.x, 0.9, 1.1]
    ty = np.r_[ves.y, 0.5, -0.6]
    oc = np.r_[np.repeat(np.arange(2), np.diff(ves.curve_off)), -1, -1].astype(np.int32)
    on = np.r_[np.arange(ves.n_nodes), -1, -1].astype(np.int32)
    u, v = oracle_lib.dlp(ves, tx, ty, oc, on, 2.5, -1, 1)
    ref = _dlp_brute(ves, tx, ty, oc, on, 2.5, [-1, 0, 1])
    assert _rel(u, v, ref) < 1e-14


# ---------------------------------------------------------------------------
def test_adam_constant_gradient_closed_form():
    """Under a constant gradient g the bias-corrected moments equal g and
    g^2 exactly at every step t, so after T steps each entry has moved by
    T lr g / (|g| + eps).  A wrong bias-correction exponent (beta^1 for
    beta^t) or a missing square root moves the entries elsewhere from t = 2."""
    from oracle import near
    g = np.array([0.3, -4.0, 1e-3, 2.5e-7])
    p0 = np.array([1.0, -2.0, 0.5, 0.0])
    for beta1, beta2, lr in ((0.9, 0.999, 0.01), (0.5, 0.9, 0.003)):
        p = {"W": p0.copy()}
        st = {}
        T = 6
        for t in range(1, T + 1):
            near.adam_step(p, {"W": g.copy()}, st, lr=lr, beta1=beta1, beta2=beta2)
            want = p0 - t * lr * g / (np.abs(g) + 1e-8)
            assert np.abs(p["W"] - want).max() < 1e-13, (t, p["W"], want)
        assert st["t"] == T


def test_adam_sign_flip_moment_closed_form():
    """Gradient +g at t = 1 and -g at t = 2: m_2 = (1 - b1)(b1 - 1) g,
    v_2 = (1 - b2^2) g^2, so the bias-corrected moments are -(1 - b1)/(1 + b1) g
    and g^2: the first step moves by -lr sign(g), the second by
    +lr (1 - b1)/(1 + b1) sign(g) (eps neglected)."""
    from oracle import near
    b1, b2, lr = 0.9, 0.999, 0.01
    g = np.array([0.7, -3.0])
    p = {"W": np.zeros(2)}
    st = {}
    near.adam_step(p, {"W": g.copy()}, st, lr=lr, beta1=b1, beta2=b2)
    near.adam_step(p, {"W": -g}, st, lr=lr, beta1=b1, beta2=b2)
    want = -lr * np.sign(g) + lr * (1 - b1) / (1 + b1) * np.sign(g)
    assert np.abs(p["W"] - want).max() < 1e-9, (p["W"], want)
