"""FP64 numpy reference for the periodization system of an empty channel cell.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The velocity in one unit cell is represented (Section 2.2, Eq. (urep)) as the
double layer of the wall densities tau summed over the near images |n| <= 1
(Eq. (Dnr)) plus M Stokeslets at proxy points on a circle of radius R_p
around the cell (Eq. (phi)); the pressure likewise (Eq. (prep)).  Imposing
the wall velocity data (Eqs. (BIEU), (BIED), with the -1/2 jump of the n = 0
term) and the velocity and traction matching between the side walls L and R
= L + d (Eqs. (BIEgu), (BIEgT)) gives the block system (Eq. (bsys))

    [ A  B ] [ tau ]   [ v ]
    [ C  Q ] [  c  ] = [ g ],

discretised by Nystrom (Section 2.3): the trapezoid weights w_j multiply the
kernel, the n = 0 self term is the diagonal limit -(kappa/2 pi) t t^T w, the
side walls carry K Gauss-Legendre collocation heights (no weights).  The
system is solved as in Section 4.1: S = Q - C A^-1 B,
c = S^+ (g - C A^-1 v), tau = A^-1 (v - B c), with S^+ the pseudo-inverse.

Layout: every 2-vector is stored interleaved (x, y) per node; unknowns are
[tau at the 2N wall nodes (U then D), c at the M proxies]; rows are [the 2N
wall nodes, then the K side heights for the velocity difference, then the K
side heights for the traction difference].
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# 2 x 2 kernel blocks, arrays of shape (n_targets, n_sources, 2, 2)
# ---------------------------------------------------------------------------


def _diff(tx, ty, sx, sy):
    rx = np.asarray(tx, float)[:, None] - np.asarray(sx, float)[None, :]
    ry = np.asarray(ty, float)[:, None] - np.asarray(sy, float)[None, :]
    return rx, ry, rx * rx + ry * ry


def _outer(rx, ry):
    return np.stack([np.stack([rx * rx, rx * ry], -1), np.stack([ry * rx, ry * ry], -1)], -2)


def stokeslet(tx, ty, sx, sy, mu):
    """S_ij = 1/(4 pi mu) (delta_ij log(1/r) + r_i r_j / r^2)  (Section 2.1, Eq. (S))."""
    rx, ry, q = _diff(tx, ty, sx, sy)
    eye = np.eye(2)[None, None]
    return (-0.5 * np.log(q)[..., None, None] * eye + _outer(rx, ry) / q[..., None, None]) / (4 * math.pi * mu)


def stokeslet_pressure(tx, ty, sx, sy):
    """Q_j = 1/(2 pi) r_j / r^2 (Eq. (Q)); shape (nt, ns, 2)."""
    rx, ry, q = _diff(tx, ty, sx, sy)
    return np.stack([rx, ry], -1) / q[..., None] / (2 * math.pi)


def stresslet(tx, ty, sx, sy, snx, sny):
    """D_ij = 1/pi r_i r_j (r . n_y) / r^4, n_y the source normal (Eq. (D))."""
    rx, ry, q = _diff(tx, ty, sx, sy)
    rn = rx * np.asarray(snx)[None, :] + ry * np.asarray(sny)[None, :]
    return _outer(rx, ry) * (rn / (q * q))[..., None, None] / math.pi


def stresslet_pressure(tx, ty, sx, sy, snx, sny, mu):
    """P_j = mu/pi (-n_y,j / r^2 + 2 (r . n_y) r_j / r^4) (Eq. (P)); shape (nt, ns, 2)."""
    rx, ry, q = _diff(tx, ty, sx, sy)
    nx = np.broadcast_to(np.asarray(snx)[None, :], rx.shape)
    ny = np.broadcast_to(np.asarray(sny)[None, :], rx.shape)
    rn = rx * nx + ry * ny
    return mu / math.pi * np.stack([-nx / q + 2 * rn * rx / (q * q), -ny / q + 2 * rn * ry / (q * q)], -1)


def stokeslet_traction(tx, ty, tnx, tny, sx, sy):
    """K_ik = -1/pi r_i r_k (r . n_x) / r^4, n_x the target normal (Eq. (K))."""
    rx, ry, q = _diff(tx, ty, sx, sy)
    rm = rx * np.asarray(tnx)[:, None] + ry * np.asarray(tny)[:, None]
    return -_outer(rx, ry) * (rm / (q * q))[..., None, None] / math.pi


def stresslet_traction(tx, ty, tnx, tny, sx, sy, snx, sny, mu):
    """T_ik of Eq. (T): the traction -p n_x + mu (grad u + grad u^T) n_x, at a
    target with normal n_x, of the double-layer velocity and pressure pair
    (Eqs. (D), (P)) of a source with normal n_y,
      mu/pi [ (n_y . n_x / r^2 - 8 a b) r_i r_k / r^2 + a b delta_ik
              + n_x,i n_y,k / r^2 + b r_k n_y,i / r^2 + a r_i n_x,k / r^2 ],
    a = (r . n_y) / r^2 (source), b = (r . n_x) / r^2 (target).  Differentiating
    the pair gives b with the n_y,i term and a with the n_x,k term; the
    printed Eq. (T) pairs them the other way, which does not match the stress
    of (D, P) (the two dipole functions' definitions appear swapped there)."""
    rx, ry, q = _diff(tx, ty, sx, sy)
    shp = rx.shape
    mx = np.broadcast_to(np.asarray(tnx, float)[:, None], shp)
    my = np.broadcast_to(np.asarray(tny, float)[:, None], shp)
    nx = np.broadcast_to(np.asarray(snx, float)[None, :], shp)
    ny = np.broadcast_to(np.asarray(sny, float)[None, :], shp)
    a = (rx * nx + ry * ny) / q
    b = (rx * mx + ry * my) / q
    r = np.stack([rx, ry], -1)
    m = np.stack([mx, my], -1)
    n = np.stack([nx, ny], -1)
    nm = nx * mx + ny * my
    T = ((nm / q - 8 * a * b) / q)[..., None, None] * (r[..., :, None] * r[..., None, :])
    T = T + (a * b)[..., None, None] * np.eye(2)[None, None]
    T = T + (m[..., :, None] * n[..., None, :]) / q[..., None, None]
    T = T + b[..., None, None] * (n[..., :, None] * r[..., None, :]) / q[..., None, None]
    T = T + a[..., None, None] * (r[..., :, None] * m[..., None, :]) / q[..., None, None]
    return mu / math.pi * T


def blocks_to_matrix(blk):
    """(nt, ns, 2, 2) blocks -> (2 nt, 2 ns) matrix, row 2i+a, column 2j+b."""
    nt, ns = blk.shape[:2]
    return blk.transpose(0, 2, 1, 3).reshape(2 * nt, 2 * ns)


# ---------------------------------------------------------------------------
# the system
# ---------------------------------------------------------------------------


def proxy_points(side_y, d, M, x_left=0.0, radius=None):
    """M equispaced points on the circle of radius R_p (default d, the
    paper's choice) around the cell centre ((x_L + x_R)/2, mid-height of L)."""
    R = d if radius is None else radius
    cx = x_left + 0.5 * d
    cy = 0.5 * (float(np.min(side_y)) + float(np.max(side_y)))
    th = 2 * math.pi * np.arange(M) / M
    return cx + R * np.cos(th), cy + R * np.sin(th)


def assemble(walls, side_y, d, M, mu, x_left=0.0, radius=None):
    """The four blocks A (2N x 2N), B (2N x 2M), C (4K x 2N), Q (4K x 2M) of
    Eq. (bsys) for wall curves `walls` (all wall nodes, N in total), K side
    heights side_y, period d, M proxies, viscosity mu.  Returns
    (A, B, C, Q, (px, py))."""
    x, y, nx, ny = walls.x, walls.y, walls.nx, walls.ny
    w, kap = walls.w, walls.kappa
    N = x.shape[0]
    # A: -1/2 I + D^near on the walls, Nystrom with the diagonal limit at n = 0
    A = np.zeros((N, N, 2, 2))
    for n in (-1, 0, 1):
        with np.errstate(divide="ignore", invalid="ignore"):
            blk = stresslet(x, y, x + n * d, y, nx, ny)
        if n == 0:
            tt = np.eye(2)[None] - np.stack([np.stack([nx * nx, nx * ny], -1),
                                              np.stack([ny * nx, ny * ny], -1)], -2)
            idx = np.arange(N)
            blk[idx, idx] = -(kap / (2 * math.pi))[:, None, None] * tt
        A += blk * w[None, :, None, None]
    A = blocks_to_matrix(A) - 0.5 * np.eye(2 * N)
    px, py = proxy_points(side_y, d, M, x_left, radius)
    B = blocks_to_matrix(stokeslet(x, y, px, py, mu))
    K = len(side_y)
    xl = np.full(K, x_left)
    xr = xl + d
    ones, zeros = np.ones(K), np.zeros(K)
    # C: velocity and traction differences R - L of the far wall copies
    Cu = stresslet(xr, side_y, x - d, y, nx, ny) - stresslet(xl, side_y, x + d, y, nx, ny)
    Ct = (stresslet_traction(xr, side_y, ones, zeros, x - d, y, nx, ny, mu)
          - stresslet_traction(xl, side_y, ones, zeros, x + d, y, nx, ny, mu))
    C = np.vstack([blocks_to_matrix(Cu * w[None, :, None, None]), blocks_to_matrix(Ct * w[None, :, None, None])])
    # Q: the same differences of the proxy Stokeslets
    Qu = stokeslet(xr, side_y, px, py, mu) - stokeslet(xl, side_y, px, py, mu)
    Qt = stokeslet_traction(xr, side_y, ones, zeros, px, py) - stokeslet_traction(xl, side_y, ones, zeros, px, py)
    Q = np.vstack([blocks_to_matrix(Qu), blocks_to_matrix(Qt)])
    return A, B, C, Q, (px, py)


# Singular values of S below RCOND * max are dropped in S^+.  The paper does
# not state a cut-off; S = Q - C A^-1 B carries rounding noise of about
# cond(A) eps relative, and directions below that level only amplify it.
# 1e-8 (about sqrt(eps)) gave the smallest Poiseuille error (1e-11) over
# N = 64..512 wall nodes, K = 16..48, M = 4K.
RCOND = 1e-8


def solve(A, B, C, Q, v, g, rcond=RCOND):
    """Schur-complement solve of Section 4.1; returns (tau, c)."""
    Ainv_v = np.linalg.solve(A, v)
    Ainv_B = np.linalg.solve(A, B)
    S = Q - C @ Ainv_B
    c = np.linalg.pinv(S, rcond=rcond) @ (g - C @ Ainv_v)
    tau = Ainv_v - Ainv_B @ c
    return tau, c


def field(walls, tau, px, py, c, d, mu, X, Y):
    """Velocity (u, v) and pressure p of the representation at points (X, Y):
    wall double layer over |n| <= 1 plus the proxy Stokeslets."""
    tx, ty = tau[0::2], tau[1::2]
    cx, cy = c[0::2], c[1::2]
    u = np.zeros((len(X), 2))
    p = np.zeros(len(X))
    for n in (-1, 0, 1):
        D = stresslet(X, Y, walls.x + n * d, walls.y, walls.nx, walls.ny) * walls.w[None, :, None, None]
        u += np.einsum("tsab,sb->ta", D, np.stack([tx, ty], 1))
        P = stresslet_pressure(X, Y, walls.x + n * d, walls.y, walls.nx, walls.ny, mu) * walls.w[None, :, None]
        p += np.einsum("tsb,sb->t", P, np.stack([tx, ty], 1))
    u += np.einsum("tsab,sb->ta", stokeslet(X, Y, px, py, mu), np.stack([cx, cy], 1))
    p += np.einsum("tsb,sb->t", stokeslet_pressure(X, Y, px, py), np.stack([cx, cy], 1))
    return u, p
