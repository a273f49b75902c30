"""Seeded synthetic inputs for the periodic-channel Stokes layer potentials.

This module only builds *inputs*: node coordinates, unit normals, trapezoid
weights, signed curvature and densities of closed vesicle curves and of the two
periodic channel walls, plus the target list.  It contains none of the layer
potential arithmetic.  Both the FP64 oracle (tests) and the GPU path consume
its arrays; neither imports the other.

Geometry follows the paper's setting (Section 2, "Dirichlet problem in a
driven periodic pipe", and Section 2.3 "Discretization"): one period of an
upper wall U and a lower wall D discretised by the periodic trapezoid rule in
the horizontal coordinate, side walls L and R carrying K Gauss-Legendre
collocation nodes in the vertical coordinate (no weights), and closed vesicle
curves discretised by the periodic trapezoid rule in an equispaced parameter.

Conventions fixed here (the paper leaves them to a figure that is not
available, so they are readings):
  * wall normals point out of the fluid (U up, D down); vesicle normals point
    out of the vesicle;
  * signed curvature kappa = -(x'' . n) / |x'|^2, positive on a convex curve
    with outward normal; with this sign the double-layer diagonal limit is
    -(kappa / 2 pi) t t^T (Section 2.3);
  * trapezoid weights: vesicles (2 pi / N) |x'(t_k)|, walls (d / N) |x'(x_j)|;
  * densities: per curve and component, sum_{k=1..K} k^-2 (a_k cos k th +
    b_k sin k th), a_k, b_k ~ N(0, 1), th the curve parameter on [0, 2 pi)
    (walls: th = 2 pi x / d); draws in the order (curve, component, k, cos
    then sin) from numpy's default_rng([seed, 1]); geometry draws use
    default_rng([seed, 0]).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "CurveSet", "Targets", "Problem", "make_config", "ellipse_axes_for",
    "reduced_area_of_ellipse", "concat_curves", "wall_profile",
]


# ----------------------------------------------------------------------------
# containers
# ----------------------------------------------------------------------------
@dataclass
class CurveSet:
    """A set of source curves, structure-of-arrays, FP64 (int32 offsets)."""
    x: np.ndarray
    y: np.ndarray
    nx: np.ndarray
    ny: np.ndarray
    w: np.ndarray
    kappa: np.ndarray
    fx: np.ndarray
    fy: np.ndarray
    curve_off: np.ndarray          # int32 [n_curves + 1]

    @property
    def n_nodes(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_curves(self) -> int:
        return int(self.curve_off.shape[0] - 1)

    def curve_sizes(self) -> np.ndarray:
        return np.diff(self.curve_off)


@dataclass
class Targets:
    """Target points; on_curve/on_node refer to a source CurveSet (or -1)."""
    x: np.ndarray
    y: np.ndarray
    ves_curve: np.ndarray          # int32, curve of the vesicle set or -1
    ves_node: np.ndarray           # int32, global node of the vesicle set or -1
    wall_curve: np.ndarray         # int32, curve of the wall set or -1
    wall_node: np.ndarray          # int32, global node of the wall set or -1
    kind: np.ndarray               # int8: 0 vesicle node, 1 wall node, 2 side node, 3 free

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class Problem:
    ves: CurveSet
    wall: CurveSet
    trg: Targets
    d: float
    mu: float
    meta: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# curve primitives
# ----------------------------------------------------------------------------
def reduced_area_of_ellipse(ratio: float) -> float:
    """nu = 4 pi A / L^2 for an ellipse with axis ratio b/a = ratio <= 1."""
    from scipy.special import ellipe
    a, b = 1.0, float(ratio)
    area = math.pi * a * b
    perim = 4.0 * a * ellipe(1.0 - b * b)
    return 4.0 * math.pi * area / perim ** 2


def ellipse_axes_for(nu: float, area: float) -> tuple[float, float]:
    """Semi-axes (a, b) of the ellipse of reduced area nu and the given area."""
    from scipy.optimize import brentq
    ratio = brentq(lambda r: reduced_area_of_ellipse(r) - nu, 1e-3, 1.0 - 1e-12,
                   xtol=1e-15, rtol=1e-15)
    a = math.sqrt(area / (math.pi * ratio))
    return a, a * ratio


def _ellipse(cx, cy, a, b, phi, n):
    t = 2.0 * np.pi * np.arange(n) / n
    c, s = math.cos(phi), math.sin(phi)
    ex, ey = a * np.cos(t), b * np.sin(t)            # body frame
    dx, dy = -a * np.sin(t), b * np.cos(t)           # x'(t)
    ddx, ddy = -a * np.cos(t), -b * np.sin(t)        # x''(t)
    rot = lambda u, v: (c * u - s * v, s * u + c * v)
    x, y = rot(ex, ey)
    x, y = x + cx, y + cy
    xp, yp = rot(dx, dy)
    xpp, ypp = rot(ddx, ddy)
    sp = np.hypot(xp, yp)
    nx, ny = yp / sp, -xp / sp                        # outward for a CCW curve
    kappa = -(xpp * nx + ypp * ny) / sp ** 2
    w = (2.0 * np.pi / n) * sp
    return x, y, nx, ny, w, kappa, t


def wall_profile(kind: str):
    """Half-height h(x) of the symmetric channel and its first two derivatives."""
    if kind == "sin1":        # y = +-(1 + 0.3 sin x)
        return (lambda x: 1.0 + 0.3 * np.sin(x),
                lambda x: 0.3 * np.cos(x),
                lambda x: -0.3 * np.sin(x))
    if kind == "flat":        # y = +-1 (the straight channel)
        return (lambda x: np.ones_like(np.asarray(x, float)),
                lambda x: np.zeros_like(np.asarray(x, float)),
                lambda x: np.zeros_like(np.asarray(x, float)))
    if kind == "sin13":       # y = +-(1.5 + 0.4 sin x + 0.2 sin 3x)
        return (lambda x: 1.5 + 0.4 * np.sin(x) + 0.2 * np.sin(3 * x),
                lambda x: 0.4 * np.cos(x) + 0.6 * np.cos(3 * x),
                lambda x: -0.4 * np.sin(x) - 1.8 * np.sin(3 * x))
    raise ValueError(kind)


def _wall(h, hp, hpp, d, n, upper: bool):
    xs = d * np.arange(n) / n
    sgn = 1.0 if upper else -1.0
    y = sgn * h(xs)
    yp = sgn * hp(xs)
    ypp = sgn * hpp(xs)
    sp = np.sqrt(1.0 + yp ** 2)
    if upper:                 # normal pointing up (out of the fluid)
        nx, ny = -yp / sp, 1.0 / sp
    else:                     # normal pointing down (out of the fluid)
        nx, ny = yp / sp, -1.0 / sp
    kappa = -(ypp * ny) / sp ** 2          # -(x'' . n) / |x'|^2 with x'' = (0, y'')
    w = (d / n) * sp
    th = 2.0 * np.pi * xs / d
    return xs, y, nx, ny, w, kappa, th


def _density(rng, th, K):
    out = []
    for _comp in range(2):
        f = np.zeros_like(th)
        for k in range(1, K + 1):
            a = rng.standard_normal()
            b = rng.standard_normal()
            f += (a * np.cos(k * th) + b * np.sin(k * th)) / (k * k)
        out.append(f)
    return out[0], out[1]


def concat_curves(parts) -> CurveSet:
    """parts: list of (x, y, nx, ny, w, kappa, fx, fy) per curve."""
    sizes = [len(p[0]) for p in parts]
    off = np.zeros(len(parts) + 1, dtype=np.int32)
    off[1:] = np.cumsum(sizes)
    cat = lambda i: (np.concatenate([p[i] for p in parts]) if parts
                     else np.zeros(0))
    return CurveSet(*(np.ascontiguousarray(cat(i), dtype=np.float64) for i in range(8)),
                    curve_off=off)


# ----------------------------------------------------------------------------
# random sequential placement of non-overlapping vesicles in the channel
# ----------------------------------------------------------------------------
def _place_vesicles(rng, n_ves, nus, area, h, d, gap, max_tries=20000):
    """Centres, axes and rotations of n_ves ellipses inside the channel
    |y| < h(x), pairwise gap >= gap (periodic in x with period d, checked on
    finely resolved outlines) and gap >= gap to both walls (checked with the
    wall's largest slope)."""
    from scipy.spatial import cKDTree
    # a point with |y| <= h(x) - gap * sqrt(1 + max h'^2) is at least `gap`
    # from both walls (the wall is a graph whose slope never exceeds max |h'|)
    xs = np.linspace(0.0, 2.0 * d, 20000)
    wall_margin = gap * math.sqrt(1.0 + float(np.max(np.abs(
        np.gradient(h(xs), xs)))) ** 2)
    placed = []          # (cx, cy, a, outline points)
    grid = {}
    cell = 1.0
    nfine = 256
    for i in range(n_ves):
        a, b = ellipse_axes_for(nus[i], area)
        for _ in range(max_tries):
            cx = rng.uniform(0.0, d)
            hl = float(h(np.array([cx]))[0])
            room = max(hl - b - gap, 1e-3)
            cy = rng.uniform(-room, room)
            phi = rng.uniform(0.0, np.pi)
            ex, ey, *_ = _ellipse(cx, cy, a, b, phi, nfine)
            pts = np.stack([ex, ey], 1)
            if np.any(np.abs(ey) > h(ex) - wall_margin):
                continue
            ok = True
            gx = int(math.floor(cx / cell))
            for gxx in range(gx - 2, gx + 3):
                for j in grid.get(gxx % max(1, int(math.ceil(d / cell))), []):
                    ox, oy, oa, otree = placed[j]
                    for sh in (-d, 0.0, d):
                        if math.hypot(cx - ox - sh, cy - oy) > a + oa + gap:
                            continue
                        dd, _ = otree.query(pts - [sh, 0.0])
                        if dd.min() < gap:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                placed.append((cx, cy, a, cKDTree(pts)))
                grid.setdefault(gx % max(1, int(math.ceil(d / cell))), []).append(len(placed) - 1)
                yield (cx, cy, a, b, phi)
                break
        else:
            raise RuntimeError(f"could not place vesicle {i} of {n_ves}")


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------
def _side_targets(h, d, K):
    xi, _ = np.polynomial.legendre.leggauss(K)
    y0, y1 = -float(h(np.array([0.0]))[0]), float(h(np.array([0.0]))[0])
    ys = y0 + (xi + 1.0) * 0.5 * (y1 - y0)
    xs = np.concatenate([np.zeros(K), np.full(K, d)])
    return xs, np.concatenate([ys, ys])


def _assemble(ves_parts, wall_parts, side_xy, d, mu, meta):
    ves = concat_curves(ves_parts)
    wall = concat_curves(wall_parts)
    nv, nw = ves.n_nodes, wall.n_nodes
    ns = 0 if side_xy is None else len(side_xy[0])
    n = nv + nw + ns
    tx = np.concatenate([ves.x, wall.x] + ([side_xy[0]] if ns else []))
    ty = np.concatenate([ves.y, wall.y] + ([side_xy[1]] if ns else []))
    vc = np.full(n, -1, np.int32)
    vn = np.full(n, -1, np.int32)
    wc = np.full(n, -1, np.int32)
    wn = np.full(n, -1, np.int32)
    vc[:nv] = np.repeat(np.arange(ves.n_curves, dtype=np.int32), ves.curve_sizes())
    vn[:nv] = np.arange(nv, dtype=np.int32)
    wc[nv:nv + nw] = np.repeat(np.arange(wall.n_curves, dtype=np.int32), wall.curve_sizes())
    wn[nv:nv + nw] = np.arange(nw, dtype=np.int32)
    kind = np.concatenate([np.zeros(nv, np.int8), np.ones(nw, np.int8),
                           np.full(ns, 2, np.int8)])
    trg = Targets(np.ascontiguousarray(tx), np.ascontiguousarray(ty), vc, vn, wc, wn, kind)
    return Problem(ves, wall, trg, float(d), float(mu), meta)


def _channel(h, hp, hpp, d, nwall, rng_dens, K):
    parts = []
    for upper in (True, False):
        xs, y, nx, ny, w, kap, th = _wall(h, hp, hpp, d, nwall, upper)
        fx, fy = _density(rng_dens, th, K)
        parts.append((xs, y, nx, ny, w, kap, fx, fy))
    return parts


def _vesicle_parts(rng_geom, rng_dens, n_ves, sizes, nus, area, h, d, K, gap=0.1):
    parts = []
    for i, (cx, cy, a, b, phi) in enumerate(
            _place_vesicles(rng_geom, n_ves, nus, area, h, d, gap)):
        x, y, nx, ny, w, kap, t = _ellipse(cx, cy, a, b, phi, int(sizes[i]))
        fx, fy = _density(rng_dens, t, K)
        parts.append((x, y, nx, ny, w, kap, fx, fy))
    return parts


def make_channel(n_wall: int, n_side: int, profile: str = "sin1", d: float = 2 * np.pi):
    """One period of an empty symmetric channel for the periodization system:
    walls U (y = h(x), normal up) and D (y = -h(x), normal down) with n_wall
    trapezoid nodes each on x in [0, d) (zero densities), and the n_side
    Gauss-Legendre heights of the side walls L (x = 0) and R (x = d).
    Returns (walls, side_y, d)."""
    h, hp, hpp = wall_profile(profile)
    walls = concat_curves([(*_wall(h, hp, hpp, d, n_wall, up)[:6], np.zeros(n_wall), np.zeros(n_wall))
                           for up in (True, False)])
    xs, ys = _side_targets(h, d, n_side)
    return walls, ys[:n_side].copy(), float(d)


def poiseuille(X, Y, alpha, mu):
    """Manufactured Stokes flow u = (alpha y^2, 0), p = 2 alpha mu x, with a
    pressure gain of 2 alpha mu d per period d (the paper's periodization
    test, Section 5, writes p = alpha mu x, which does not satisfy
    -mu Lap u + grad p = 0; the factor 2 is restored)."""
    return np.stack([alpha * np.asarray(Y) ** 2, np.zeros_like(np.asarray(Y, float))], -1), \
        2 * alpha * mu * np.asarray(X)


def poiseuille_cell_data(walls, side_y, d, alpha, mu, x_left=0.0):
    """Right-hand sides (v, g) of the periodization system for which the
    Poiseuille flow solves the cell problem: v = u_e at the wall nodes
    (interleaved x, y); g = [u_e(R) - u_e(L) at the K side heights; the
    traction difference T(R) - T(L) for the side normal (1, 0)]."""
    ue, _ = poiseuille(walls.x, walls.y, alpha, mu)
    v = ue.reshape(-1)
    K = len(side_y)
    gu = np.zeros(2 * K)                          # u_e does not depend on x

    def traction(X, Y):
        # grad u: du1/dy = 2 alpha y, all else 0; T = -p n + mu (grad u + grad u^T) n, n = (1, 0)
        _, p = poiseuille(X, Y, alpha, mu)
        return np.stack([-p, mu * 2 * alpha * np.asarray(Y)], -1)

    xl = np.full(K, x_left)
    gt = (traction(xl + d, side_y) - traction(xl, side_y)).reshape(-1)
    return v, np.concatenate([gu, gt])


def fluid_points(prob: Problem, n: int, seed: int, gap: float = 0.02):
    """n seeded free target points in one period of the channel (between the
    walls, x in [0, d)), none within `gap` of a vesicle or wall node, e.g. for
    evaluating pressures.  Returns (x, y)."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    w = prob.wall
    lo_hi = []
    for c in range(w.n_curves):
        s = slice(w.curve_off[c], w.curve_off[c + 1])
        order = np.argsort(w.x[s])
        lo_hi.append((w.x[s][order], w.y[s][order]))
    nodes = np.concatenate([np.stack([prob.ves.x, prob.ves.y], 1), np.stack([w.x, w.y], 1)])
    tree = cKDTree(nodes)
    xs, ys = [], []
    got = 0
    while got < n:
        m = 2 * (n - got) + 64
        x = rng.uniform(0.0, prob.d, m)
        walls = [np.interp(x, cx, cy, period=prob.d) for cx, cy in lo_hi]
        y0, y1 = np.minimum(*walls), np.maximum(*walls)
        y = y0 + rng.uniform(0.0, 1.0, m) * (y1 - y0)
        keep = tree.query(np.stack([x, y], 1))[0] > gap
        xs.append(x[keep])
        ys.append(y[keep])
        got += int(keep.sum())
    return np.concatenate(xs)[:n], np.concatenate(ys)[:n]


def near_wall_points(walls: CurveSet, n: int, seed: int, lo: float = 0.05, hi: float = 3.0):
    """n seeded points near the wall curves, inside the fluid: at a random
    node i, moved against its normal (normals point out of the fluid) by
    delta_i = U(lo, hi) node spacings and along the wall by U(-1/2, 1/2)
    spacings, the spacing taken as the node's weight w_i.  Returns (x, y)."""
    rng = np.random.default_rng(seed)
    i = rng.integers(0, walls.x.shape[0], n)
    a = rng.uniform(lo, hi, n) * walls.w[i]
    b = rng.uniform(-0.5, 0.5, n) * walls.w[i]
    nx, ny = walls.nx[i], walls.ny[i]
    return walls.x[i] - a * nx - b * ny, walls.y[i] - a * ny + b * nx


def near_wall_dataset(walls: CurveSet, n: int, seed: int, lo: float = 0.05, hi: float = 5.0):
    """n seeded targets near the wall curves for the learned wall correction:
    at a uniformly drawn node i, moved into the fluid by delta = h_i
    10^U(log10 lo, log10 hi) along the normal (h_i the node's weight) and by
    U(-1/2, 1/2) h_i along the wall.  Returns (x, y, wall curve of each)."""
    rng = np.random.default_rng(seed)
    i = rng.integers(0, walls.x.shape[0], n)
    a = 10.0 ** rng.uniform(math.log10(lo), math.log10(hi), n) * walls.w[i]
    b = rng.uniform(-0.5, 0.5, n) * walls.w[i]
    nx, ny = walls.nx[i], walls.ny[i]
    curve = (np.searchsorted(walls.curve_off, i, side="right") - 1).astype(np.int32)
    return walls.x[i] - a * nx - b * ny, walls.y[i] - a * ny + b * nx, curve


def wall_densities(walls: CurveSet, seed: int, modes: int = 5) -> CurveSet:
    """The wall curves with a smooth seeded density on each: a random
    trigonometric polynomial of degree `modes` in the node parameter
    t = 2 pi j / N, mode-k amplitudes standard normal / k^2."""
    rng = np.random.default_rng(seed)
    fx, fy = np.zeros(walls.n_nodes), np.zeros(walls.n_nodes)
    for c in range(walls.n_curves):
        s = slice(walls.curve_off[c], walls.curve_off[c + 1])
        n = s.stop - s.start
        t = 2 * math.pi * np.arange(n) / n
        for k in range(1, modes + 1):
            a = rng.standard_normal(4) / k ** 2
            fx[s] += a[0] * np.cos(k * t) + a[1] * np.sin(k * t)
            fy[s] += a[2] * np.cos(k * t) + a[3] * np.sin(k * t)
    return CurveSet(walls.x, walls.y, walls.nx, walls.ny, walls.w, walls.kappa, fx, fy, walls.curve_off)


AREA_C1 = math.pi * 0.3 * 0.17          # the config-1 vesicle area, 0.160221


def make_config(k: int, seed: int | None = None, **kw) -> Problem:
    """Build configuration k (1..4) of the workloads; k = 5 lives in
    make_near_dataset.  Optional keywords shrink a configuration for tests:
    n_ves, ves_nodes, wall_nodes."""
    if k == 1:
        seed = 1 if seed is None else seed
        rg, rd = np.random.default_rng([seed, 0]), np.random.default_rng([seed, 1])
        d = 2 * np.pi
        h, hp, hpp = wall_profile("sin1")
        nves = kw.get("ves_nodes", 64)
        x, y, nx, ny, w, kap, t = _ellipse(np.pi, 0.1, 0.3, 0.17, 0.0, nves)
        fx, fy = _density(rd, t, 8)
        ves = [(x, y, nx, ny, w, kap, fx, fy)]
        walls = _channel(h, hp, hpp, d, kw.get("wall_nodes", 256), rd, 8)
        return _assemble(ves, walls, None, d, 1.0, dict(config=1, seed=seed))
    if k == 2:
        seed = 2 if seed is None else seed
        rg, rd = np.random.default_rng([seed, 0]), np.random.default_rng([seed, 1])
        d = 8 * np.pi
        h, hp, hpp = wall_profile("sin1")
        n_ves = kw.get("n_ves", 50)
        nus = rg.uniform(0.65, 0.9, n_ves)
        sizes = np.full(n_ves, kw.get("ves_nodes", 128))
        ves = _vesicle_parts(rg, rd, n_ves, sizes, nus, AREA_C1, h, d, 16)
        walls = _channel(h, hp, hpp, d, kw.get("wall_nodes", 2048), rd, 16)
        return _assemble(ves, walls, None, d, 1.0, dict(config=2, seed=seed))
    if k == 3:
        seed = 3 if seed is None else seed
        rg, rd = np.random.default_rng([seed, 0]), np.random.default_rng([seed, 1])
        d = 64 * np.pi
        h, hp, hpp = wall_profile("sin13")
        n_ves = kw.get("n_ves", 1000)
        nus = rg.uniform(0.65, 0.9, n_ves)
        area = 0.2 * (3.0 * d) / 1000.0          # 20 % of the channel area / 1000
        sizes = np.full(n_ves, kw.get("ves_nodes", 96))
        ves = _vesicle_parts(rg, rd, n_ves, sizes, nus, area, h, d, 16)
        walls = _channel(h, hp, hpp, d, kw.get("wall_nodes", 16000), rd, 16)
        side = _side_targets(h, d, kw.get("side_nodes", 32))
        return _assemble(ves, walls, side, d, 1.0, dict(config=3, seed=seed))
    if k == 4:
        raise ValueError("config 4 is a batch: use make_batch()")
    raise ValueError(f"unknown config {k}")


def make_batch(n_inst: int = 256, seed: int = 4, max_ves: int = 40,
               ves_sizes=(32, 64, 128, 256), wall_range=(256, 4096)) -> list[Problem]:
    """Configuration 4: independent channel instances with uneven vesicle and
    node counts (instance b uses seed + b)."""
    out = []
    h, hp, hpp = wall_profile("sin1")
    for b in range(n_inst):
        s = seed + b
        rg, rd = np.random.default_rng([s, 0]), np.random.default_rng([s, 1])
        n_ves = int(rg.integers(1, max_ves + 1))
        sizes = rg.choice(np.asarray(ves_sizes), n_ves)
        nwall = int(rg.integers(wall_range[0], wall_range[1] + 1))
        periods = int(math.ceil(n_ves * AREA_C1 / (0.2 * 4 * math.pi)))
        d = 2 * math.pi * periods
        nus = rg.uniform(0.65, 0.9, n_ves)
        ves = _vesicle_parts(rg, rd, n_ves, sizes, nus, AREA_C1, h, d, 8)
        walls = _channel(h, hp, hpp, d, nwall, rd, 8)
        out.append(_assemble(ves, walls, None, d, 1.0, dict(config=4, seed=s)))
    return out


def make_curve(nu: float, n: int, area: float = AREA_C1, phi: float = 0.0,
               center=(0.0, 0.0), K: int = 8, seed: int = 0) -> CurveSet:
    """One ellipse of reduced area nu with a seeded K-mode density."""
    a, b = ellipse_axes_for(nu, area)
    x, y, nx, ny, w, kap, t = _ellipse(center[0], center[1], a, b, phi, n)
    fx, fy = _density(np.random.default_rng([seed, 1]), t, K)
    return concat_curves([(x, y, nx, ny, w, kap, fx, fy)])


def ellipse_curve(a: float, b: float, n: int, center=(0.0, 0.0), phi: float = 0.0,
                  fx=None, fy=None) -> CurveSet:
    """Ellipse with semi-axes a, b; density given (callable of t) or zero."""
    x, y, nx, ny, w, kap, t = _ellipse(center[0], center[1], a, b, phi, n)
    fxv = np.zeros(n) if fx is None else np.broadcast_to(fx(t), (n,)).astype(float)
    fyv = np.zeros(n) if fy is None else np.broadcast_to(fy(t), (n,)).astype(float)
    return concat_curves([(x, y, nx, ny, w, kap, fxv, fyv)])


def ellipse_param(a: float, b: float, center=(0.0, 0.0), phi: float = 0.0):
    """Closed-form parameterisation t -> (x, y) of an ellipse (for references
    that need the curve between nodes)."""
    c, s = math.cos(phi), math.sin(phi)

    def xy(t):
        ex, ey = a * np.cos(t), b * np.sin(t)
        return center[0] + c * ex - s * ey, center[1] + s * ex + c * ey
    return xy


def make_near_dataset(n_targets: int, seed: int, per_curve: int = 200, sizes=(64, 96, 128),
                      K_range=(8, 16), delta_range=(0.05, 5.0), area: float = AREA_C1):
    """Near-field workload: closed ellipses (reduced area U[0.65, 0.9], node
    count from `sizes`, K ~ U{K_range} density modes, random rotation) and
    targets x(th) + delta n(th) outside them, th ~ U[0, 2 pi) continuous,
    delta = h 10^U[log10 lo, log10 hi] with h = (sum of weights) / N.
    Returns (curves, tx, ty, trg_curve, delta_over_h)."""
    rng = np.random.default_rng([seed, 0])
    rd = np.random.default_rng([seed, 1])
    n_curves = (n_targets + per_curve - 1) // per_curve
    parts, tx, ty, tc, dh = [], [], [], [], []
    left = n_targets
    for c in range(n_curves):
        nu = rng.uniform(0.65, 0.9)
        N = int(rng.choice(np.asarray(sizes)))
        K = int(rng.integers(K_range[0], K_range[1] + 1))
        phi = rng.uniform(0.0, np.pi)
        a, b = ellipse_axes_for(nu, area)
        x, y, nx, ny, w, kap, t = _ellipse(0.0, 0.0, a, b, phi, N)
        fx, fy = _density(rd, t, K)
        parts.append((x, y, nx, ny, w, kap, fx, fy))
        m = min(per_curve, left)
        left -= m
        h = w.sum() / N
        th = rng.uniform(0.0, 2 * np.pi, m)
        lg = rng.uniform(np.log10(delta_range[0]), np.log10(delta_range[1]), m)
        cs, sn = math.cos(phi), math.sin(phi)
        ex, ey = a * np.cos(th), b * np.sin(th)
        px, py = cs * ex - sn * ey, sn * ex + cs * ey
        dx, dy = -a * np.sin(th), b * np.cos(th)
        qx, qy = cs * dx - sn * dy, sn * dx + cs * dy
        sp = np.hypot(qx, qy)
        onx, ony = qy / sp, -qx / sp
        delta = h * 10.0 ** lg
        tx.append(px + delta * onx)
        ty.append(py + delta * ony)
        tc.append(np.full(m, c, np.int32))
        dh.append(10.0 ** lg)
    return (concat_curves(parts), np.concatenate(tx), np.concatenate(ty), np.concatenate(tc),
            np.concatenate(dh))
