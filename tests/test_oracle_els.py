"""Pins of the oracle for the periodization system of an empty channel cell
(CPU, no GPU), against what the mathematics fixes:

  * the double-layer traction kernel equals the stress -p m + mu (grad u +
    grad u^T) m of the double-layer velocity and pressure pair (central
    differences) -- this is how the printed kernel's dipole functions were
    paired;
  * the assembled blocks act as the independently pinned pair sums of the C
    oracle (double layer with the diagonal limit and the -1/2 jump on the
    walls, Stokeslets from the proxies, the side-wall differences);
  * the solved system reproduces a Poiseuille flow (Section 5 test: alpha =
    0.2, mu = 0.7, d = 2 pi, points (0.8, 0), (3.2, 0), (4.8, 0)) to about
    1e-11, converging as N, K and M grow.
"""
import numpy as np
import pytest

import synth
from oracle import els


def test_stresslet_traction_is_the_stress_of_the_double_layer():
    mu = 0.7
    rng = np.random.default_rng(1)
    for _ in range(3):
        s = rng.normal(size=2)
        th = rng.uniform(0, 2 * np.pi)
        nu = np.array([np.cos(th), np.sin(th)])
        tau = rng.normal(size=2)
        X, Y = s[0] + rng.uniform(0.5, 1.5, 4) * rng.choice([-1, 1], 4), s[1] + rng.uniform(-1, 1, 4)
        tm = rng.uniform(0, 2 * np.pi, 4)
        M = np.stack([np.cos(tm), np.sin(tm)], 1)
        sx, sy = s[:1], s[1:]
        vel = lambda x, y: np.einsum("tsab,b->ta", els.stresslet(x, y, sx, sy, nu[:1], nu[1:]), tau)
        prs = lambda x, y: np.einsum("tsb,b->t", els.stresslet_pressure(x, y, sx, sy, nu[:1], nu[1:], mu), tau)
        h = 1e-6
        g = np.zeros((4, 2, 2))
        for j, (ex, ey) in enumerate(((h, 0), (0, h))):
            g[:, :, j] = (vel(X + ex, Y + ey) - vel(X - ex, Y - ey)) / (2 * h)
        t_fd = -prs(X, Y)[:, None] * M + mu * np.einsum("kij,kj->ki", g + g.transpose(0, 2, 1), M)
        T = els.stresslet_traction(X, Y, M[:, 0], M[:, 1], sx, sy, nu[:1], nu[1:], mu)
        t = np.einsum("tsab,b->ta", T, tau)
        assert np.abs(t - t_fd).max() < 1e-7 * np.abs(t_fd).max(), (t, t_fd)


def test_blocks_act_as_the_pair_sums(oracle_lib):
    mu = 0.9
    walls, sy, d = synth.make_channel(48, 8)
    A, B, C, Q, (px, py) = els.assemble(walls, sy, d, 24, mu)
    rng = np.random.default_rng(2)
    tau = rng.normal(size=2 * walls.n_nodes)
    c = rng.normal(size=2 * 24)
    wt = synth.CurveSet(walls.x, walls.y, walls.nx, walls.ny, walls.w, walls.kappa, tau[0::2], tau[1::2],
                        walls.curve_off)
    n = walls.n_nodes
    oc = np.repeat(np.arange(2, dtype=np.int32), n // 2)
    on = np.arange(n, dtype=np.int32)
    du, dv = oracle_lib.dlp(wt, walls.x, walls.y, oc, on, d, -1, 1)
    ref = np.stack([du, dv], 1).reshape(-1) - 0.5 * tau
    assert np.abs(A @ tau - ref).max() < 1e-13 * np.abs(ref).max()
    prox = synth.CurveSet(px, py, np.zeros(24), np.zeros(24), np.ones(24), np.zeros(24), c[0::2], c[1::2],
                          np.array([0, 24], np.int32))
    su, sv = oracle_lib.slp(prox, walls.x, walls.y, mu=mu)
    assert np.abs(B @ c - np.stack([su, sv], 1).reshape(-1)).max() < 1e-13 * np.abs(su).max()
    K = len(sy)
    xl, xr = np.zeros(K), np.full(K, d)
    ar, br = oracle_lib.dlp(wt, xr, sy, None, None, d, -1, -1)
    al, bl = oracle_lib.dlp(wt, xl, sy, None, None, d, 1, 1)
    gu = np.stack([ar - al, br - bl], 1).reshape(-1)
    assert np.abs((C @ tau)[:2 * K] - gu).max() < 1e-13 * np.abs(gu).max()
    ur, vr = oracle_lib.slp(prox, xr, sy, mu=mu)
    ul, vl = oracle_lib.slp(prox, xl, sy, mu=mu)
    qu = np.stack([ur - ul, vr - vl], 1).reshape(-1)
    assert np.abs((Q @ c)[:2 * K] - qu).max() < 1e-13 * np.abs(qu).max()
    tr = oracle_lib.slp_traction(prox, xr, sy, np.ones(K), np.zeros(K))
    tl = oracle_lib.slp_traction(prox, xl, sy, np.ones(K), np.zeros(K))
    qt = np.stack([tr[0] - tl[0], tr[1] - tl[1]], 1).reshape(-1)
    assert np.abs((Q @ c)[2 * K:] - qt).max() < 1e-13 * np.abs(qt).max()


def _poiseuille_error(Nw, K, M, alpha=0.2, mu=0.7):
    walls, sy, d = synth.make_channel(Nw, K)
    A, B, C, Q, (px, py) = els.assemble(walls, sy, d, M, mu)
    v, g = synth.poiseuille_cell_data(walls, sy, d, alpha, mu)
    tau, c = els.solve(A, B, C, Q, v, g)
    X, Y = np.array([0.8, 3.2, 4.8]), np.zeros(3)
    u, p = els.field(walls, tau, px, py, c, d, mu, X, Y)
    ue, pe = synth.poiseuille(X, Y, alpha, mu)
    eu = np.abs(u - ue).max() / (alpha * 1.3 ** 2)            # max |u_e| over the cell
    # the pressure is fixed up to a constant: compare differences
    ep = np.abs((p - p[0]) - (pe - pe[0])).max() / (2 * alpha * mu * d)
    return eu, ep


def test_poiseuille_flow_is_reproduced():
    eu, ep = _poiseuille_error(128, 32, 128)
    assert eu < 1e-10 and ep < 1e-10, (eu, ep)


def test_poiseuille_error_converges_in_the_side_and_proxy_counts():
    coarse = max(_poiseuille_error(128, 4, 16))
    mid = max(_poiseuille_error(128, 8, 32))
    fine = max(_poiseuille_error(128, 32, 128))
    assert coarse > 10 * mid > 10 * fine, (coarse, mid, fine)


def test_poiseuille_data_is_the_exact_traction_jump():
    # the traction jump of u = (a y^2, 0), p = 2 a mu x across one period is
    # -(p(R) - p(L)) n = -2 a mu d n at every height
    walls, sy, d = synth.make_channel(16, 8)
    v, g = synth.poiseuille_cell_data(walls, sy, d, 0.2, 0.7)
    K = len(sy)
    assert np.allclose(g[:2 * K], 0.0)
    assert np.allclose(g[2 * K::2], -2 * 0.2 * 0.7 * d) and np.allclose(g[2 * K + 1::2], 0.0)
