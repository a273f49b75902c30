"""GPU parity of the pressure and traction entry points (free targets) with
the FP64 oracle, element by element: single-layer pressure from the
vesicles, double-layer pressure from the walls, single-layer traction with
target normals, over image ranges and single images (the side-wall traction
data of the periodicity conditions), FP64 within 1e-12 and FP32C within 1e-6
(E = max |GPU - oracle| / max |oracle| per operator)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-6}


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1510_05616_amd as s2d
    s2d.stokes2d_init(0)
    yield


def _rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def _eval_all(mode, prob, x, y, mx, my, img, idx=None):
    """GPU (all targets) and oracle (targets idx) for the three operators."""
    import torch
    import oracle
    import paper_1510_05616_amd as s2d
    n = x.shape[0]
    tg = s2d.Targets(x, y)
    ves, wall = s2d.Curves(prob.ves), s2d.Curves(prob.wall)
    f64 = dict(dtype=torch.float64, device="cuda")
    p1, p2, t1, t2 = (torch.zeros(n, **f64) for _ in range(4))
    nx, ny = torch.as_tensor(mx, **f64), torch.as_tensor(my, **f64)
    s2d.stokes2d_slp_pressure_eval(mode, ves, tg, prob.d, img[0], img[1], p1)
    s2d.stokes2d_dlp_pressure_eval(mode, wall, tg, prob.d, img[0], img[1], prob.mu, p2)
    s2d.stokes2d_slp_traction_eval(mode, ves, tg, nx, ny, prob.d, img[0], img[1], t1, t2)
    torch.cuda.synchronize()
    g = [a.cpu().numpy() for a in (p1, p2, t1, t2)]
    if idx is None:
        idx = np.arange(n)
    g = [a[idx] for a in g]
    xs, ys = x[idx], y[idx]
    o1 = oracle.slp_pressure(prob.ves, xs, ys, prob.d, img[0], img[1])
    o2 = oracle.dlp_pressure(prob.wall, xs, ys, prob.d, img[0], img[1], prob.mu)
    o3, o4 = oracle.slp_traction(prob.ves, xs, ys, mx[idx], my[idx], prob.d, img[0], img[1])
    errs = {"slp_pressure": _rel(g[0], o1), "dlp_pressure": _rel(g[1], o2),
            "slp_traction": max(_rel(g[2], o3), _rel(g[3], o4))}
    return errs


def _normals(n, seed):
    th = np.random.default_rng(seed).uniform(0, 2 * np.pi, n)
    return np.cos(th), np.sin(th)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("img", [(-1, 1), (0, 0), (-2, 1)])
def test_config2_free_targets(mode, img):
    prob = synth.make_config(2)
    x, y = synth.fluid_points(prob, 3001, seed=5)           # not a multiple of a wave
    mx, my = _normals(x.shape[0], 6)
    errs = _eval_all(mode, prob, x, y, mx, my, img)
    print(f"mode={mode} img={img} {errs}", flush=True)
    assert max(errs.values()) <= TOL[mode], errs


@pytest.mark.parametrize("mode", [0, 1])
def test_config3_sampled(mode):
    # the 128k-node channel; 20,000 fluid points plus the 64 side-wall points,
    # the GPU on all of them, the oracle on a seeded sample
    prob = synth.make_config(3)
    fx, fy = synth.fluid_points(prob, 20000, seed=7)
    side = prob.trg.kind == 2
    x = np.concatenate([fx, prob.trg.x[side]])
    y = np.concatenate([fy, prob.trg.y[side]])
    mx, my = _normals(x.shape[0], 8)
    idx = np.concatenate([np.random.default_rng(9).choice(20000, 300, replace=False), 20000 + np.arange(64)])
    errs = _eval_all(mode, prob, x, y, mx, my, (-1, 1), idx)
    print(f"mode={mode} {errs}", flush=True)
    assert max(errs.values()) <= TOL[mode], errs


@pytest.mark.parametrize("mode", [0, 1])
def test_side_wall_traction_data(mode):
    # traction discrepancy of the periodicity conditions: the vesicles' single
    # layer shifted by -d seen at R minus shifted by +d seen at L, normal (1, 0)
    import torch
    import oracle
    import paper_1510_05616_amd as s2d
    prob = synth.make_config(3)                             # 32 + 32 side-wall points
    t = prob.trg
    side = np.where(t.kind == 2)[0]
    assert side.shape[0] == 64
    K = side.shape[0] // 2
    xl, yl = t.x[side[:K]], t.y[side[:K]]
    xr, yr = t.x[side[K:]], t.y[side[K:]]
    ones, zeros = np.ones(K), np.zeros(K)
    f64 = dict(dtype=torch.float64, device="cuda")
    ves = s2d.Curves(prob.ves)
    nx, ny = torch.as_tensor(ones, **f64), torch.as_tensor(zeros, **f64)
    gx, gy = torch.zeros(K, **f64), torch.zeros(K, **f64)
    s2d.stokes2d_slp_traction_eval(mode, ves, s2d.Targets(xr, yr), nx, ny, prob.d, -1, -1, gx, gy)
    gx.neg_()
    gy.neg_()
    s2d.stokes2d_slp_traction_eval(mode, ves, s2d.Targets(xl, yl), nx, ny, prob.d, 1, 1, gx, gy, accumulate=1)
    torch.cuda.synchronize()
    ax, ay = oracle.slp_traction(prob.ves, xr, yr, ones, zeros, prob.d, -1, -1)
    bx, by = oracle.slp_traction(prob.ves, xl, yl, ones, zeros, prob.d, 1, 1)
    ox, oy = bx - ax, by - ay
    # E of the paper's definition: max error over max |result|; these are
    # far-field sums (the copies at distance d), whose terms cancel in part
    err = np.hypot(gx.cpu().numpy() - ox, gy.cpu().numpy() - oy).max() / np.hypot(ox, oy).max()
    print(f"mode={mode} traction data E {err:.2e}", flush=True)
    assert err <= TOL[mode]


def test_accumulate_and_empty():
    import torch
    import paper_1510_05616_amd as s2d
    prob = synth.make_config(1)
    x, y = synth.fluid_points(prob, 200, seed=2)
    tg = s2d.Targets(x, y)
    ves, wall = s2d.Curves(prob.ves), s2d.Curves(prob.wall)
    f64 = dict(dtype=torch.float64, device="cuda")
    for mode in (0, 1):
        a = torch.zeros(200, **f64)
        s2d.stokes2d_dlp_pressure_eval(mode, wall, tg, prob.d, -1, 1, 0.7, a)
        b = torch.full((200,), 1.25, **f64)
        s2d.stokes2d_dlp_pressure_eval(mode, wall, tg, prob.d, -1, 1, 0.7, b, accumulate=1)
        torch.cuda.synchronize()
        assert torch.equal(b, a + 1.25)
        # no sources: zero
        e = s2d.Curves(synth.concat_curves([]))
        s2d.stokes2d_slp_pressure_eval(mode, e, tg, prob.d, -1, 1, b)
        torch.cuda.synchronize()
        assert torch.all(b == 0)
        # no targets: a no-op
        z = torch.zeros(0, **f64)
        s2d.stokes2d_slp_traction_eval(mode, ves, s2d.Targets(np.zeros(0), np.zeros(0)), z, z, prob.d, 0, 0, z, z)
