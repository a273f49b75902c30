"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element
by element on the same seeded inputs.

Tolerances (relative error E of Section 5, per target class and per part):
FP64 mode 1e-12, FP32C mode 1e-6.  Full-size (config 3, 128,064 targets x
128,000 sources x 3 images) runs the GPU on every target in the same launch
configuration the benchmark times, and checks a seeded sample of targets that
the oracle computes one by one.
"""
import numpy as np
import pytest

import synth
from _common import class_errors, gpu_eval, oracle_eval, rel_err, sample_targets

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-6}
MODES = [0, 1]


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1510_05616_amd as s2d
    s2d.stokes2d_init(0)
    yield


def _check(prob, mode, idx=None, img=(-1, 1), tol=None):
    tol = TOL[mode] if tol is None else tol
    g = gpu_eval(prob, mode, *img, idx=idx)
    o = oracle_eval(prob, *img, idx=idx)
    kind = prob.trg.kind if idx is None else prob.trg.kind[idx]
    errs = {}
    for part, (gu, gv, ou, ov) in (("slp", (g[0], g[1], o[0], o[1])), ("dlp", (g[2], g[3], o[2], o[3]))):
        for cls, e in class_errors(kind, gu, gv, ou, ov).items():
            errs[f"{part}/{cls}"] = e
    tot = class_errors(kind, g[0] + g[2], g[1] + g[3], o[0] + o[2], o[1] + o[3])
    for cls, e in tot.items():
        errs[f"total/{cls}"] = e
    worst = max(errs.values())
    print(f"mode={mode} worst E={worst:.3e} {errs}", flush=True)
    assert worst <= tol, errs
    return errs


@pytest.mark.parametrize("mode", MODES)
def test_config1_parity(mode):
    _check(synth.make_config(1), mode)


@pytest.mark.parametrize("mode", MODES)
def test_config2_parity(mode):
    _check(synth.make_config(2), mode)


@pytest.fixture(scope="module")
def cfg3():
    return synth.make_config(3)


@pytest.mark.parametrize("mode", MODES)
def test_config3_full_size_sampled(cfg3, mode):
    idx = sample_targets(cfg3, per_class=256, seed=5)
    _check(cfg3, mode, idx=idx)


@pytest.mark.parametrize("img", [(0, 0), (1, 1), (-1, -1), (-2, 2), (-3, 0)])
@pytest.mark.parametrize("mode", MODES)
def test_image_ranges(mode, img):
    _check(synth.make_config(1), mode, img=img)


@pytest.mark.parametrize("mode", MODES)
def test_ragged_sizes(mode):
    # sizes that are not multiples of the wave (64), the target tile or the
    # source superblock (256); odd wall node count
    prob = synth.make_config(2, n_ves=7, ves_nodes=38, wall_nodes=1001)
    _check(prob, mode)


def _translated(prob, dx, dy):
    import dataclasses
    move = lambda cs: dataclasses.replace(cs, x=cs.x + dx, y=cs.y + dy)
    trg = dataclasses.replace(prob.trg, x=prob.trg.x + dx, y=prob.trg.y + dy)
    return dataclasses.replace(prob, ves=move(prob.ves), wall=move(prob.wall), trg=trg)


@pytest.mark.parametrize("mode", MODES)
def test_translated_channel(mode):
    """The whole channel moved far from the origin. FP32C forms differences
    against FP64 origins per tile, so its error must not grow with the
    coordinates' magnitude; both sides see the same translated inputs."""
    _check(_translated(synth.make_config(2), 3.0e3, -7.0e2), mode)


@pytest.mark.parametrize("mode", MODES)
def test_near_touching_vesicles(mode):
    """Vesicle 1 moved towards vesicle 0 until their nearest nodes are a fifth
    of a node spacing apart (the near sub-blocks of FP32C, r formed in FP64)."""
    import dataclasses
    prob = synth.make_config(2)
    v, off = prob.ves, prob.ves.curve_off
    s0, s1 = slice(off[0], off[1]), slice(off[1], off[2])
    x0, y0, x1, y1 = v.x[s0], v.y[s0], v.x[s1], v.y[s1]
    h = np.sum(v.w[s0]) / (off[1] - off[0])
    ux, uy = x0.mean() - x1.mean(), y0.mean() - y1.mean()
    gap = lambda a: np.sqrt(((x0[:, None] - (x1[None, :] + a * ux)) ** 2 +
                             (y0[:, None] - (y1[None, :] + a * uy)) ** 2).min())
    # the first approach to 0.2 h along the line of centres: scan, then bisect
    steps = np.linspace(0.0, 1.0, 401)
    k = int(np.argmax([gap(a) < 0.2 * h for a in steps]))
    assert k > 0
    lo, hi = steps[k - 1], steps[k]
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if gap(mid) > 0.2 * h else (lo, mid)
    sx, sy = lo * ux, lo * uy
    x, y = v.x.copy(), v.y.copy()
    x[s1] += sx
    y[s1] += sy
    tx, ty = prob.trg.x.copy(), prob.trg.y.copy()
    on1 = prob.trg.ves_curve == 1
    tx[on1] += sx
    ty[on1] += sy
    prob = dataclasses.replace(prob, ves=dataclasses.replace(v, x=x, y=y),
                               trg=dataclasses.replace(prob.trg, x=tx, y=ty))
    print(f"nearest node gap {gap(lo) / h:.3f} h", flush=True)
    _check(prob, mode)


def test_single_node_sources_and_free_targets():
    import torch
    import oracle
    import paper_1510_05616_amd as s2d
    rng = np.random.default_rng(9)
    src = synth.concat_curves([(rng.normal(size=1), rng.normal(size=1), np.ones(1), np.zeros(1),
                                np.ones(1), np.zeros(1), rng.normal(size=1), rng.normal(size=1))
                               for _ in range(3)])
    tx, ty = rng.normal(size=5) + 5.0, rng.normal(size=5)
    c, tg = s2d.Curves(src), s2d.Targets(tx, ty)
    for mode in MODES:
        u = torch.zeros(5, dtype=torch.float64, device="cuda")
        v = torch.zeros_like(u)
        s2d.stokes2d_slp_eval(mode, c, tg, 3.0, -1, 1, 0.7, u, v)
        ou, ov = oracle.slp(src, tx, ty, d=3.0, img_lo=-1, img_hi=1, mu=0.7)
        assert rel_err(u.cpu().numpy(), v.cpu().numpy(), ou, ov) < TOL[mode]
        s2d.stokes2d_dlp_eval(mode, c, tg, 3.0, -1, 1, u, v)
        ou, ov = oracle.dlp(src, tx, ty, d=3.0, img_lo=-1, img_hi=1)
        assert rel_err(u.cpu().numpy(), v.cpu().numpy(), ou, ov) < TOL[mode]


def test_empty_inputs_and_accumulate():
    import torch
    import paper_1510_05616_amd as s2d
    prob = synth.make_config(1)
    t = prob.trg
    ves = s2d.Curves(prob.ves)
    tv = s2d.Targets(t.x, t.y, t.ves_curve, t.ves_node)
    # no targets: a no-op
    e = s2d.Targets(np.zeros(0), np.zeros(0))
    z = torch.zeros(0, dtype=torch.float64, device="cuda")
    s2d.stokes2d_slp_eval(0, ves, e, prob.d, -1, 1, 1.0, z, z)
    # no sources: zero output; with accumulate the outputs are unchanged
    empty = synth.concat_curves([])
    ec = s2d.Curves(empty)
    tf = s2d.Targets(t.x, t.y)
    u = torch.full((t.n,), 3.5, dtype=torch.float64, device="cuda")
    v = torch.full((t.n,), -1.5, dtype=torch.float64, device="cuda")
    s2d.stokes2d_slp_eval(0, ec, tf, prob.d, -1, 1, 1.0, u, v, accumulate=1)
    torch.cuda.synchronize()
    assert torch.all(u == 3.5) and torch.all(v == -1.5)
    s2d.stokes2d_dlp_eval(1, ec, tf, prob.d, -1, 1, u, v)
    torch.cuda.synchronize()
    assert torch.all(u == 0) and torch.all(v == 0)
    # accumulate adds exactly the non-accumulated result
    for mode in MODES:
        a = torch.zeros(t.n, dtype=torch.float64, device="cuda")
        b = torch.zeros_like(a)
        s2d.stokes2d_slp_eval(mode, ves, tv, prob.d, -1, 1, 1.0, a, b)
        u = torch.full((t.n,), 0.25, dtype=torch.float64, device="cuda")
        v = torch.full((t.n,), -0.5, dtype=torch.float64, device="cuda")
        s2d.stokes2d_slp_eval(mode, ves, tv, prob.d, -1, 1, 1.0, u, v, accumulate=1)
        torch.cuda.synchronize()
        assert torch.equal(u, a + 0.25) and torch.equal(v, b - 0.5)


def test_inconsistent_on_curve_entries_give_nan():
    import torch
    import paper_1510_05616_amd as s2d
    prob = synth.make_config(1)
    t = prob.trg
    vc, vn = t.ves_curve.copy(), t.ves_node.copy()
    vn[3] = vn[3] + 200                 # node outside its curve
    vc[5] = 7                           # curve that does not exist
    wc, wn = t.wall_curve.copy(), t.wall_node.copy()
    j = int(np.where(wc >= 0)[0][0])
    wn[j] = -5
    ves, wall = s2d.Curves(prob.ves), s2d.Curves(prob.wall)
    for mode in MODES:
        u = torch.zeros(t.n, dtype=torch.float64, device="cuda")
        v = torch.zeros_like(u)
        s2d.stokes2d_slp_eval(mode, ves, s2d.Targets(t.x, t.y, vc, vn), prob.d, -1, 1, 1.0, u, v)
        un = u.cpu().numpy()
        assert np.isnan(un[3]) and np.isnan(un[5])
        assert np.isfinite(np.delete(un, [3, 5])).all()
        s2d.stokes2d_dlp_eval(mode, wall, s2d.Targets(t.x, t.y, wc, wn), prob.d, -1, 1, u, v)
        un = u.cpu().numpy()
        assert np.isnan(un[j]) and np.isfinite(np.delete(un, [j])).all()


def test_odd_curve_with_self_target_gives_nan():
    import torch
    import paper_1510_05616_amd as s2d
    c = synth.ellipse_curve(0.3, 0.2, 33, fx=np.cos, fy=np.sin)
    oc = np.zeros(33, np.int32)
    on = np.arange(33, dtype=np.int32)
    u = torch.zeros(33, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(u)
    s2d.stokes2d_slp_eval(0, s2d.Curves(c), s2d.Targets(c.x, c.y, oc, on), 0.0, 0, 0, 1.0, u, v)
    assert torch.isnan(u).all()


@pytest.mark.parametrize("mode", MODES)
def test_bitwise_deterministic(mode):
    prob = synth.make_config(2)
    a = gpu_eval(prob, mode)
    b = gpu_eval(prob, mode)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_workspace_errors():
    import torch
    import paper_1510_05616_amd as s2d
    prob = synth.make_config(1)
    t = prob.trg
    ves = s2d.Curves(prob.ves)
    tv = s2d.Targets(t.x, t.y, t.ves_curve, t.ves_node)
    u = torch.zeros(t.n, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(u)
    need = s2d.stokes2d_workspace_size(0, 0, ves, tv)
    small = torch.empty(need // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(s2d.S2DError) as ei:
        s2d.stokes2d_slp_eval(0, ves, tv, prob.d, -1, 1, 1.0, u, v, ws=small)
    assert ei.value.code == s2d.S2D_EWORKSPACE
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(s2d.S2DError) as ei:   # misaligned pointer
        s2d.stokes2d_slp_eval(0, ves, tv, prob.d, -1, 1, 1.0, u, v, ws=big[8:])
    assert ei.value.code == s2d.S2D_EWORKSPACE


@pytest.mark.parametrize("mode", MODES)
def test_side_targets_few_targets_many_sources(cfg3, mode):
    # only the 64 side-wall collocation points of the 128k workload: one target
    # tile against every source superblock, so the call splits the sources over
    # hundreds of waves and reduces the partials in a second pass
    import torch
    import oracle
    import paper_1510_05616_amd as s2d
    t = cfg3.trg
    side = np.where(t.kind == 2)[0]
    tx, ty = t.x[side], t.y[side]
    ves, wall = s2d.Curves(cfg3.ves), s2d.Curves(cfg3.wall)
    tg = s2d.Targets(tx, ty)
    for img in ((-1, 1), (1, 1), (-1, -1)):
        u = torch.zeros(len(side), dtype=torch.float64, device="cuda")
        v = torch.zeros_like(u)
        s2d.stokes2d_slp_eval(mode, ves, tg, cfg3.d, img[0], img[1], cfg3.mu, u, v)
        ou, ov = oracle.slp(cfg3.ves, tx, ty, None, None, cfg3.d, img[0], img[1], cfg3.mu)
        e1 = rel_err(u.cpu().numpy(), v.cpu().numpy(), ou, ov)
        s2d.stokes2d_dlp_eval(mode, wall, tg, cfg3.d, img[0], img[1], u, v)
        ou, ov = oracle.dlp(cfg3.wall, tx, ty, None, None, cfg3.d, img[0], img[1])
        e2 = rel_err(u.cpu().numpy(), v.cpu().numpy(), ou, ov)
        print(f"side targets mode={mode} images={img}: slp {e1:.2e} dlp {e2:.2e}", flush=True)
        assert e1 <= TOL[mode] and e2 <= TOL[mode]
