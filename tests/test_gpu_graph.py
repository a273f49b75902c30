"""Single-call entry points recorded into a HIP graph (stream capture through
torch.cuda.graph) and replayed: every call launches kernels only, so a replay
must reproduce an eager call bit for bit, also after the inputs the graph
reads were overwritten in place and with unrelated eager work between
replays."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1510_05616_amd as s2d
    s2d.stokes2d_init(0)
    yield


def _capture(fn):
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):          # warm-up outside the capture
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("mode", [0, 1])
def test_layer_potentials_replay_in_a_graph(mode):
    import torch
    import paper_1510_05616_amd as s2d
    prob = synth.make_config(2)
    t = prob.trg
    ves, wall = s2d.Curves(prob.ves), s2d.Curves(prob.wall)
    tv = s2d.Targets(t.x, t.y, t.ves_curve, t.ves_node)
    tw = s2d.Targets(t.x, t.y, t.wall_curve, t.wall_node)
    n = t.n
    f64 = dict(dtype=torch.float64, device="cuda")

    def ws(op, trg, src):
        return torch.empty(s2d.stokes2d_workspace_size(op, mode, src, trg), dtype=torch.uint8, device="cuda")

    ws_g = (ws(s2d.S2D_OP_SLP, tv, ves), ws(s2d.S2D_OP_DLP, tw, wall))
    ws_e = (ws(s2d.S2D_OP_SLP, tv, ves), ws(s2d.S2D_OP_DLP, tw, wall))
    u, v = torch.zeros(n, **f64), torch.zeros(n, **f64)

    def step(w, uu, vv):
        s2d.stokes2d_slp_eval(mode, ves, tv, prob.d, -1, 1, prob.mu, uu, vv, ws=w[0])
        s2d.stokes2d_dlp_eval(mode, wall, tw, prob.d, -1, 1, uu, vv, accumulate=1, ws=w[1])

    g = _capture(lambda: step(ws_g, u, v))
    fx0, fy0, tx0 = ves.fx.clone(), ves.fy.clone(), wall.fx.clone()
    other_u, other_v = torch.zeros(n, **f64), torch.zeros(n, **f64)
    for k in range(4):
        # new densities in the buffers the graph reads
        ves.fx.copy_(fx0 * (1.0 + 0.25 * k))
        ves.fy.copy_(fy0 - 0.5 * k)
        wall.fx.copy_(tx0 * math.cos(0.3 * k))
        ue, ve = torch.zeros(n, **f64), torch.zeros(n, **f64)
        step(ws_e, ue, ve)
        # unrelated eager work on the stream, with the other precision
        s2d.stokes2d_slp_eval(1 - mode, ves, tv, prob.d, 0, 0, 2.0, other_u, other_v)
        torch.cuda.synchronize()
        u.fill_(float("nan"))
        v.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(u, ue) and torch.equal(v, ve), f"replay {k}"
    # the replayed field still matches the oracle for the last densities
    import oracle
    c = synth.CurveSet(prob.ves.x, prob.ves.y, prob.ves.nx, prob.ves.ny, prob.ves.w, prob.ves.kappa,
                       ves.fx.cpu().numpy(), ves.fy.cpu().numpy(), curve_off=prob.ves.curve_off)
    idx = np.arange(0, n, 37)
    ou, ov = oracle.slp(c, t.x[idx], t.y[idx], t.ves_curve[idx], t.ves_node[idx], prob.d, -1, 1, prob.mu)
    w_ = prob.wall
    cw = synth.CurveSet(w_.x, w_.y, w_.nx, w_.ny, w_.w, w_.kappa, wall.fx.cpu().numpy(), w_.fy,
                        curve_off=w_.curve_off)
    du, dv = oracle.dlp(cw, t.x[idx], t.y[idx], t.wall_curve[idx], t.wall_node[idx], prob.d, -1, 1)
    ou, ov = ou + du, ov + dv
    un, vn = u.cpu().numpy()[idx], v.cpu().numpy()[idx]
    err = np.hypot(un - ou, vn - ov).max() / np.hypot(ou, ov).max()
    print(f"mode={mode} replayed field vs oracle: {err:.2e}", flush=True)
    assert err <= (1e-12 if mode == 0 else 1e-6)


def test_near_correction_replays_in_a_graph():
    import torch
    from paper_1510_05616_amd import near
    from oracle import near as onear
    c, tx, ty, tc, dh = synth.make_near_dataset(3000, seed=23, per_curve=150)
    data = near.NearData(c, tx, ty, tc, mu=1.0, upsample=8, labels=False)
    p = onear.init_params(seed=4, mu_in=np.zeros(14), sd_in=np.ones(14))
    prm = torch.as_tensor(near.dict_to_params(p).astype(np.float32), device="cuda")
    # bins below b = 0.5 fall back to the upsampled quadrature, the others use
    # the learned route: both branches and the fallback mask are exercised
    half = int(round((math.log10(0.5) - near.BIN_LO) / near.BIN_W))
    bound = torch.tensor([1.0] * half + [1e-9] * (near.N_BINS - half), dtype=torch.float32,
                         device="cuda").repeat_interleave(near.CELL)
    bound0 = torch.ones(near.N_BINS * near.CELL, dtype=torch.float32, device="cuda")
    blob = torch.zeros(near.near_mlp_blob_size(), dtype=torch.uint8, device="cuda")
    near.near_mlp_pack(prm, bound, near.N_BINS, near.BIN_LO, near.BIN_W, blob, bound_zero=bound0)
    n = data.n
    f64 = dict(dtype=torch.float64, device="cuda")
    wsz = near.near_workspace_size(near.S2D_NEAR_AUTO, data.curves, data.trg, 8)
    ws_g = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    ws_e = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    du, dv = torch.zeros(n, **f64), torch.zeros(n, **f64)
    fb = torch.zeros(n, dtype=torch.int32, device="cuda")

    def step(w, a, b, f):
        near.near_correct_eval(near.S2D_NEAR_AUTO, data.curves, data.trg, data.tc, 8, blob, 1e-6, 1.0, a, b, f,
                               ws=w)

    g = _capture(lambda: step(ws_g, du, dv, fb))
    fx0 = data.curves.fx.clone()
    for k in range(3):
        data.curves.fx.copy_(fx0 * (1.0 - 0.3 * k))
        de, ee = torch.zeros(n, **f64), torch.zeros(n, **f64)
        fe = torch.zeros(n, dtype=torch.int32, device="cuda")
        step(ws_e, de, ee, fe)
        torch.cuda.synchronize()
        du.fill_(float("nan"))
        dv.fill_(float("nan"))
        fb.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(fb, fe), f"replay {k}"
        assert bool((fe == 0).any()) and bool((fe == 1).any())
        assert torch.equal(du, de) and torch.equal(dv, ee), f"replay {k}"
