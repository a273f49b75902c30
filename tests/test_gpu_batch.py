"""Batched evaluation (persistent work-list launch recorded in a HIP graph)
against the FP64 oracle, per instance; graph replays re-read the inputs."""
import numpy as np
import pytest

import synth
from _common import rel_err, worse

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-6}


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    assert torch.cuda.is_available()
    import paper_1510_05616_amd as s2d
    s2d.stokes2d_init(0)
    yield
    s2d.stokes2d_batch_release()


def _instances(probs):
    import torch
    import paper_1510_05616_amd as s2d
    out = []
    for p in probs:
        t = p.trg
        u = torch.zeros(t.n, dtype=torch.float64, device="cuda")
        v = torch.zeros_like(u)
        out.append(s2d.BatchInstance(s2d.Curves(p.ves), s2d.Curves(p.wall),
                                     s2d.Targets(t.x, t.y, t.ves_curve, t.ves_node),
                                     s2d.Targets(t.x, t.y, t.wall_curve, t.wall_node), p.d, p.mu, u, v))
    return out


def _oracle(p, idx=None):
    import oracle
    t = p.trg
    sel = slice(None) if idx is None else idx
    us, vs = oracle.slp(p.ves, t.x[sel], t.y[sel], t.ves_curve[sel], t.ves_node[sel], p.d, -1, 1, p.mu)
    ud, vd = oracle.dlp(p.wall, t.x[sel], t.y[sel], t.wall_curve[sel], t.wall_node[sel], p.d, -1, 1)
    return us + ud, vs + vd


@pytest.fixture(scope="module")
def small_batch():
    return synth.make_batch(12, seed=40, max_ves=8, wall_range=(200, 900))


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_parity_small(small_batch, mode):
    import torch
    import paper_1510_05616_amd as s2d
    insts = _instances(small_batch)
    ws = torch.empty(s2d.stokes2d_batch_workspace_size(mode, insts), dtype=torch.uint8, device="cuda")
    s2d.stokes2d_batch_eval(mode, insts, ws)
    torch.cuda.synchronize()
    worst = 0.0
    for p, b in zip(small_batch, insts):
        ou, ov = _oracle(p)
        e = rel_err(b.u.cpu().numpy(), b.v.cpu().numpy(), ou, ov)
        worst = worse(worst, e)
    print(f"batch mode={mode} worst E={worst:.3e}", flush=True)
    assert worst <= TOL[mode]


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_instances_far_from_the_origin(small_batch, mode):
    """Instances moved to different places up to 5e4 from the origin (FP32C
    works in offsets from per-sub-block origins; the padding records of each
    instance copy its last source)."""
    import dataclasses
    import torch
    import paper_1510_05616_amd as s2d
    rng = np.random.default_rng(7)
    moved = []
    for p in small_batch[:6]:
        dx, dy = rng.uniform(-5e4, 5e4, 2)
        mv = lambda cs: dataclasses.replace(cs, x=cs.x + dx, y=cs.y + dy)
        moved.append(dataclasses.replace(p, ves=mv(p.ves), wall=mv(p.wall),
                                         trg=dataclasses.replace(p.trg, x=p.trg.x + dx, y=p.trg.y + dy)))
    insts = _instances(moved)
    ws = torch.empty(s2d.stokes2d_batch_workspace_size(mode, insts), dtype=torch.uint8, device="cuda")
    s2d.stokes2d_batch_eval(mode, insts, ws)
    torch.cuda.synchronize()
    worst = 0.0
    for p, b in zip(moved, insts):
        ou, ov = _oracle(p)
        worst = worse(worst, rel_err(b.u.cpu().numpy(), b.v.cpu().numpy(), ou, ov))
    print(f"moved batch mode={mode} worst E={worst:.3e}", flush=True)
    assert worst <= TOL[mode]


def test_batch_replay_rereads_inputs(small_batch):
    import torch
    import paper_1510_05616_amd as s2d
    mode = 1
    insts = _instances(small_batch)
    ws = torch.empty(s2d.stokes2d_batch_workspace_size(mode, insts), dtype=torch.uint8, device="cuda")
    s2d.stokes2d_batch_eval(mode, insts, ws)
    torch.cuda.synchronize()
    first = [b.u.clone() for b in insts]
    s2d.stokes2d_batch_eval(mode, insts, ws)           # graph replay
    torch.cuda.synchronize()
    for a, b in zip(first, insts):
        assert torch.equal(a, b.u)
    # change densities in place (same pointers): the replay must see them
    rng = np.random.default_rng(3)
    for p, b in zip(small_batch, insts):
        p.ves.fx[:] = rng.normal(size=p.ves.n_nodes) * 0.3
        p.wall.fy[:] = rng.normal(size=p.wall.n_nodes) * 0.2
        b.ves.fx.copy_(torch.as_tensor(p.ves.fx))
        b.wall.fy.copy_(torch.as_tensor(p.wall.fy))
    s2d.stokes2d_batch_eval(mode, insts, ws)
    torch.cuda.synchronize()
    for p, b in zip(small_batch, insts):
        ou, ov = _oracle(p)
        assert rel_err(b.u.cpu().numpy(), b.v.cpu().numpy(), ou, ov) <= TOL[mode]


def test_batch_matches_single_calls(small_batch):
    import torch
    import paper_1510_05616_amd as s2d
    insts = _instances(small_batch[:4])
    mode = 1
    ws = torch.empty(s2d.stokes2d_batch_workspace_size(mode, insts), dtype=torch.uint8, device="cuda")
    s2d.stokes2d_batch_eval(mode, insts, ws)
    for b in insts:
        u = torch.zeros_like(b.u)
        v = torch.zeros_like(b.v)
        s2d.stokes2d_slp_eval(mode, b.ves, b.trg_ves, b.d, -1, 1, b.mu, u, v)
        s2d.stokes2d_dlp_eval(mode, b.wall, b.trg_wall, b.d, -1, 1, u, v, accumulate=1)
        torch.cuda.synchronize()
        sc = torch.hypot(u, v).max().item()
        assert (torch.hypot(u - b.u, v - b.v).max().item() / sc) < 2e-7


def test_batch_config4_full_size_sampled():
    import torch
    import paper_1510_05616_amd as s2d
    probs = synth.make_batch(256)
    insts = _instances(probs)
    mode = 1
    ws = torch.empty(s2d.stokes2d_batch_workspace_size(mode, insts), dtype=torch.uint8, device="cuda")
    s2d.stokes2d_batch_eval(mode, insts, ws)
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    worst = 0.0
    for k in rng.choice(len(probs), 6, replace=False):
        p, b = probs[k], insts[k]
        idx = np.sort(rng.choice(p.trg.n, min(200, p.trg.n), replace=False))
        ou, ov = _oracle(p, idx)
        e = rel_err(b.u.cpu().numpy()[idx], b.v.cpu().numpy()[idx], ou, ov)
        worst = worse(worst, e)
    print(f"config4 sampled worst E={worst:.3e}", flush=True)
    assert worst <= TOL[mode]
