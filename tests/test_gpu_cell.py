"""GPU checks of the periodization system of one channel cell: the four
blocks filled on the GPU against the oracle's dense assembly, and the
factored solve (rocSOLVER LU, rocBLAS GEMM, SVD pseudo-inverse) reproducing
the Poiseuille flow of the paper's periodization test (Section 5) and the
oracle's solution."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

ALPHA, MU = 0.2, 0.7
PTS = (np.array([0.8, 3.2, 4.8]), np.zeros(3))


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1510_05616_amd as s2d
    s2d.stokes2d_init(0)
    yield


def test_blocks_match_the_oracle():
    from oracle import els
    from paper_1510_05616_amd.cell import Cell
    walls, sy, d = synth.make_channel(64, 8)
    ref = els.assemble(walls, sy, d, 32, 0.9)[:4]
    got = Cell(walls, sy, d, 32, 0.9).assemble()
    for name, g, r in zip("ABCQ", got, ref):
        g = g.cpu().numpy()
        assert g.shape == r.shape, name
        e = np.abs(g - r).max() / np.abs(r).max()
        print(f"block {name} {r.shape}: {e:.2e}", flush=True)
        assert e < 1e-13, name


def _solve(Nw, K, M, alpha=ALPHA, lu_panel=0):
    import torch
    from paper_1510_05616_amd.cell import Cell
    walls, sy, d = synth.make_channel(Nw, K)
    cell = Cell(walls, sy, d, M, MU, lu_panel=lu_panel)
    cell.factor()
    v, g = synth.poiseuille_cell_data(walls, sy, d, alpha, MU)
    f64 = dict(dtype=torch.float64, device="cuda")
    tau, c = cell.solve(torch.as_tensor(v, **f64), torch.as_tensor(g, **f64))
    return walls, sy, d, cell, tau, c


def _errors(u, v, p, d, alpha=ALPHA):
    ue, pe = synth.poiseuille(*PTS, alpha, MU)
    un = np.stack([u.cpu().numpy(), v.cpu().numpy()], 1)
    pn = p.cpu().numpy()
    eu = np.abs(un - ue).max() / (alpha * 1.3 ** 2)
    ep = np.abs((pn - pn[0]) - (pe - pe[0])).max() / (2 * alpha * MU * d)
    return eu, ep


def test_poiseuille_flow_on_the_gpu():
    from oracle import els
    walls, sy, d, cell, tau, c = _solve(128, 32, 128)
    u, v, p = cell.flow(tau, c, *PTS)
    eu, ep = _errors(u, v, p, d)
    print(f"GPU Poiseuille: velocity {eu:.2e}, pressure {ep:.2e}", flush=True)
    assert eu < 1e-10 and ep < 1e-10
    # the same representation from the oracle's solve
    A, B, C, Q, (px, py) = els.assemble(walls, sy, d, 128, MU)
    vv, gg = synth.poiseuille_cell_data(walls, sy, d, ALPHA, MU)
    t_o, c_o = els.solve(A, B, C, Q, vv, gg)
    uo, po = els.field(walls, t_o, px, py, c_o, d, MU, *PTS)
    du = np.abs(np.stack([u.cpu().numpy(), v.cpu().numpy()], 1) - uo).max() / (ALPHA * 1.3 ** 2)
    print(f"GPU vs oracle field: {du:.2e}", flush=True)
    assert du < 1e-10


def test_one_factorization_serves_several_right_hand_sides():
    import torch
    walls, sy, d, cell, tau, c = _solve(96, 16, 64)
    v, g = synth.poiseuille_cell_data(walls, sy, d, ALPHA, MU)
    f64 = dict(dtype=torch.float64, device="cuda")
    # scaling by 2 is exact, so the solve must scale bit for bit
    t2, c2 = cell.solve(torch.as_tensor(2.0 * v, **f64), torch.as_tensor(2.0 * g, **f64))
    t1, c1 = cell.solve(torch.as_tensor(v, **f64), torch.as_tensor(g, **f64))
    torch.cuda.synchronize()
    assert torch.equal(t1, tau) and torch.equal(c1, c)                # deterministic
    assert torch.equal(t2, 2.0 * t1) and torch.equal(c2, 2.0 * c1)
    # superposition of two flows (alpha = 0.2 and 0.5), seen in the velocity
    # field to the accuracy of the method (c itself is only determined up to
    # the dropped singular directions, which the pseudo-inverse amplifies)
    v5, g5 = synth.poiseuille_cell_data(walls, sy, d, 0.5, MU)
    ts, cs = cell.solve(torch.as_tensor(v + v5, **f64), torch.as_tensor(g + g5, **f64))
    t5, c5 = cell.solve(torch.as_tensor(v5, **f64), torch.as_tensor(g5, **f64))
    us = cell.flow(ts, cs, *PTS)
    ua = cell.flow(t1, c1, *PTS)
    ub = cell.flow(t5, c5, *PTS)
    for s_, a_, b_ in zip(us[:2], ua[:2], ub[:2]):
        assert (s_ - a_ - b_).abs().max().item() < 1e-10 * max(1.0, s_.abs().max().item())
    # the pressure is fixed only up to a constant (the cell problem's nullity)
    dp = [q - q[0] for q in (us[2], ua[2], ub[2])]
    assert (dp[0] - dp[1] - dp[2]).abs().max().item() < 1e-10 * max(1.0, dp[0].abs().max().item())


@pytest.mark.parametrize("mode", [0, 1])
def test_larger_channel_both_evaluation_modes(mode):
    walls, sy, d, cell, tau, c = _solve(1000, 32, 128)
    u, v, p = cell.flow(tau, c, *PTS, mode=mode)
    eu, ep = _errors(u, v, p, d)
    print(f"N=2x1000 mode={mode}: velocity {eu:.2e}, pressure {ep:.2e}", flush=True)
    assert max(eu, ep) < (1e-10 if mode == 0 else 1e-6)


def test_narrow_lu_panels_give_the_same_flow():
    """The blocked LU with narrow panels (many rocSOLVER panels, row
    interchanges across panels, TRSM / GEMM updates cut into column chunks)
    against the single-panel factorisation and the oracle's dense solve."""
    import torch
    from oracle import els
    fields = {}
    for panel in (0, 100, 37):
        walls, sy, d, cell, tau, c = _solve(300, 16, 64, lu_panel=panel)
        u, v, p = cell.flow(tau, c, *PTS)
        eu, ep = _errors(u, v, p, d)
        # the first block row holds to rounding: tau = A^-1 (v - B c)
        A, B, _, _ = cell.assemble()
        vv, _ = synth.poiseuille_cell_data(walls, sy, d, ALPHA, MU)
        vt = torch.as_tensor(vv, dtype=torch.float64, device="cuda")
        res = (A @ tau + B @ c - vt).abs().max().item()
        scale = (A.abs().sum(1).max() * tau.abs().max() + B.abs().sum(1).max() * c.abs().max()).item()
        print(f"lu_panel {panel}: velocity {eu:.2e}, pressure {ep:.2e}, A tau + B c - v {res / scale:.2e}",
              flush=True)
        assert eu < 1e-10 and ep < 1e-10, panel
        assert res < 1e-14 * scale, panel
        fields[panel] = np.stack([u.cpu().numpy(), v.cpu().numpy()], 1)
    # the truncated pseudo-inverse passes rounding differences of S on to c
    # (the dropped directions), so the fields agree to the method's accuracy
    for panel in (100, 37):
        assert np.abs(fields[panel] - fields[0]).max() < 1e-10 * ALPHA, panel
    A, B, C, Q, (px, py) = els.assemble(walls, sy, d, 64, MU)
    vv, gg = synth.poiseuille_cell_data(walls, sy, d, ALPHA, MU)
    t_o, c_o = els.solve(A, B, C, Q, vv, gg)
    uo, _ = els.field(walls, t_o, px, py, c_o, d, MU, *PTS)
    assert np.abs(fields[37] - uo).max() < 1e-10 * ALPHA


def test_poiseuille_at_16000_nodes_per_wall():
    """The cell at 2 x 16,000 wall nodes (a 64,000^2 dense block, 4.1e9
    elements, factored in four panels of at most 16,640 columns): the
    Poiseuille flow at the test points."""
    import time
    import torch
    t0 = time.time()
    walls, sy, d, cell, tau, c = _solve(16000, 32, 128)
    torch.cuda.synchronize()
    t1 = time.time()
    u, v, p = cell.flow(tau, c, *PTS)
    eu, ep = _errors(u, v, p, d)
    print(f"N=2x16000: factor + solve {t1 - t0:.1f} s, velocity {eu:.2e}, pressure {ep:.2e}", flush=True)
    assert eu < 1e-9 and ep < 1e-9
    del cell
    torch.cuda.empty_cache()
