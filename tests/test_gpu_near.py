"""GPU checks of the near-field correction: upsampled FP64 quadrature, node
derivatives, features, frames, training records, the straight-line part and
the network head against the oracle; training-kernel gradients against the
FP64 oracle backward pass and finite differences, Adam against the oracle
step, BF16 inference against the FP32 forward pass, feature statistics and
calibration against plain reductions, the AUTO decision rule, and what a
trained network gains over the plain trapezoid rule."""
import math

import numpy as np

from _common import worse
import pytest

import synth
from oracle import near as onear

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    assert torch.cuda.is_available()
    import paper_1510_05616_amd as s2d
    s2d.stokes2d_init(0)
    yield


@pytest.fixture(scope="module")
def small():
    from paper_1510_05616_amd import near
    c, tx, ty, tc, dh = synth.make_near_dataset(3000, seed=21, per_curve=150)
    return c, tx, ty, tc, dh, near.NearData(c, tx, ty, tc, mu=1.0, upsample=8)


def test_upsampled_quadrature_matches_oracle(small):
    import oracle
    c, tx, ty, tc, dh, data = small
    du = data.du.cpu().numpy()
    dv = data.dv.cpu().numpy()
    worst = 0.0
    for k in range(c.n_curves):
        sel = np.where(tc == k)[0]
        s = slice(c.curve_off[k], c.curve_off[k + 1])
        ou, ov = onear.near_label(c.x[s], c.y[s], c.fx[s], c.fy[s], c.w[s], tx[sel], ty[sel], P=8)
        sub = synth.CurveSet(*(getattr(c, a)[s] for a in ("x", "y", "nx", "ny", "w", "kappa", "fx", "fy")),
                             curve_off=np.array([0, s.stop - s.start], np.int32))
        u1, v1 = oracle.slp(sub, tx[sel], ty[sel])
        sc = np.hypot(u1 + ou, v1 + ov).max()
        worst = worse(worst, np.hypot(du[sel] - ou, dv[sel] - ov).max() / sc)
    print(f"upsampled quadrature worst rel err {worst:.2e}", flush=True)
    assert worst < 1e-12


@pytest.mark.parametrize("P,sizes", [(1, (66, 70)), (3, (66, 126)), (5, (64, 98)), (16, (4, 128)), (32, (64,)),
                                     (8, (256,))])
def test_upsampled_quadrature_other_factors(P, sizes):
    """Upsampling factors other than 8, curve sizes with N/2 odd (P N not a
    multiple of 4), and the largest N (256) and P N (2048) the kernel takes."""
    import oracle
    from paper_1510_05616_amd import near
    c, tx, ty, tc, dh = synth.make_near_dataset(600, seed=40 + P, per_curve=100, sizes=sizes)
    data = near.NearData(c, tx, ty, tc, mu=1.0, upsample=P)
    du = data.du.cpu().numpy()
    dv = data.dv.cpu().numpy()
    worst = 0.0
    for k in range(c.n_curves):
        sel = np.where(tc == k)[0]
        s = slice(c.curve_off[k], c.curve_off[k + 1])
        ou, ov = onear.near_label(c.x[s], c.y[s], c.fx[s], c.fy[s], c.w[s], tx[sel], ty[sel], P=P)
        sub = synth.CurveSet(*(getattr(c, a)[s] for a in ("x", "y", "nx", "ny", "w", "kappa", "fx", "fy")),
                             curve_off=np.array([0, s.stop - s.start], np.int32))
        u1, v1 = oracle.slp(sub, tx[sel], ty[sel])
        sc = np.hypot(u1 + ou, v1 + ov).max()
        worst = worse(worst, np.hypot(du[sel] - ou, dv[sel] - ov).max() / sc)
    print(f"P={P} sizes={sizes}: upsampled quadrature worst rel err {worst:.2e}", flush=True)
    assert worst < 1e-12


def test_upsampled_and_trapezoid_sums_match_oracle(small):
    """near_upsampled_slp returns the fine (P = 8) and plain trapezoid single
    layers separately; each against the oracle's sums over the upsampled and
    the given nodes, and their difference against near_correct_eval."""
    import torch
    from paper_1510_05616_amd import near
    c, tx, ty, tc, dh, data = small
    n = len(tx)
    out = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(4)]
    near.near_upsampled_slp(data.curves, data.trg, data.tc, 8, 1.0, *out)
    uP, vP, u1, v1 = (o.cpu().numpy() for o in out)
    worst_f = worst_c = 0.0
    for k in range(c.n_curves):
        sel = np.where(tc == k)[0]
        s = slice(c.curve_off[k], c.curve_off[k + 1])
        xu, yu, wu, fxu, fyu = onear.upsample_curve(c.x[s], c.y[s], c.fx[s], c.fy[s], 8)
        ouP, ovP = onear.slp_trap(xu, yu, wu, fxu, fyu, tx[sel], ty[sel])
        ou1, ov1 = onear.slp_trap(c.x[s], c.y[s], c.w[s], c.fx[s], c.fy[s], tx[sel], ty[sel])
        sc = np.hypot(ouP, ovP).max()
        worst_f = worse(worst_f, np.hypot(uP[sel] - ouP, vP[sel] - ovP).max() / sc)
        worst_c = worse(worst_c, np.hypot(u1[sel] - ou1, v1[sel] - ov1).max() / sc)
    du, dv = data.du.cpu().numpy(), data.dv.cpu().numpy()
    gap = np.hypot((uP - u1) - du, (vP - v1) - dv).max() / np.hypot(uP, vP).max()
    print(f"fine {worst_f:.2e} trapezoid {worst_c:.2e} difference vs near_correct_eval {gap:.2e}", flush=True)
    assert worst_f < 1e-12 and worst_c < 1e-12 and gap < 1e-14


def test_invalid_targets_and_curves_give_nan():
    """Targets with a curve index out of range and targets of odd-sized
    curves get NaN; the valid targets sharing their waves still match the
    oracle (the per-lane path of the quadrature)."""
    import oracle
    from paper_1510_05616_amd import near
    c, tx, ty, tc, dh = synth.make_near_dataset(700, seed=44, per_curve=70, sizes=(63, 64, 96))
    tc = tc.copy()
    rng = np.random.default_rng(4)
    bad = rng.choice(len(tx), 40, replace=False)
    tc[bad[:20]] = -1
    tc[bad[20:]] = c.n_curves
    data = near.NearData(c, tx, ty, tc, mu=1.0, upsample=8)
    du, dv = data.du.cpu().numpy(), data.dv.cpu().numpy()
    N = np.diff(c.curve_off)
    valid = (tc >= 0) & (tc < c.n_curves)
    valid[valid] &= N[tc[valid]] % 2 == 0
    assert (~valid).sum() > 40 and valid.sum() > 300
    assert np.all(np.isnan(du[~valid])) and np.all(np.isnan(dv[~valid]))
    worst = 0.0
    for k in range(c.n_curves):
        if N[k] % 2:
            continue
        sel = np.where(tc == k)[0]
        s = slice(c.curve_off[k], c.curve_off[k + 1])
        ou, ov = onear.near_label(c.x[s], c.y[s], c.fx[s], c.fy[s], c.w[s], tx[sel], ty[sel], P=8)
        sub = synth.CurveSet(*(getattr(c, a)[s] for a in ("x", "y", "nx", "ny", "w", "kappa", "fx", "fy")),
                             curve_off=np.array([0, s.stop - s.start], np.int32))
        u1, v1 = oracle.slp(sub, tx[sel], ty[sel])
        sc = np.hypot(u1 + ou, v1 + ov).max()
        worst = worse(worst, np.hypot(du[sel] - ou, dv[sel] - ov).max() / sc)
    print(f"valid targets beside invalid ones: worst rel err {worst:.2e}", flush=True)
    assert worst < 1e-12


def test_curves_beyond_the_upsampling_limits_give_nan():
    """Curves of more than 256 nodes, or with P N above 2048, are not
    upsampled: their targets get NaN, the other curves' targets do not."""
    from paper_1510_05616_amd import near
    c, tx, ty, tc, dh = synth.make_near_dataset(400, seed=46, per_curve=100, sizes=(96, 258))
    N = np.diff(c.curve_off)
    assert (N == 258).any() and (N == 96).any()
    for P, big in ((8, N[tc] == 258), (32, N[tc] >= 96)):
        data = near.NearData(c, tx, ty, tc, mu=1.0, upsample=P)
        du = data.du.cpu().numpy()
        assert np.all(np.isnan(du[big])) and np.all(np.isfinite(du[~big])), P


def _sub(c, k):
    s = slice(c.curve_off[k], c.curve_off[k + 1])
    return synth.CurveSet(*(getattr(c, a)[s] for a in ("x", "y", "nx", "ny", "w", "kappa", "fx", "fy")),
                          curve_off=np.array([0, s.stop - s.start], np.int32))


def _oracle_features(c, tx, ty, tc):
    """Oracle features, frames (9) and head data d (n, 5, 2) per target."""
    n = len(tx)
    X = np.zeros((n, onear.N_FEAT))
    fr = np.zeros((n, onear.FRAME))
    dd = np.zeros((n, onear.N_DERIV, 2))
    for k in range(c.n_curves):
        sel = np.where(tc == k)[0]
        if sel.size:
            X[sel], fr[sel], dd[sel] = onear.features(_sub(c, k), tx[sel], ty[sel])
    return X, fr, dd


def test_node_derivatives_match_oracle():
    """Direct-sum node derivatives against the oracle's FFT ones: small curves
    (one workgroup each) and large ones (a wave per coefficient and node),
    N/2 odd and even, white-noise densities (every mode present)."""
    import torch
    from paper_1510_05616_amd import Curves
    from paper_1510_05616_amd import near
    rng = np.random.default_rng(12)
    parts = []
    for N in (8, 66, 256, 258, 2048, 4000):
        t = 2 * np.pi * np.arange(N) / N
        parts.append((np.cos(t), np.sin(t), np.cos(t), np.sin(t), np.full(N, 2 * np.pi / N), np.ones(N),
                      rng.standard_normal(N), rng.standard_normal(N)))
    c = synth.concat_curves(parts)
    dtab = torch.empty((c.x.shape[0], near.NDERIV), dtype=torch.float64, device="cuda")
    near.near_derivs_eval(Curves(c), dtab)
    got = dtab.cpu().numpy()
    for k in range(c.n_curves):
        s = slice(c.curve_off[k], c.curve_off[k + 1])
        ref = np.stack([onear.node_derivatives(c.fx[s]), onear.node_derivatives(c.fy[s])], 2)   # [p, N, comp]
        g = got[s].reshape(-1, onear.N_DERIV, 2).transpose(1, 0, 2)
        for p in range(onear.N_DERIV):
            e = np.abs(g[p] - ref[p]).max() / max(np.abs(ref[p]).max(), 1e-300)
            N = s.stop - s.start
            assert e < 1e-12 * max(1.0, math.sqrt(N) / 8), (N, p, e)
    # odd and tiny curves give NaN rows
    bad = synth.concat_curves([parts[0][:6] + (rng.standard_normal(8), rng.standard_normal(8)),
                               tuple(a[:7] for a in parts[1]), tuple(a[:2] for a in parts[1])])
    dtab = torch.zeros((bad.x.shape[0], near.NDERIV), dtype=torch.float64, device="cuda")
    near.near_derivs_eval(Curves(bad), dtab)
    g = dtab.cpu().numpy()
    assert np.all(np.isfinite(g[:8])) and np.all(np.isnan(g[8:]))


def test_features_match_oracle(small):
    c, tx, ty, tc, dh, data = small
    X = data.X.cpu().numpy()
    fr = data.frame.cpu().numpy()
    oX, ofr, odd = _oracle_features(c, tx, ty, tc)
    ex = np.abs(X - oX.astype(np.float32)) / np.maximum(np.abs(oX), 1.0)
    ef = np.abs(fr[:, :9] - ofr).max()
    dsc = np.abs(odd).max()
    ed = np.abs(fr[:, 9:19] - odd.reshape(-1, 10)).max() / dsc
    print(f"features {ex.max():.2e}, frame {ef:.2e}, derivatives {ed:.2e}", flush=True)
    assert ex.max() < 4e-7 and ef < 1e-12 and ed < 1e-12
    assert np.abs(fr[:, 19] - oX[:, 3]).max() < 1e-12


def test_training_records_match_oracle(small):
    """T = [d, R, wt, exp(-2 pi b)]: the label in the frame over the scale
    minus the oracle's straight-line prediction, the weight gain times the
    scale over the curve's largest |u_8|."""
    c, tx, ty, tc, dh, data = small
    from paper_1510_05616_amd import near
    T = data.T.cpu().numpy().astype(np.float64)
    fr = data.frame.cpu().numpy()
    du, dv = data.du.cpu().numpy(), data.dv.cpu().numpy()
    sc = fr[:, 6] / (4 * math.pi)
    oX, ofr, odd = _oracle_features(c, tx, ty, tc)
    R = onear.velocity_to_frame(du, dv, ofr, sc) - onear.flat_predict(ofr, odd, "slp", P=8)
    uref, vref = data.u_ref.cpu().numpy(), data.v_ref.cpu().numpy()
    cs = np.array([np.hypot(uref[tc == k], vref[tc == k]).max() for k in range(c.n_curves)])
    wt = near.WEIGHT_GAIN * sc / cs[tc]
    assert np.allclose(data.curve_scale.cpu().numpy()[:c.n_curves], cs, rtol=1e-7, atol=0)
    er = np.abs(T[:, 10:12] - R).max() / np.abs(R).max()
    ew = np.abs(T[:, 12] - wt).max() / wt.max()
    ee = np.abs(T[:, 13] - np.exp(-2 * np.pi * ofr[:, 1])).max()
    ed = np.abs(T[:, :10] - odd.reshape(-1, 10)).max() / np.abs(odd).max()
    print(f"records: R {er:.2e} wt {ew:.2e} env {ee:.2e} d {ed:.2e}", flush=True)
    assert er < 1e-6 and ew < 1e-6 and ee < 1e-7 and ed < 1e-7


def _rand_params(seed=3, scale_out=1.0):
    rng = np.random.default_rng(seed)
    p = onear.init_params(seed=seed, mu_in=rng.normal(size=14) * 0.2, sd_in=0.5 + rng.random(14))
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = rng.normal(size=p[k].shape) * 0.1
    p["W4"] *= scale_out
    p["b4"] *= scale_out
    return p


def _rand_records(rng, n):
    X = rng.normal(size=(n, 14))
    X[:, 1] = rng.uniform(0.05, 1.5, n)                   # b (the envelope reads it)
    dd = rng.normal(size=(n, 5, 2))
    R = rng.normal(size=(n, 2)) * 0.05
    wt = rng.uniform(0.2, 2.0, n)
    T = np.concatenate([dd.reshape(n, 10), R, wt[:, None], np.exp(-2 * np.pi * X[:, 1])[:, None]], 1)
    return X, dd, R, wt, T


def test_training_gradient_matches_oracle_and_finite_differences():
    import torch
    from paper_1510_05616_amd import near
    rng = np.random.default_rng(5)
    B = 96
    X, dd, R, wt, T = _rand_records(rng, B + 10)
    X32, T32 = X.astype(np.float32), T.astype(np.float32)
    idx = rng.permutation(B + 10)[:B].astype(np.int32)
    pd = _rand_params()
    p32 = near.dict_to_params(pd).astype(np.float32)
    pd32 = near.params_to_dict(p32)                      # the oracle sees the FP32-rounded weights
    T64 = T32.astype(np.float64)
    L, g = onear.mlp_loss_grad(pd32, X32.astype(np.float64)[idx], T64[idx, :10].reshape(-1, 5, 2),
                               T64[idx, 10:12], T64[idx, 12])
    dev = "cuda"
    Xt = torch.as_tensor(X32, device=dev)
    Tt = torch.as_tensor(T32, device=dev)
    it = torch.as_tensor(idx, device=dev)
    prm = torch.as_tensor(p32, device=dev)
    grad = torch.zeros_like(prm)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    ws = torch.empty(near.near_mlp_train_workspace_size(B), dtype=torch.uint8, device=dev)
    near.near_mlp_train_step(B, it, Xt, Tt, prm, None, None, 0, 0.0, grad, loss, ws)
    torch.cuda.synchronize()
    gg = near.params_to_dict(grad.cpu().numpy())
    print(f"loss {loss.item():.6e} oracle {L:.6e}", flush=True)
    assert abs(loss.item() - L) <= 1e-5 * abs(L)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"):
        sc = np.abs(g[k]).max()
        assert np.abs(gg[k] - g[k]).max() <= 2e-4 * sc, k
    # the training kernels read the stored envelope; the oracle recomputes it
    # from b = X[:, 1]: equal up to FP32 rounding, covered by the tolerances
    for name, j in (("W1", 37), ("W3", 1000), ("b4", 1), ("W4", 50)):
        e = 1e-2
        vals = []
        for sgn in (1, -1):
            q = p32.copy()
            q[near.OFF[name] + j] += sgn * e
            near.near_mlp_train_step(B, it, Xt, Tt, torch.as_tensor(q, device=dev), None, None, 0, 0.0, grad, loss,
                                     ws)
            torch.cuda.synchronize()
            vals.append(loss.item())
        fd = (vals[0] - vals[1]) / (2 * e)
        gj = gg[name].reshape(-1)[j]
        assert abs(fd - gj) <= 2e-2 * max(abs(gj), 1e-3 * abs(L)), (name, fd, gj)


def test_adam_step_matches_oracle():
    import torch
    from paper_1510_05616_amd import near
    rng = np.random.default_rng(7)
    B = 64
    X, dd, R, wt, T = _rand_records(rng, B)
    X32, T32 = X.astype(np.float32), T.astype(np.float32)
    p32 = near.dict_to_params(_rand_params(8)).astype(np.float32)
    dev = "cuda"
    prm = torch.as_tensor(p32, device=dev)
    m = torch.zeros_like(prm)
    v = torch.zeros_like(prm)
    grad = torch.zeros_like(prm)
    ws = torch.empty(near.near_mlp_train_workspace_size(B), dtype=torch.uint8, device=dev)
    Xt, Tt = torch.as_tensor(X32, device=dev), torch.as_tensor(T32, device=dev)
    st = {}
    pd = near.params_to_dict(p32)
    T64 = T32.astype(np.float64)
    for step in (1, 2, 3):
        near.near_mlp_train_step(B, None, Xt, Tt, prm, m, v, step, 1e-3, grad, None, ws)
        L, g = onear.mlp_loss_grad(pd, X32.astype(np.float64), T64[:, :10].reshape(-1, 5, 2), T64[:, 10:12],
                                   T64[:, 12])
        onear.adam_step(pd, g, st, lr=1e-3)
    torch.cuda.synchronize()
    got = near.params_to_dict(prm.cpu().numpy())
    for k in ("W1", "W2", "b3", "W4"):
        assert np.abs(got[k] - pd[k]).max() < 5e-6, k


def test_feature_statistics_match_numpy(small):
    import torch
    from paper_1510_05616_amd import near
    c, tx, ty, tc, dh, data = small
    prm = torch.zeros(near.NPARAM, dtype=torch.float32, device="cuda")
    near.near_feature_stats(data.X, prm)
    torch.cuda.synchronize()
    X = data.X.double().cpu().numpy()
    p = prm.cpu().numpy()
    sd = X.std(0)
    assert np.allclose(p[:14], X.mean(0), rtol=1e-6, atol=1e-7 * np.abs(X).max())
    assert np.allclose(p[14:28], np.where(sd > 1e-30, sd, 1.0), rtol=1e-6)


def test_flat_part_and_bf16_head_match_oracle(small):
    """The learned route with an all-zero network is the straight-line part
    alone: FP64 against the oracle's closed form.  With a random network the
    head adds exp(-2 pi b) sum_p dC_p d_p from BF16 weights and activations:
    against the oracle's FP64 head of the same FP32 weights, within the BF16
    rounding; the FP32 forward pass against the oracle's forward pass."""
    import torch
    from paper_1510_05616_amd import near
    c, tx, ty, tc, dh, data = small
    oX, ofr, odd = _oracle_features(c, tx, ty, tc)
    sc = ofr[:, 6] / (4 * math.pi)
    flat = onear.flat_predict(ofr, odd, "slp", P=8)
    blob = torch.zeros(near.near_mlp_blob_size(), dtype=torch.uint8, device="cuda")
    du = torch.empty(data.n, dtype=torch.float64, device="cuda")
    dv = torch.empty_like(du)
    zero = torch.zeros(near.NPARAM, dtype=torch.float32, device="cuda")
    zero[14:28] = 1.0
    near.near_mlp_pack(zero, None, 0, near.BIN_LO, near.BIN_W, blob)
    data.correct(near.S2D_NEAR_MLP, blob, 0.0, du, dv)
    torch.cuda.synchronize()
    fu, fv = onear.frame_to_velocity(flat, ofr, sc)
    ref = np.hypot(fu, fv).max()
    e_flat = np.hypot(du.cpu().numpy() - fu, dv.cpu().numpy() - fv).max() / ref
    print(f"straight-line part vs oracle: {e_flat:.2e}", flush=True)
    assert e_flat < 1e-12
    pd = _rand_params(9, scale_out=0.1)
    p32 = torch.as_tensor(near.dict_to_params(pd).astype(np.float32), device="cuda")
    Y = torch.empty((data.n, near.NOUT), dtype=torch.float32, device="cuda")
    near.near_mlp_forward(data.X, p32, Y)
    torch.cuda.synchronize()
    pd32 = near.params_to_dict(p32.cpu().numpy())
    Yo, _ = onear.mlp_forward(pd32, data.X.double().cpu().numpy())
    assert np.abs(Y.cpu().numpy() - Yo).max() < 2e-5 * np.abs(Yo).max()
    near.near_mlp_pack(p32, None, 0, near.BIN_LO, near.BIN_W, blob)
    data.correct(near.S2D_NEAR_MLP, blob, 0.0, du, dv)
    torch.cuda.synchronize()
    hd = onear.head(Yo, data.X.double().cpu().numpy(), odd)
    hu, hv = onear.frame_to_velocity(flat + hd, ofr, sc)
    gu, gv = du.cpu().numpy(), dv.cpu().numpy()
    hs = np.hypot(*onear.frame_to_velocity(hd, ofr, sc)).max()
    err = np.hypot(gu - hu, gv - hv).max() / hs
    print(f"bf16 head vs fp64 oracle head: {err:.2e} of the largest head", flush=True)
    assert err < 3e-2


def _auto_blob(params_np, bound, bound_zero):
    import torch
    from paper_1510_05616_amd import near
    p32 = torch.as_tensor(near.dict_to_params(params_np).astype(np.float32), device="cuda")
    blob = torch.zeros(near.near_mlp_blob_size(), dtype=torch.uint8, device="cuda")
    near.near_mlp_pack(p32, bound, near.N_BINS, near.BIN_LO, near.BIN_W, blob, bound_zero=bound_zero)
    return blob


def test_auto_extremes(small):
    import torch
    from paper_1510_05616_amd import near
    c, tx, ty, tc, dh, data = small
    nt = near.N_BINS * near.CELL
    blob = _auto_blob(_rand_params(2), torch.full((nt,), 1e-3, device="cuda"), torch.full((nt,), 1.0, device="cuda"))
    du = torch.empty(data.n, dtype=torch.float64, device="cuda")
    dv = torch.empty_like(du)
    fb = torch.zeros(data.n, dtype=torch.int32, device="cuda")
    data.correct(near.S2D_NEAR_AUTO, blob, 0.0, du, dv, fb)
    torch.cuda.synchronize()
    assert torch.all(fb == 1)
    assert torch.equal(du, data.du) and torch.equal(dv, data.dv)
    # a huge threshold needs no correction at all (b >= b_min) ...
    data.correct(near.S2D_NEAR_AUTO, blob, 1e30, du, dv, fb)
    torch.cuda.synchronize()
    low = data.b < near.B_MIN
    assert low.any() and torch.all(fb[~low] == 2) and torch.all(du[~low] == 0)
    # ... and targets closer than b_min always take the quadrature
    assert torch.all(fb[low] == 1) and torch.equal(du[low], data.du[low])
    # between the two bounds the learned route is used inside the bins; past
    # the last bin only "none" or the quadrature
    sF = (data.frame[:, 6] / (4 * math.pi) * data.frame[:, 7])
    thr = 2e-3 * sF.max().item()
    data.correct(near.S2D_NEAR_AUTO, blob, thr, du, dv, fb)
    torch.cuda.synchronize()
    high = data.b >= near.B_MAX * (1 + 1e-6)
    mid = ~low & (data.b < near.B_MAX * (1 - 1e-6))
    assert high.any() and torch.all(fb[mid] == 0) and torch.all(fb[high] == 1)
    # targets at 1e-3 h, far below the trained and calibrated range, always
    # take the quadrature, whatever the tolerance
    close = near.NearData(*synth.make_near_dataset(640, seed=27, per_curve=160, delta_range=(1e-3, 1.2e-3))[:4])
    du2, dv2 = torch.empty(close.n, dtype=torch.float64, device="cuda"), torch.empty(close.n, dtype=torch.float64,
                                                                                      device="cuda")
    fb2 = torch.zeros(close.n, dtype=torch.int32, device="cuda")
    for tol in (0.0, thr, 1e30):
        close.correct(near.S2D_NEAR_AUTO, blob, tol, du2, dv2, fb2)
        torch.cuda.synchronize()
        assert torch.all(fb2 == 1) and torch.equal(du2, close.du) and torch.equal(dv2, close.dv)


def test_auto_mixed_decisions_match_each_route(small):
    """Bins alternate between the network, no correction and the fallback, so
    the three decisions interleave within waves. Fallback targets (compacted
    in order before the quadrature) must equal the upsampled result bit for
    bit, network targets the MLP route's result, the rest zero."""
    import torch
    from paper_1510_05616_amd import near
    c, tx, ty, tc, dh, data = small
    k = torch.arange(near.N_BINS * near.CELL, device="cuda") // near.CELL    # the b bin of each entry
    bound = torch.where(k % 3 == 0, 1e-3, 10.0).float()
    bound_zero = torch.where(k % 3 == 1, 1e-3, 10.0).float()
    blob = _auto_blob(_rand_params(3), bound, bound_zero)
    sF = (data.frame[:, 6] / (4 * math.pi) * data.frame[:, 7])
    thr = 2e-3 * sF.max().item()
    du, dv = (torch.empty(data.n, dtype=torch.float64, device="cuda") for _ in range(2))
    fb = torch.full((data.n,), -1, dtype=torch.int32, device="cuda")
    data.correct(near.S2D_NEAR_AUTO, blob, thr, du, dv, fb)
    mu_, mv_ = torch.empty_like(du), torch.empty_like(dv)
    data.correct(near.S2D_NEAR_MLP, blob, 0.0, mu_, mv_)
    torch.cuda.synchronize()
    counts = [int((fb == j).sum()) for j in range(3)]
    print(f"network/fallback/none {counts}", flush=True)
    assert min(counts) > 100 and sum(counts) == data.n
    f1, f0, f2 = fb == 1, fb == 0, fb == 2
    assert torch.equal(du[f1], data.du[f1]) and torch.equal(dv[f1], data.dv[f1])
    assert torch.equal(du[f0], mu_[f0]) and torch.equal(dv[f0], mv_[f0])
    assert torch.all(du[f2] == 0) and torch.all(dv[f2] == 0)
    # the decisions follow the bins: recompute them on the host in FP32
    b = data.b.float().cpu().numpy()
    pos = np.floor((np.log10(b) - np.float32(near.BIN_LO)) / np.float32(near.BIN_W))
    kk = pos.astype(int)
    exp = np.where(b < near.B_MIN, 1, np.where(kk % 3 == 1, 2, np.where(kk % 3 == 0, 0, 1)))
    past = 2 if (near.N_BINS - 1) % 3 == 1 else 1          # past the last b bin: its "none" entry or the quadrature
    exp = np.where((kk >= near.N_BINS) & (b >= near.B_MIN), past, exp)
    agree = (exp == fb.cpu().numpy()).mean()
    assert agree > 0.999, agree


def test_auto_lists_beyond_one_scan_segment():
    """300,000 targets: 1,172 compaction workgroups, more than the scan's
    1,024 threads, so each scan thread sums two counts. Both lists must still
    be complete and in order: fallback targets equal the upsampled route bit
    for bit, learned ones the MLP route, the rest zero."""
    import torch
    from paper_1510_05616_amd import near
    c, tx, ty, tc, dh = synth.make_near_dataset(300000, seed=29)
    data = near.NearData(c, tx, ty, tc, mu=1.0, upsample=8)
    assert (data.n + 255) // 256 > 1024
    k = torch.arange(near.N_BINS * near.CELL, device="cuda") // near.CELL
    bound = torch.where(k % 3 == 0, 1e-3, 10.0).float()
    bound_zero = torch.where(k % 3 == 1, 1e-3, 10.0).float()
    blob = _auto_blob(_rand_params(7), bound, bound_zero)
    sF = (data.frame[:, 6] / (4 * math.pi) * data.frame[:, 7])
    thr = 2e-3 * sF.max().item()
    du, dv = (torch.empty(data.n, dtype=torch.float64, device="cuda") for _ in range(2))
    fb = torch.full((data.n,), -1, dtype=torch.int32, device="cuda")
    data.correct(near.S2D_NEAR_AUTO, blob, thr, du, dv, fb)
    mu_, mv_ = torch.empty_like(du), torch.empty_like(dv)
    data.correct(near.S2D_NEAR_MLP, blob, 0.0, mu_, mv_)
    torch.cuda.synchronize()
    counts = [int((fb == j).sum()) for j in range(3)]
    print(f"network/fallback/none {counts}", flush=True)
    assert min(counts) > 10000 and sum(counts) == data.n
    f1, f0, f2 = fb == 1, fb == 0, fb == 2
    assert torch.equal(du[f1], data.du[f1]) and torch.equal(dv[f1], data.dv[f1])
    assert torch.equal(du[f0], mu_[f0]) and torch.equal(dv[f0], mv_[f0])
    assert torch.all(du[f2] == 0) and torch.all(dv[f2] == 0)


def test_auto_on_a_side_stream_sees_the_callers_prior_work(small):
    """AUTO forks work to a second stream of the device: it must wait for
    what the caller queued on its own stream just before the call (here the
    density, rewritten on that stream) and finish there. The result on a
    user stream equals the default-stream result for the same density."""
    import torch
    from paper_1510_05616_amd import near
    c, tx, ty, tc, dh, data = small
    k = torch.arange(near.N_BINS * near.CELL, device="cuda") // near.CELL
    bound = torch.where(k % 2 == 0, 1e-3, 10.0).float()
    blob = _auto_blob(_rand_params(5), bound, torch.full_like(bound, 10.0))
    sF = (data.frame[:, 6] / (4 * math.pi) * data.frame[:, 7])
    thr = 2e-3 * sF.max().item()
    fx0, fy0 = data.curves.fx.clone(), data.curves.fy.clone()
    ref = [torch.empty(data.n, dtype=torch.float64, device="cuda") for _ in range(2)]
    fr = torch.full((data.n,), -1, dtype=torch.int32, device="cuda")
    data.curves.fx.mul_(-2.0)
    data.curves.fy.mul_(0.5)
    data.correct(near.S2D_NEAR_AUTO, blob, thr, ref[0], ref[1], fr)
    torch.cuda.synchronize()
    assert bool((fr == 0).any()) and bool((fr == 1).any())
    data.curves.fx.copy_(fx0)
    data.curves.fy.copy_(fy0)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    du, dv = (torch.full((data.n,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(2))
    fb = torch.full((data.n,), -1, dtype=torch.int32, device="cuda")
    ws = near._empty(near.near_workspace_size(near.S2D_NEAR_AUTO, data.curves, data.trg, 8))
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        # queued on the side stream right before the call: a long chain of
        # kernels ending with the density the call must see
        for _ in range(20):
            data.curves.fx.mul_(1.0)
        data.curves.fx.mul_(-2.0)
        data.curves.fy.mul_(0.5)
        near.near_correct_eval(near.S2D_NEAR_AUTO, data.curves, data.trg, data.tc, 8, blob, thr, 1.0, du, dv, fb,
                               ws, stream=side)
    side.synchronize()
    data.curves.fx.copy_(fx0)
    data.curves.fy.copy_(fy0)
    torch.cuda.synchronize()
    assert torch.equal(fb, fr)
    assert torch.equal(du, ref[0]) and torch.equal(dv, ref[1])


def test_auto_per_curve_tolerances(small):
    """With curve_tol, each target is held to its own curve's tolerance: a
    zero tolerance sends every target of those curves to the quadrature, a
    huge one needs no correction, and the result matches the scalar
    threshold's on each group."""
    import torch
    from paper_1510_05616_amd import near
    c, tx, ty, tc, dh, data = small
    nt = near.N_BINS * near.CELL
    blob = _auto_blob(_rand_params(2), torch.full((nt,), 1e-3, device="cuda"), torch.full((nt,), 1.0, device="cuda"))
    tol = torch.where(torch.arange(c.n_curves, device="cuda") % 2 == 0, 0.0, 1e30).double()
    du, dv = (torch.empty(data.n, dtype=torch.float64, device="cuda") for _ in range(2))
    fb = torch.full((data.n,), -1, dtype=torch.int32, device="cuda")
    data.correct(near.S2D_NEAR_AUTO, blob, 0.5, du, dv, fb, curve_tol=tol)
    torch.cuda.synchronize()
    even = (data.tc % 2 == 0)
    low = data.b < near.B_MIN
    assert torch.all(fb[even] == 1) and torch.equal(du[even], data.du[even]) and torch.equal(dv[even], data.dv[even])
    odd = ~even & ~low
    assert odd.sum() > 100 and torch.all(fb[odd] == 2) and torch.all(du[odd] == 0)
    assert torch.all(fb[~even & low] == 1)


def test_calibration_matches_numpy(small):
    import torch
    from paper_1510_05616_amd import near
    c, tx, ty, tc, dh, data = small
    rng = np.random.default_rng(3)
    du = data.du + torch.as_tensor(rng.normal(size=data.n) * 1e-4, device="cuda")
    dv = data.dv + torch.as_tensor(rng.normal(size=data.n) * 1e-4, device="cuda")
    bound = torch.zeros(near.N_BINS * near.CELL, dtype=torch.float32, device="cuda")
    bound0, count = torch.zeros_like(bound), torch.zeros(near.N_BINS * near.CELL, dtype=torch.int32, device="cuda")
    near.near_calibrate(near.S2D_OP_SLP, data.frame, du, dv, data.du, data.dv, 1.0, near.N_BINS, near.BIN_LO,
                        near.BIN_W, near.B_MIN, 1.5, bound, bound0, count, count_margin=2.0)
    torch.cuda.synchronize()
    fr = data.frame.cpu().numpy()
    sF = fr[:, 6] / (4 * math.pi) * fr[:, 7]
    e = (np.hypot((du - data.du).cpu().numpy(), (dv - data.dv).cpu().numpy()) / sF).astype(np.float32)
    z = (np.hypot(data.du.cpu().numpy(), data.dv.cpu().numpy()) / sF).astype(np.float32)
    b = fr[:, 1].astype(np.float32)
    pos = np.floor((np.log10(b) - np.float32(near.BIN_LO)) / np.float32(near.BIN_W))
    ok = (b >= near.B_MIN) & (fr[:, 8] > 0) & (pos >= 0) & (pos < near.N_BINS)
    kk = near.table_index(fr[:, 1], fr[:, 0], fr[:, 19])[ok]
    nt = near.N_BINS * near.CELL
    be, bz, cn = np.zeros(nt), np.zeros(nt), np.zeros(nt, int)
    np.maximum.at(be, kk, e[ok])
    np.maximum.at(bz, kk, z[ok])
    np.add.at(cn, kk, 1)
    gb, gz, gc = bound.cpu().numpy(), bound0.cpu().numpy(), count.cpu().numpy()
    full = cn > 0
    assert np.array_equal(gc, cn)
    m = 1.5 * (1 + 2.0 / np.sqrt(np.maximum(cn, 1)))
    # past the midpoint between two nodes (the last |s| bin) the learned route is never admitted
    mid = (np.arange(nt) % near.CELL) // near.K_BINS == near.S_BINS - 1
    assert (full & mid).any() and (full & ~mid).any()
    assert np.allclose(gb[full & ~mid], (m * be)[full & ~mid], rtol=1e-6)
    assert np.allclose(gz[full], (m * bz)[full], rtol=1e-6)
    assert np.all(gb[~full | mid] == np.float32(3e38)) and np.all(gz[~full] == np.float32(3e38))


@pytest.fixture(scope="module")
def trained():
    """The learned correction trained on the GPU: 200,000 targets of the
    near-field workload, 200,000 steps of 1024, calibrated on 1,000,000
    held-out targets with margin 1.5 (1 + 2 / sqrt(targets per bin))."""
    from paper_1510_05616_amd import near
    tr = near.NearData(*synth.make_near_dataset(200000, seed=51)[:4], mu=1.0, upsample=8)
    params, hist = near.train(tr, steps=200000, batch=1024, lr=2e-3, log_every=25000)
    del tr
    va = near.NearData(*synth.make_near_dataset(1000000, seed=52)[:4], mu=1.0, upsample=8)
    blob, bound, bound0, count = near.calibrate(va, params, margin=1.5, count_margin=2.0)
    del va
    return params, hist, blob


@pytest.fixture(scope="module")
def held_out():
    from paper_1510_05616_amd import near
    return near.NearData(*synth.make_near_dataset(100000, seed=53)[:4], mu=1.0, upsample=8)


def test_training_gains_over_plain_trapezoid(trained, held_out):
    """The learned route's normalised error at targets within h/2 of their
    curve is far below the plain trapezoid rule's (the correction left out),
    and the loss fell by orders of magnitude."""
    import torch
    from paper_1510_05616_amd import near
    params, hist, blob = trained
    te = held_out
    print(f"losses {hist}", flush=True)
    assert hist[-1][1] < 1e-3 * hist[0][1]
    du = torch.empty(te.n, dtype=torch.float64, device="cuda")
    dv = torch.empty_like(du)
    te.correct(near.S2D_NEAR_MLP, blob, 0.0, du, dv)
    torch.cuda.synchronize()
    e_mlp = te.scaled_errors(du, dv).cpu().numpy()
    e_plain = te.scaled_errors(torch.zeros_like(du), torch.zeros_like(dv)).cpu().numpy()
    sel = ((te.b < 0.5) & (te.b >= near.B_MIN)).cpu().numpy()
    print(f"targets within h/2: plain median {np.median(e_plain[sel]):.2e} max {e_plain[sel].max():.2e}; "
          f"learned median {np.median(e_mlp[sel]):.2e} max {e_mlp[sel].max():.2e}", flush=True)
    assert np.median(e_mlp[sel]) < 1e-3 * np.median(e_plain[sel])


def test_auto_meets_1e5_on_held_out_targets(trained, held_out):
    """The contract of the learned correction on 100,000 held-out targets:
    AUTO with per-curve tolerances of 1e-5 times each curve's largest |u_8|
    stays within 1e-5 of the 8x upsampled quadrature in that normalised
    measure, and takes the learned route for most targets."""
    import torch
    from paper_1510_05616_amd import near
    params, hist, blob = trained
    te = held_out
    du = torch.empty(te.n, dtype=torch.float64, device="cuda")
    dv = torch.empty_like(du)
    fb = torch.zeros(te.n, dtype=torch.int32, device="cuda")
    te.correct(near.S2D_NEAR_AUTO, blob, 0.0, du, dv, fb, curve_tol=te.curve_tolerance(1e-5))
    torch.cuda.synchronize()
    E = te.scaled_errors(du, dv).max().item()
    frac = [(fb == k).double().mean().item() for k in range(3)]
    print(f"AUTO at 1e-5 per curve: E = {E:.2e}, learned/quadrature/none {frac}", flush=True)
    assert E <= 1e-5 and frac[0] > 0.5
