"""GPU parity of the wall upsampling (stokes2d_wall_upsample) and the
near-wall double-layer correction (near_wall_correct_eval, Delta = D_P - D_1
of the walls) with the FP64 oracle: oracle.near.wall_upsample per curve (numpy
FFT interpolation) and oracle.dlp on the oracle's refined and given walls.

Tolerances (FP64): the GPU takes each coefficient as a direct sum of N terms
and each fine value as a sum of N/2 terms, where the oracle uses FFTs; both
round at about sqrt(N) eps relative to the largest term.  Values (nodes,
density) within 1e-12 of their array's largest magnitude; normals and
weights come from spectral derivatives, whose mode-k rounding error is
amplified by k, within 1e-11 at N up to 16,000, and both sides are also
held to the closed-form wall.  Delta is linear in the fine normals and
weights; at targets a fraction of a spacing from the wall its terms exceed the
result, so it inherits their 1e-11 (measured about 3e-12 against the largest
|D_P|, E of the paper's definition for the corrected field)."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL_VAL, TOL_DER, TOL_DELTA = 1e-12, 1e-11, 1e-11
NAMES = ("x", "y", "nx", "ny", "w", "fx", "fy")


@pytest.fixture(scope="module", autouse=True)
def device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1510_05616_amd as s2d
    s2d.stokes2d_init(0)
    yield


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _oracle_upsample(walls, d, P):
    from oracle import near as onear
    outs = [[] for _ in NAMES]
    for c in range(walls.n_curves):
        s = slice(walls.curve_off[c], walls.curve_off[c + 1])
        r = onear.wall_upsample(walls.x[s], walls.y[s], walls.nx[s], walls.ny[s], walls.fx[s], walls.fy[s], d, P)
        for o, a in zip(outs, r):
            o.append(a)
    return [np.concatenate(o) for o in outs]


def _gpu_upsample(walls, d, P):
    from paper_1510_05616_amd import Curves
    from paper_1510_05616_amd.near import stokes2d_wall_upsample
    f = stokes2d_wall_upsample(Curves(walls), d, P)
    import torch
    torch.cuda.synchronize()
    return [getattr(f, k).cpu().numpy() for k in NAMES], f.curve_off.cpu().numpy()


def _mixed_walls(sizes, seed):
    # channels of period 2 pi with n nodes per wall, white-noise densities
    # (every mode present, the Nyquist one included)
    rng = np.random.default_rng(seed)
    parts = []
    for n in sizes:
        w, _, d = synth.make_channel(n, 4)
        for c in range(2):
            s = slice(w.curve_off[c], w.curve_off[c + 1])
            parts.append((w.x[s], w.y[s], w.nx[s], w.ny[s], w.w[s], w.kappa[s], rng.standard_normal(n),
                          rng.standard_normal(n)))
    return synth.concat_curves(parts), d


def _check_upsample(walls, d, P, tag):
    g, off = _gpu_upsample(walls, d, P)
    o = _oracle_upsample(walls, d, P)
    assert np.array_equal(off, P * walls.curve_off)
    errs = {k: _rel(a, b) for k, a, b in zip(NAMES, g, o)}
    print(f"{tag} P={P} {errs}", flush=True)
    for k in NAMES:
        assert errs[k] <= (TOL_DER if k in ("nx", "ny", "w") else TOL_VAL), (k, errs)


@pytest.mark.parametrize("P", [1, 3, 8])
def test_upsample_ragged_curves(P):
    # curve sizes 4 .. 510 so that waves straddle curves (the vector-load
    # path) and lie inside one (the scalar-load path)
    walls, d = _mixed_walls((4, 6, 10, 64, 100, 510), seed=P)
    _check_upsample(walls, d, P, "ragged")


@pytest.mark.parametrize("cfg,profile", [(2, "sin1"), (3, "sin13")])
def test_upsample_config_walls(cfg, profile):
    prob = synth.make_config(cfg)
    P = 8
    _check_upsample(prob.wall, prob.d, P, f"config{cfg}")
    # the GPU's refined walls lie on the closed-form walls y = +-h(x)
    (x, y, nx, ny, w, _, _), off = _gpu_upsample(prob.wall, prob.d, P)
    h, hp, _ = synth.wall_profile(profile)
    sq = np.sqrt(1 + hp(x) ** 2)
    for c in range(prob.wall.n_curves):
        s = slice(off[c], off[c + 1])
        sg = np.sign(y[s].mean())
        M = s.stop - s.start
        errs = (np.abs(y[s] - sg * h(x[s])).max(), np.abs(nx[s] + hp(x[s]) / sq[s]).max(),
                np.abs(ny[s] - sg / sq[s]).max(), np.abs(w[s] / (prob.d / M) - sq[s]).max())
        print(f"config{cfg} curve {c} closed-form errors y, nx, ny, w {errs}", flush=True)
        assert max(errs) <= TOL_DER, errs


def test_upsample_invalid_curves_nan():
    # an odd curve and a 2-node curve come out NaN, their neighbours exact
    walls, d = _mixed_walls((8, 16), seed=4)
    x = walls
    odd = synth.make_channel(7, 4)[0]
    parts = []
    for cs, c in ((x, 0), (odd, 0), (x, 1), (x, 2)):
        s = slice(cs.curve_off[c], cs.curve_off[c + 1])
        parts.append(tuple(getattr(cs, k)[s] for k in ("x", "y", "nx", "ny", "w", "kappa", "fx", "fy")))
    s = slice(x.curve_off[3], x.curve_off[3] + 2)
    parts.append(tuple(getattr(x, k)[s] for k in ("x", "y", "nx", "ny", "w", "kappa", "fx", "fy")))
    walls2 = synth.concat_curves(parts)
    P = 4
    g, _ = _gpu_upsample(walls2, d, P)
    off = P * walls2.curve_off
    good = synth.concat_curves([parts[0], parts[2], parts[3]])
    o = _oracle_upsample(good, d, P)
    for k, a, b in zip(NAMES, g, o):
        assert np.all(np.isnan(a[off[1]:off[2]])) and np.all(np.isnan(a[off[4]:off[5]])), k
        keep = np.concatenate([a[off[0]:off[1]], a[off[2]:off[4]]])
        assert _rel(keep, b) <= TOL_DER, k


def _walls_with_density(prob, seed):
    # smooth densities on the walls (the wall double-layer density is smooth)
    return synth.wall_densities(prob.wall, seed)


def _oracle_delta(walls, d, P, tx, ty, img):
    import oracle
    f = _oracle_upsample(walls, d, P)
    fine = synth.concat_curves([(f[0], f[1], f[2], f[3], f[4], np.zeros_like(f[0]), f[5], f[6])])
    uP, vP = oracle.dlp(fine, tx, ty, None, None, d, img[0], img[1])
    u1, v1 = oracle.dlp(walls, tx, ty, None, None, d, img[0], img[1])
    return uP - u1, vP - v1, np.hypot(uP, vP).max()


def _gpu_delta(walls, d, P, tx, ty, img, accumulate_onto=None):
    import torch
    from paper_1510_05616_amd import Curves, Targets
    from paper_1510_05616_amd.near import near_wall_correct_eval
    f64 = dict(dtype=torch.float64, device="cuda")
    n = tx.shape[0]
    if accumulate_onto is None:
        du, dv = torch.zeros(n, **f64), torch.zeros(n, **f64)
    else:
        du, dv = (torch.as_tensor(a, **f64).clone() for a in accumulate_onto)
    near_wall_correct_eval(Curves(walls), Targets(tx, ty), d, img[0], img[1], P, du, dv,
                           accumulate=0 if accumulate_onto is None else 1)
    torch.cuda.synchronize()
    return du.cpu().numpy(), dv.cpu().numpy()


@pytest.mark.parametrize("img", [(-1, 1), (0, 0)])
def test_delta_config2(img):
    prob = synth.make_config(2)
    walls = _walls_with_density(prob, 11)
    tx, ty = synth.near_wall_points(walls, 1001, seed=12)
    P = 8
    du, dv = _gpu_delta(walls, prob.d, P, tx, ty, img)
    ou, ov, scale = _oracle_delta(walls, prob.d, P, tx, ty, img)
    err = max(np.abs(du - ou).max(), np.abs(dv - ov).max()) / scale
    print(f"config2 img={img} Delta E {err:.2e}, max|Delta|/max|D_P| "
          f"{max(np.abs(ou).max(), np.abs(ov).max()) / scale:.2e}", flush=True)
    assert err <= TOL_DELTA


def test_delta_config3_sampled():
    # the 32,000-node channel refined to 256,000 nodes: the GPU at 20,000
    # near-wall points, the oracle at a seeded sample of 200
    prob = synth.make_config(3)
    walls = _walls_with_density(prob, 13)
    tx, ty = synth.near_wall_points(walls, 20000, seed=14)
    P = 8
    du, dv = _gpu_delta(walls, prob.d, P, tx, ty, (-1, 1))
    idx = np.random.default_rng(15).choice(20000, 200, replace=False)
    ou, ov, scale = _oracle_delta(walls, prob.d, P, tx[idx], ty[idx], (-1, 1))
    err = max(np.abs(du[idx] - ou).max(), np.abs(dv[idx] - ov).max()) / scale
    print(f"config3 Delta E {err:.2e}", flush=True)
    assert err <= TOL_DELTA


def test_delta_accumulate_and_edges():
    import torch
    from paper_1510_05616_amd import Curves, Targets
    from paper_1510_05616_amd.near import near_wall_correct_eval
    prob = synth.make_config(1)
    walls = _walls_with_density(prob, 16)
    tx, ty = synth.near_wall_points(walls, 300, seed=17)
    du, dv = _gpu_delta(walls, prob.d, 4, tx, ty, (-1, 1))
    base = (np.full(300, 0.5), np.full(300, -2.0))
    au, av = _gpu_delta(walls, prob.d, 4, tx, ty, (-1, 1), accumulate_onto=base)
    assert np.array_equal(au, base[0] + du) and np.array_equal(av, base[1] + dv)
    # P = 1: the refined wall is the wall to one DFT round trip (and the
    # given weights to spectral differentiation): Delta is rounding
    u1, v1 = _gpu_delta(walls, prob.d, 1, tx, ty, (-1, 1))
    r1 = max(np.abs(u1).max(), np.abs(v1).max()) / max(np.abs(du).max(), np.abs(dv).max())
    print(f"P=1 Delta / P=4 Delta {r1:.2e}", flush=True)
    assert r1 <= 1e-10
    # no targets: a no-op; no walls: zero
    f64 = dict(dtype=torch.float64, device="cuda")
    z = torch.zeros(0, **f64)
    near_wall_correct_eval(Curves(walls), Targets(np.zeros(0), np.zeros(0)), prob.d, -1, 1, 4, z, z)
    e = Curves(synth.concat_curves([]))
    a, b = torch.ones(300, **f64), torch.ones(300, **f64)
    near_wall_correct_eval(e, Targets(tx, ty), prob.d, -1, 1, 4, a, b)
    torch.cuda.synchronize()
    assert torch.all(a == 0) and torch.all(b == 0)


# ---------------------------------------------------------------------------
# the learned route for the walls (features, network, AUTO)
# ---------------------------------------------------------------------------
def _wall_learning_set(n, seed):
    prob = synth.make_config(2)
    walls = synth.wall_densities(prob.wall, 31)
    tx, ty, tc = synth.near_wall_dataset(walls, n, seed)
    return walls, prob.d, tx, ty, tc


def _gpu_wall_features(walls, d, tx, ty, tc):
    import torch
    from paper_1510_05616_amd import Curves, Targets
    from paper_1510_05616_amd import near as pn
    n = tx.shape[0]
    cw = Curves(walls)
    dtab = torch.empty((walls.x.shape[0], pn.NDERIV), dtype=torch.float64, device="cuda")
    pn.near_derivs_eval(cw, dtab)
    X = torch.empty((n, pn.NFEAT), dtype=torch.float32, device="cuda")
    fr = torch.empty((n, pn.NFRAME), dtype=torch.float64, device="cuda")
    pn.near_wall_features_eval(cw, Targets(tx, ty), torch.as_tensor(tc, device="cuda"), d, dtab, X, fr)
    torch.cuda.synchronize()
    return X.cpu().numpy(), fr.cpu().numpy()


def _features_vs_oracle(walls, d, tx, ty, tc):
    from oracle import near as onear
    gx, gfr = _gpu_wall_features(walls, d, tx, ty, tc)
    ox, ofr, odd = onear.wall_features(walls, d, tx, ty, tc)
    err_x = np.abs(gx - ox.astype(np.float32)) / np.maximum(np.abs(ox), 1.0)
    err_f = np.abs(gfr[:, :9] - ofr).max()
    err_d = np.abs(gfr[:, 9:19] - odd.reshape(-1, 10)).max() / np.abs(odd).max()
    return err_x.max(), err_f, err_d


def test_wall_features_match_the_oracle():
    walls, d, tx, ty, tc = _wall_learning_set(3000, 33)
    # and targets across the period boundary of each wall
    h = walls.w[:2048].mean()
    tx = np.r_[tx, [-0.4 * h, d + 0.3 * h, 0.1 * h, d - 0.2 * h]]
    ty = np.r_[ty, [0.95, -0.97, 0.9, -0.9]]
    tc = np.r_[tc, [0, 1, 0, 1]].astype(np.int32)
    ex, ef, ed = _features_vs_oracle(walls, d, tx, ty, tc)
    print(f"wall features: max rel diff {ex:.2e}, frame {ef:.2e}, derivatives {ed:.2e}", flush=True)
    assert ex < 4e-7 and ef < 1e-12 and ed < 1e-11


def test_wall_features_interior_targets_and_large_walls():
    """The nearest-node search prunes by cells of wall nodes.  Targets deep in
    the channel (many cells pass the bound, so a lane scans every passing cell
    in order), and walls with more cells than the search's table holds (plain
    scan), match the oracle as the near-wall targets do."""
    rng = np.random.default_rng(37)
    walls, d, tx, ty, tc = _wall_learning_set(200, 38)
    m = 60
    tx = np.r_[tx, rng.uniform(0.0, d, m)]
    ty = np.r_[ty, rng.uniform(-0.6, 0.6, m)]
    tc = np.r_[tc, rng.integers(0, 2, m)].astype(np.int32)
    ex, ef, ed = _features_vs_oracle(walls, d, tx, ty, tc)
    print(f"interior targets: features {ex:.2e}, frame {ef:.2e}, derivatives {ed:.2e}", flush=True)
    assert ex < 4e-7 and ef < 1e-12 and ed < 1e-11
    big, _, dbig = synth.make_channel(66000, 4)        # 2 x 516 cells of 128: over the table
    big = synth.wall_densities(big, 39)
    bx, by, bc = synth.near_wall_dataset(big, 40, 40)
    bx = np.r_[bx, rng.uniform(0.0, dbig, 8)]
    by = np.r_[by, rng.uniform(-0.5, 0.5, 8)]
    bc = np.r_[bc, rng.integers(0, 2, 8)].astype(np.int32)
    ex, ef, ed = _features_vs_oracle(big, dbig, bx, by, bc)
    print(f"large walls: features {ex:.2e}, frame {ef:.2e}, derivatives {ed:.2e}", flush=True)
    # the offsets s, b are differences of coordinates of size ~d over the
    # spacing h ~ 1e-4: their rounding is about eps d / h ~ 1e-11
    assert ex < 4e-7 and ef < 1e-11 and ed < 1e-10


def test_wall_flat_part_matches_oracle():
    """The learned wall route with an all-zero network is the double layer's
    straight-line part alone (times the sign of the normal offset): FP64
    against the oracle's closed form."""
    import torch
    from oracle import near as onear
    from paper_1510_05616_amd import near as pn
    walls, d, tx, ty, tc = _wall_learning_set(4000, 41)
    data = pn.WallNearData(walls, d, tx, ty, tc, labels=False)
    ox, ofr, odd = onear.wall_features(walls, d, tx, ty, tc)
    flat = onear.flat_predict(ofr, odd, "dlp", P=8)
    fu, fv = onear.frame_to_velocity(flat, ofr, 1.0 / math.pi)
    zero = torch.zeros(pn.NPARAM, dtype=torch.float32, device="cuda")
    zero[14:28] = 1.0
    blob = torch.zeros(pn.near_mlp_blob_size(), dtype=torch.uint8, device="cuda")
    pn.near_mlp_pack(zero, None, 0, pn.BIN_LO, pn.BIN_W, blob)
    du = torch.empty(data.n, dtype=torch.float64, device="cuda")
    dv = torch.empty_like(du)
    data.correct(pn.S2D_NEAR_MLP, blob, 0.0, du, dv)
    torch.cuda.synchronize()
    err = np.hypot(du.cpu().numpy() - fu, dv.cpu().numpy() - fv).max() / np.hypot(fu, fv).max()
    print(f"wall straight-line part vs oracle: {err:.2e}", flush=True)
    assert err < 1e-12


def test_wall_auto_extremes_and_network_gain():
    import torch
    from paper_1510_05616_amd import near as pn
    walls, d, tx, ty, tc = _wall_learning_set(60000, 34)
    tr = pn.WallNearData(walls, d, tx, ty, tc)
    params, hist = pn.train(tr, steps=4000, batch=512, lr=3e-3, log_every=1000)
    print(f"losses {hist}", flush=True)
    assert hist[-1][1] < 0.2 * hist[0][1]
    va = pn.WallNearData(walls, d, *_wall_learning_set(10000, 35)[2:])
    blob, bound, bound0, count = pn.calibrate(va, params)
    te = pn.WallNearData(walls, d, *_wall_learning_set(10000, 36)[2:])
    du = torch.empty(te.n, dtype=torch.float64, device="cuda")
    dv = torch.empty_like(du)
    fb = torch.zeros(te.n, dtype=torch.int32, device="cuda")
    # the learned route gains over no correction near the walls
    te.correct(pn.S2D_NEAR_MLP, blob, 0.0, du, dv, fb)
    torch.cuda.synchronize()
    e_mlp = te.scaled_errors(du, dv).cpu().numpy()
    e_plain = te.scaled_errors(torch.zeros_like(du), torch.zeros_like(dv)).cpu().numpy()
    sel = ((te.b < 0.5) & (te.b >= pn.B_MIN)).cpu().numpy()
    print(f"walls, targets within h/2: plain median {np.median(e_plain[sel]):.2e}, learned median "
          f"{np.median(e_mlp[sel]):.2e} max {e_mlp[sel].max():.2e}", flush=True)
    assert np.median(e_mlp[sel]) < 1e-2 * np.median(e_plain[sel])
    assert torch.all(fb == 0)
    # AUTO: threshold 0 is the refined quadrature everywhere; a huge one no
    # correction beyond b_min; in between every target within the threshold
    te.correct(pn.S2D_NEAR_AUTO, blob, 0.0, du, dv, fb)
    torch.cuda.synchronize()
    assert torch.all(fb == 1)
    e = max((du - te.du).abs().max().item(), (dv - te.dv).abs().max().item())
    assert e <= 1e-12 * max(te.du.abs().max().item(), te.dv.abs().max().item()), e
    te.correct(pn.S2D_NEAR_AUTO, blob, 1e30, du, dv, fb)
    torch.cuda.synchronize()
    low = te.b < pn.B_MIN
    assert torch.all(fb[~low] == 2) and torch.all(du[~low] == 0) and torch.all(dv[~low] == 0)
    assert torch.all(fb[low] == 1)
    # per-wall tolerances: every target within its wall's tolerance, and the
    # learned route taken where its calibrated bound allows
    for rel in (1e-4, 1e-3):
        te.correct(pn.S2D_NEAR_AUTO, blob, 0.0, du, dv, fb, curve_tol=te.curve_tolerance(rel))
        torch.cuda.synchronize()
        E = te.scaled_errors(du, dv).max().item()
        used = [(fb == k).float().mean().item() for k in range(3)]
        print(f"walls AUTO at {rel:g} per wall: max normalised error {E:.2e}, learned/quadrature/none {used}",
              flush=True)
        assert E <= rel
    assert used[0] > 0.2
