"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/stokes2d.h, and rejects bad arguments
(before touching the device) with the documented status codes."""
import ctypes
from pathlib import Path
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"S2D_API\s+[\w\s\*]+?\b(\w+)\s*\(", txt)
    return names


@pytest.fixture(scope="module")
def L():
    import paper_1510_05616_amd as s2d
    return s2d.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "stokes2d_slp_eval" in names and "stokes2d_dlp_eval" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/ but not exported"


def test_version(L):
    import paper_1510_05616_amd as s2d
    assert s2d.stokes2d_version() >= 100


def _structs(n_src=8, n_trg=4, on=False):
    import paper_1510_05616_amd as s2d
    fake = ctypes.c_void_p(0x1000)          # never dereferenced: validation fails first
    cs = s2d._Curves(n_src, 1, fake, fake, fake, fake, fake, fake, fake, fake, fake)
    ts = s2d._Targets(n_trg, fake, fake, fake if on else None, fake if on else None)
    return cs, ts


def test_bad_arguments_return_einval(L):
    import paper_1510_05616_amd as s2d
    cs, ts = _structs()
    out = ctypes.c_void_p(0x2000)
    ws = ctypes.c_void_p(0x3000)
    by = ctypes.byref
    # bad mode
    assert L.stokes2d_slp_eval(7, by(cs), by(ts), 1.0, 0, 0, 1.0, out, out, 0, ws, 1 << 20, None) == s2d.S2D_EINVAL
    # NULL structs
    assert L.stokes2d_slp_eval(0, None, by(ts), 1.0, 0, 0, 1.0, out, out, 0, ws, 1 << 20, None) == s2d.S2D_EINVAL
    # img_lo > img_hi
    assert L.stokes2d_dlp_eval(0, by(cs), by(ts), 1.0, 1, 0, out, out, 0, ws, 1 << 20, None) == s2d.S2D_EINVAL
    # images without a period
    assert L.stokes2d_slp_eval(0, by(cs), by(ts), 0.0, -1, 1, 1.0, out, out, 0, ws, 1 << 20, None) == s2d.S2D_EINVAL
    assert L.stokes2d_slp_eval(0, by(cs), by(ts), float("nan"), -1, 1, 1.0, out, out, 0, ws, 1 << 20, None) == s2d.S2D_EINVAL
    # mu <= 0
    assert L.stokes2d_slp_eval(0, by(cs), by(ts), 1.0, 0, 0, 0.0, out, out, 0, ws, 1 << 20, None) == s2d.S2D_EINVAL
    # too many images
    assert L.stokes2d_slp_eval(0, by(cs), by(ts), 1.0, -65, 0, 1.0, out, out, 0, ws, 1 << 20, None) == s2d.S2D_EINVAL
    # on_curve without on_node
    ts2 = s2d._Targets(4, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), None)
    assert L.stokes2d_slp_eval(0, by(cs), by(ts2), 1.0, 0, 0, 1.0, out, out, 0, ws, 1 << 20, None) == s2d.S2D_EINVAL
    # DLP with on-curve targets but no curvature
    cs2, ts3 = _structs(on=True)
    cs2.kappa = None
    assert L.stokes2d_dlp_eval(0, by(cs2), by(ts3), 1.0, 0, 0, out, out, 0, ws, 1 << 20, None) == s2d.S2D_EINVAL
    # negative sizes
    cs3, _ = _structs(n_src=-1)
    assert L.stokes2d_slp_eval(0, by(cs3), by(ts), 1.0, 0, 0, 1.0, out, out, 0, ws, 1 << 20, None) == s2d.S2D_EINVAL
    assert "n_nodes" in s2d.stokes2d_last_error()


def test_workspace_size_is_zero_on_bad_arguments(L):
    import paper_1510_05616_amd as s2d
    cs, ts = _structs()
    assert L.stokes2d_workspace_size(5, 0, ctypes.byref(cs), ctypes.byref(ts)) == 0
    assert L.stokes2d_workspace_size(0, 0, ctypes.byref(cs), ctypes.byref(ts)) > 0


def test_workspace_grows_with_problem(L):
    import paper_1510_05616_amd as s2d
    small = _structs(100, 100)
    big = _structs(100000, 100000)
    for op in (0, 1):
        for mode in (0, 1):
            a = L.stokes2d_workspace_size(op, mode, ctypes.byref(small[0]), ctypes.byref(small[1]))
            b = L.stokes2d_workspace_size(op, mode, ctypes.byref(big[0]), ctypes.byref(big[1]))
            assert 0 < a < b


def test_batch_tuned_is_host_only_and_reports_the_default(L, tmp_path, monkeypatch):
    import paper_1510_05616_amd as s2d
    monkeypatch.setenv("S2D_TUNE_CACHE", str(tmp_path / "absent.json"))
    t = ctypes.c_int32()
    by = ctypes.byref
    assert L.stokes2d_batch_tuned(1, 0, None, None, by(t), by(t)) == s2d.S2D_EINVAL
    assert L.stokes2d_batch_tuned(3, 0, None, by(t), by(t), by(t)) == s2d.S2D_EINVAL
    assert L.stokes2d_batch_tuned(1, -1, None, by(t), by(t), by(t)) == s2d.S2D_EINVAL
    for mode in (s2d.S2D_FP64, s2d.S2D_FP32C):
        shape = s2d.stokes2d_batch_tuned(mode, [])
        assert shape["tuned"] is False
        assert shape["targets_per_lane"] in (1, 2, 4)
        assert shape["superblocks_per_split"] > 0 and shape["waves_per_cu"] > 0


def test_pressure_and_traction_argument_checks(L):
    import paper_1510_05616_amd as s2d
    cs, ts = _structs()
    cs_on, ts_on = _structs(on=True)
    out = ctypes.c_void_p(0x2000)
    ws = ctypes.c_void_p(0x3000)
    by = ctypes.byref
    # on-curve targets are not supported for the singular kernels
    assert L.stokes2d_slp_pressure_eval(0, by(cs), by(ts_on), 1.0, 0, 0, out, 0, ws, 1 << 20, None) == s2d.S2D_EINVAL
    assert "free targets" in s2d.stokes2d_last_error()
    # double-layer pressure needs mu > 0
    assert L.stokes2d_dlp_pressure_eval(0, by(cs), by(ts), 1.0, 0, 0, 0.0, out, 0, ws, 1 << 20, None) == s2d.S2D_EINVAL
    # traction needs the target normals
    assert L.stokes2d_slp_traction_eval(0, by(cs), by(ts), None, out, 1.0, 0, 0, out, out, 0, ws, 1 << 20,
                                        None) == s2d.S2D_EINVAL
    # unknown op code
    assert L.stokes2d_workspace_size(5, 0, by(cs), by(ts)) == 0
    for op in (s2d.S2D_OP_SLP_PRESSURE, s2d.S2D_OP_DLP_PRESSURE, s2d.S2D_OP_SLP_TRACTION):
        assert L.stokes2d_workspace_size(op, 1, by(cs), by(ts)) > 0
        assert L.stokes2d_workspace_size(op, 1, by(cs_on), by(ts_on)) == 0


def test_cell_argument_checks(L):
    import paper_1510_05616_amd as s2d
    from paper_1510_05616_amd import cell as pc
    pc._bind()
    fake = ctypes.c_void_p(0x1000)
    walls = s2d._Curves(64, 2, fake, fake, fake, fake, fake, fake, fake, fake, fake)
    good = pc._Cell(walls, 8, fake, 0.0, 32, 3.0, 0.0, 6.0, 6.0, 0.7)
    by = ctypes.byref
    assert L.stokes2d_cell_workspace_size(None) == 0
    assert L.stokes2d_cell_workspace_size(by(good)) > (2 * 64) ** 2 * 8
    for field, value in (("n_side", 0), ("n_proxy", 0), ("d", 0.0), ("mu", -1.0), ("proxy_r", 0.0)):
        bad = pc._Cell(walls, 8, fake, 0.0, 32, 3.0, 0.0, 6.0, 6.0, 0.7)
        setattr(bad, field, value)
        assert L.stokes2d_cell_workspace_size(by(bad)) == 0, field
        assert L.stokes2d_cell_factor(by(bad), 1e-8, fake, 1 << 30, None) == s2d.S2D_EINVAL, field
    big = s2d._Curves(65537, 2, fake, fake, fake, fake, fake, fake, fake, fake, fake)
    assert L.stokes2d_cell_workspace_size(by(pc._Cell(big, 8, fake, 0.0, 32, 3.0, 0.0, 6.0, 6.0, 0.7))) == 0
    assert L.stokes2d_cell_factor(by(pc._Cell(big, 8, fake, 0.0, 32, 3.0, 0.0, 6.0, 6.0, 0.7)), 1e-8, fake,
                                  1 << 40, None) == s2d.S2D_EINVAL
    assert "65536" in s2d.stokes2d_last_error()
    # LU panel width: 0 (widest), 1 .. widest; C and X within 2^30 elements
    for panel, ok in ((0, True), (1, True), (128, True), (128 + 1, False), (-1, False)):
        c = pc._Cell(walls, 8, fake, 0.0, 32, 3.0, 0.0, 6.0, 6.0, 0.7, panel)
        assert (L.stokes2d_cell_workspace_size(by(c)) > 0) == ok, panel
    wide = s2d._Curves(65536, 2, fake, fake, fake, fake, fake, fake, fake, fake, fake)
    for K, M, ok in ((8, 32, True), (4096, 32, False), (8, 8192, False)):
        c = pc._Cell(wide, K, fake, 0.0, M, 3.0, 0.0, 6.0, 6.0, 0.7)
        assert (L.stokes2d_cell_workspace_size(by(c)) > 0) == ok, (K, M)
    nok = s2d._Curves(64, 2, fake, fake, fake, fake, fake, fake, None, fake, fake)     # no kappa
    assert L.stokes2d_cell_workspace_size(by(pc._Cell(nok, 8, fake, 0.0, 32, 3.0, 0.0, 6.0, 6.0, 0.7))) == 0
    assert L.stokes2d_cell_factor(by(good), 1.5, fake, 1 << 30, None) == s2d.S2D_EINVAL     # rcond
    assert L.stokes2d_cell_factor(by(good), 1e-8, fake, 16, None) == s2d.S2D_EWORKSPACE
    assert L.stokes2d_cell_solve(by(good), None, fake, fake, fake, fake, 1 << 30, None) == s2d.S2D_EINVAL


def _cell_layout_bytes(N, K, M, panel):
    """The cell workspace written out in 64-bit integers: each block rounded
    up to 256 bytes, in the order A, B, X, C, S, U, Vt, sv, E, P, y, rr,
    pivots, permutation, the two sweeps' tiles (512 doubles per row), the
    sweep scratch vector, LU status per panel + the SVD's."""
    n, nc, mr = 2 * N, 2 * M, 4 * K
    r = min(mr, nc)
    sizes = [n * n * 8, n * nc * 8, n * nc * 8, mr * n * 8, mr * nc * 8, mr * r * 8, r * nc * 8, r * 8, r * 8,
             nc * mr * 8, n * 8, mr * 8, n * 4, n * 4, n * 512 * 8, n * 512 * 8, n * 8, (-(-n // panel) + 1) * 4]
    return sum(-(-b // 256) * 256 for b in sizes)


@pytest.mark.parametrize("N,panel", [(32128, 16640), (65536, 8192), (4000, 8000), (23171, 23040)])
def test_cell_workspace_at_the_largest_walls(L, N, panel):
    """The workspace of cells whose dense block has more than 2^31 elements
    (2 x 16,064 and 2 x 32,768 wall nodes): sizes and offsets in 64 bits, and
    the widest LU panel is the one the plan check below uses."""
    import paper_1510_05616_amd as s2d
    from paper_1510_05616_amd import cell as pc
    pc._bind()
    fake = ctypes.c_void_p(0x1000)
    walls = s2d._Curves(N, 2, fake, fake, fake, fake, fake, fake, fake, fake, fake)
    c = pc._Cell(walls, 32, fake, 0.0, 128, 3.0, 0.0, 6.0, 6.0, 0.7)
    assert L.stokes2d_cell_workspace_size(ctypes.byref(c)) == _cell_layout_bytes(N, 32, 128, panel)
    c.lu_panel = panel
    assert L.stokes2d_cell_workspace_size(ctypes.byref(c)) == _cell_layout_bytes(N, 32, 128, panel)
    c.lu_panel = panel + 1
    assert L.stokes2d_cell_workspace_size(ctypes.byref(c)) == 0


@pytest.fixture(scope="module")
def lu_check(tmp_path_factory):
    """The host check of the blocked LU schedule, compiled with g++."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = tmp_path_factory.mktemp("lu") / "lu_plan_check"
    src = Path(__file__).with_name("lu_plan_check.cpp")
    subprocess.run([gxx, "-O2", "-std=c++17", "-Wall", "-Werror", "-o", str(exe), str(src)], check=True)

    def run(*args):
        p = subprocess.run([str(exe), *map(str, args)], capture_output=True, text=True, timeout=120)
        assert p.returncode == 0 and p.stdout.startswith("OK"), p.stdout + p.stderr
        return p.stdout
    return run


@pytest.mark.parametrize("n,S,nrhs", [(64256, 16640, 256), (64256, 8192, 1), (131072, 8192, 256),
                                       (131072, 8192, 1), (46340, 8192, 1)])
def test_lu_schedule_offsets_at_full_size(lu_check, n, S, nrhs):
    """Every call of the factor and solve schedules of a 64,256^2 and a
    131,072^2 system (config-3 and the largest walls) addresses at most 2^30
    elements from its operand's base and stays inside its buffer."""
    out = lu_check("check", n, 1 << 30, 0, S, nrhs)
    if n > 46340:
        assert int(out.split(" W ")[1].split()[0]) < n          # several panels


@pytest.mark.parametrize("n,lim,W,S,nrhs,seed", [(60, 1000, 0, 7, 1, 1), (60, 1000, 0, 7, 5, 2),
                                                 (97, 2500, 0, 9, 3, 3), (200, 1 << 31, 0, 50, 2, 4),
                                                 (200, 1 << 31, 64, 50, 2, 5), (150, 4000, 13, 11, 1, 6),
                                                 (301, 40000, 0, 40, 4, 7), (1, 1, 0, 1, 1, 8)])
def test_lu_schedule_solves(lu_check, n, lim, W, S, nrhs, seed):
    """The schedule at small bounds (narrow panels, chunked operands) run with
    plain loops: the same pivots and solution as unblocked elimination."""
    lu_check("run", n, lim, W, S, nrhs, seed)


def test_wall_argument_checks(L):
    import paper_1510_05616_amd as s2d
    from paper_1510_05616_amd import near as pn
    pn._bind()
    fake = ctypes.c_void_p(0x1000)
    by = ctypes.byref
    walls = s2d._Curves(64, 2, fake, fake, fake, fake, fake, None, None, fake, fake)    # w, kappa unused
    _, ts = _structs()
    _, ts_on = _structs(on=True)
    o = [fake] * 8
    assert L.stokes2d_wall_upsample_workspace_size(None, 8) == 0
    assert L.stokes2d_wall_upsample_workspace_size(by(walls), 0) == 0
    assert L.stokes2d_wall_upsample_workspace_size(by(walls), 8) >= 64 * 64
    assert L.near_wall_workspace_size(0, by(walls), by(ts), 8) > 8 * 64 * 7 * 8
    assert L.near_wall_workspace_size(0, by(walls), by(ts), 33) == 0
    assert L.near_wall_workspace_size(3, by(walls), by(ts), 8) == 0
    assert L.near_wall_workspace_size(1, by(walls), by(ts), 8) > 0
    # upsample factor, period, missing normals, missing outputs
    assert L.stokes2d_wall_upsample(by(walls), 1.0, 0, *o, fake, 1 << 20, None) == s2d.S2D_EINVAL
    assert L.stokes2d_wall_upsample(by(walls), 0.0, 4, *o, fake, 1 << 20, None) == s2d.S2D_EINVAL
    non = s2d._Curves(64, 2, fake, fake, fake, None, fake, None, None, fake, fake)
    assert L.stokes2d_wall_upsample(by(non), 1.0, 4, *o, fake, 1 << 20, None) == s2d.S2D_EINVAL
    assert L.stokes2d_wall_upsample(by(walls), 1.0, 4, None, *o[1:], fake, 1 << 20, None) == s2d.S2D_EINVAL
    none = s2d._Curves(64, 0, fake, fake, fake, fake, fake, None, None, fake, fake)     # nodes but no curves
    assert L.stokes2d_wall_upsample(by(none), 1.0, 4, *o, fake, 1 << 20, None) == s2d.S2D_EINVAL
    # the correction: free targets only, outputs, images, method, network
    def corr(method, trg, lo, hi, du, mlp=None, tc=fake):
        return L.near_wall_correct_eval(method, by(walls), by(trg), tc, 1.0, lo, hi, 8, mlp, 0.0, None, du, fake,
                                        None, 0, fake, 1 << 30, None)
    assert corr(0, ts_on, -1, 1, fake) == s2d.S2D_EINVAL
    assert corr(0, ts, -1, 1, None) == s2d.S2D_EINVAL
    assert corr(0, ts, 1, -1, fake) == s2d.S2D_EINVAL
    assert corr(5, ts, -1, 1, fake) == s2d.S2D_EINVAL
    assert corr(1, ts, -1, 1, fake, mlp=None) == s2d.S2D_EINVAL            # MLP needs the network
    assert corr(2, ts, -1, 1, fake, mlp=fake, tc=None) == s2d.S2D_EINVAL   # and trg_curve
    assert corr(1, ts, -1, 1, fake, mlp=fake) == s2d.S2D_EINVAL            # and the walls' w, kappa
    assert L.near_wall_features_eval(by(walls), by(ts), None, 1.0, fake, fake, fake, None) == s2d.S2D_EINVAL
    assert L.near_wall_features_eval(by(walls), by(ts), fake, 1.0, None, fake, fake, None) == s2d.S2D_EINVAL


def test_learned_near_argument_checks(L):
    """Argument checks of the learned correction's entry points (all fail
    before any device call)."""
    import paper_1510_05616_amd as s2d
    from paper_1510_05616_amd import near as pn
    pn._bind()
    fake = ctypes.c_void_p(0x1000)
    odd = ctypes.c_void_p(0x1004)
    by = ctypes.byref
    small = s2d._Curves(200, 2, fake, fake, fake, fake, fake, fake, fake, fake, fake)
    big = s2d._Curves(4000, 2, fake, fake, fake, fake, fake, fake, fake, fake, fake)
    assert L.near_derivs_workspace_size(by(small)) == 256
    need = L.near_derivs_workspace_size(by(big))
    assert need >= 4000 * 6 * 8
    assert L.near_derivs_eval(by(big), fake, fake, need - 256, None) == s2d.S2D_EWORKSPACE
    assert L.near_derivs_eval(by(big), None, fake, need, None) == s2d.S2D_EINVAL
    nof = s2d._Curves(200, 2, fake, fake, fake, fake, fake, fake, fake, None, fake)     # no fx
    assert L.near_derivs_eval(by(nof), fake, None, 0, None) == s2d.S2D_EINVAL
    # training records: op, weight gain, mu, upsample, NULL arrays
    tt = lambda op=0, n=10, gain=1.0, mu=1.0, P=8, cs=fake: L.near_train_targets(
        op, n, fake, fake, fake, fake, 2, fake, fake, mu, P, gain, cs, fake, None)
    assert tt(op=2) == s2d.S2D_EINVAL and tt(op=4) == s2d.S2D_EINVAL
    assert tt(gain=0.0) == s2d.S2D_EINVAL and tt(gain=float("nan")) == s2d.S2D_EINVAL
    assert tt(mu=0.0) == s2d.S2D_EINVAL and tt(P=0) == s2d.S2D_EINVAL and tt(n=-1) == s2d.S2D_EINVAL
    assert tt(cs=None) == s2d.S2D_EINVAL
    # calibration: bins, margin, b_min
    cal = lambda nb=64, w=0.03, bmin=0.05, margin=1.25, cm=2.0, op=0: L.near_calibrate(
        op, 10, fake, fake, fake, fake, fake, 1.0, nb, -1.3, w, bmin, margin, cm, fake, fake, fake, None)
    assert cal(nb=0) == s2d.S2D_EINVAL and cal(nb=65) == s2d.S2D_EINVAL
    assert cal(w=0.0) == s2d.S2D_EINVAL and cal(margin=0.9) == s2d.S2D_EINVAL
    assert cal(cm=-1.0) == s2d.S2D_EINVAL and cal(cm=float("inf")) == s2d.S2D_EINVAL
    assert cal(bmin=-1.0) == s2d.S2D_EINVAL and cal(op=3) == s2d.S2D_EINVAL
    # packing: bins, bounds, b_min, upsample, blob alignment
    pk = lambda nb=64, bound=fake, bmin=0.05, P=8, blob=fake: L.near_mlp_pack(
        fake, bound, None, nb, -1.3, 0.03, bmin, P, blob, None)
    assert pk(nb=65) == s2d.S2D_EINVAL and pk(bound=None) == s2d.S2D_EINVAL
    assert pk(bmin=-0.1) == s2d.S2D_EINVAL and pk(P=33) == s2d.S2D_EINVAL
    assert pk(blob=odd) == s2d.S2D_EINVAL
    assert L.near_feature_stats(10, fake, None, None) == s2d.S2D_EINVAL
    assert L.near_feature_stats(-1, fake, fake, None) == s2d.S2D_EINVAL
    assert L.near_mlp_blob_size() >= 4 * (64 * 8 + 2 * 64 * 32 + 32 * 32)


def test_vesicle_argument_checks(L):
    import paper_1510_05616_amd as s2d
    from paper_1510_05616_amd import vesicle as pv
    pv._bind()
    fake = ctypes.c_void_p(0x1000)
    by = ctypes.byref
    good = pv.params(dt=1e-3)
    assert L.ves_step_workspace_size(96, 1, by(good)) > 0
    assert L.ves_step_workspace_size(96, 1, None) == 0
    for field, value in (("dt", 0.0), ("mu", -1.0), ("restart", 0), ("restart", 129), ("max_iter", 0),
                         ("mode", 3), ("kappa_b", -1.0), ("precond", 1), ("nmax", 600)):
        bad = pv.params(dt=1e-3)
        setattr(bad, field, value)
        assert L.ves_step_solve(96, 1, fake, fake, fake, by(bad), fake, None, None, fake, 1 << 30,
                                None) == s2d.S2D_EINVAL, field
    img = pv.params(dt=1e-3, img_lo=-1, img_hi=1)          # images need d > 0
    assert L.ves_step_solve(96, 1, fake, fake, fake, by(img), fake, None, None, fake, 1 << 30,
                            None) == s2d.S2D_EINVAL
    half = pv.params(dt=1e-3)
    half.u_resp_x = 0x2000                                  # u_resp comes in pairs
    assert L.ves_step_apply(96, 1, fake, fake, fake, by(half), fake, fake, None, fake, 1 << 30,
                            None) == s2d.S2D_EINVAL
    assert L.ves_forces(96, 1, fake, fake, fake, None, 1.0, fake, None, None, None, None) == s2d.S2D_EINVAL
    assert L.ves_area_correct(96, 1, fake, fake, fake, None, None) == s2d.S2D_EINVAL
    assert L.ves_measure(96, 0, fake, fake, fake, fake, fake, None) == s2d.S2D_EINVAL
