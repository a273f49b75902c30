"""Benchmark of the hot path: free-space Stokes single layer (1,000 vesicles x
96 nodes) plus double layer (2 walls x 16,000 nodes) with the +-d near images,
at every vesicle, wall and side target of the 128k-node periodic channel
(128,064 targets x 128,000 sources x 3 images = 4.918e10 pair evaluations per
step), on one MI355X.

A step is one SLP evaluation followed by one DLP evaluation accumulated into
the same velocity, inputs already resident in HBM.  `value` is FP32C
pair-evals/s; the FP64 run is reported in the same line under "fp64".
The dominant kernel (the single-layer pair kernel) is timed with HIP events
recorded by the library around its launches on the benchmark stream;
`roofline` prices it at 19 algorithmic flops per pair against the FP32 (or
FP64) vector peak.  `cpu_baseline` times the FP64 oracle on a seeded sample of
targets of the same workload on the host cores (65,536 targets by default,
about 10 s on 16 threads).

Further sections, each with its own timing, parity against the oracle on a
sample and, where it has one, roofline: pressures and traction at 128,064
free points; the walls' near-field correction; the vesicle time step of the
1,000 vesicles; Algorithm 1 in the channel (cell factored once); the
periodization cell at the paper's 4,000 nodes per wall; the learned near
field; the batched 256-instance graph launch.  --<section> 0 skips one.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--cpu-sample T]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 19          # algorithmic flops per pair, SLP and DLP alike
PEAK = {"f32": 157.3e12, "f64": 78.6e12}


PAIR_SOURCES = ("paper_1510_05616_amd/csrc/pair_impl.h", "paper_1510_05616_amd/csrc/pair.hip",
                "paper_1510_05616_amd/csrc/s2d_internal.h", "paper_1510_05616_amd/csrc/plan.hip")
SLP_KERNEL = {"f32": "pair_kernel<0,1,3>", "f64": "pair_kernel<0,0,3>"}
PROFILE = "profiles/pair_kernels_config3.md"
VALU_PROFILE = "profiles/pair_kernels_valu_config3.md"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pair_source_sha1():
    h = hashlib.sha1()
    for f in PAIR_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` recorded in the committed rocprofv3
    summary, or None when the pair-kernel sources changed since it was taken."""
    try:
        txt = open(os.path.join(ROOT, PROFILE)).read()
    except OSError:
        return None
    m = re.search(r"pair-kernel source sha1: ([0-9a-f]{40})", txt)
    if not m or m.group(1) != pair_source_sha1():
        return None
    m = re.search(r"traffic_bytes " + re.escape(kernel) + r" (\d+)", txt)
    return int(m.group(1)) if m else None


def measured_valu(kernel):
    """VALU issue counters of `kernel` from the committed rocprofv3 summary
    (VALUBusy %, share of SIMD quad-cycles issuing VALU work, share issuing two
    VALU instructions, clock), or None when the pair-kernel sources changed
    since they were taken."""
    try:
        txt = open(os.path.join(ROOT, VALU_PROFILE)).read()
    except OSError:
        return None
    m = re.search(r"pair-kernel source sha1: ([0-9a-f]{40})", txt)
    if not m or m.group(1) != pair_source_sha1():
        return None
    m = re.search(r"valu_busy " + re.escape(kernel) + r" ([\d.]+) issuing ([\d.]+) dual ([\d.]+) ghz ([\d.]+)"
                  r" valu_per_pair ([\d.]+)", txt)
    if not m:
        return None
    return {"valu_busy_pct": float(m.group(1)), "valu_issuing_pct": float(m.group(2)),
            "dual_issue_pct": float(m.group(3)), "clock_ghz": float(m.group(4)),
            "valu_per_pair": float(m.group(5)), "source": VALU_PROFILE}


def issue_probe(blocks=2048, iters=20000, reps=3):
    """The VALU issue ceiling: stokes2d_valu_probe's rate (wave-instructions
    per second, 8 waves per SIMD of independent FMA chains) for FP32 with
    VGPR operands, FP32 with an SGPR operand, and FP64, timed with HIP events
    on the launch stream."""
    import ctypes
    import torch
    import paper_1510_05616_amd as s2d
    L = s2d.lib()
    L.stokes2d_valu_probe.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    L.stokes2d_valu_probe.restype = ctypes.c_int
    sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    out = {}
    for form, name in ((0, "f32_vgpr"), (1, "f32_sgpr"), (2, "f64")):
        best = None
        for _ in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(st)
            rc = L.stokes2d_valu_probe(form, blocks, iters, ctypes.c_void_p(sink.data_ptr()),
                                       ctypes.c_void_p(st.cuda_stream))
            b.record(st)
            assert rc == 0, s2d.stokes2d_last_error()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
        winstr = blocks * 4 * iters * 8                      # wave-instructions (4 waves per block)
        out[name] = {"wave_instr_per_s": winstr / (best * 1e-3), "ms": best,
                     "tflops": 2 * 64 * winstr / (best * 1e-3) / 1e12}
    return out


def copy_probe():
    """A device-to-device copy of exactly 1 GiB, three times (for calibrating
    the FETCH_SIZE / WRITE_SIZE counters)."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied 3 x {4 * n} bytes", flush=True)


def near_probe(reps=3):
    """The near-field routes alone, for kernel traces and counters: the
    upsampled route and the learned route (every target) on the 1e6-target
    test set, with an untrained packed network (the kernels' work does not
    depend on the weights), reps times each."""
    import torch
    import synth
    import paper_1510_05616_amd as s2d
    from paper_1510_05616_amd import near
    s2d.stokes2d_init(0)
    te = near.NearData(*synth.make_near_dataset(1000000, 7)[:4], mu=1.0, upsample=8, labels=False)
    prm = torch.as_tensor(near.init_weights(0), dtype=torch.float32, device="cuda")
    blob = torch.empty(near.near_mlp_blob_size(), dtype=torch.uint8, device="cuda")
    near.near_mlp_pack(prm, torch.zeros(64 * near.CELL, dtype=torch.float32, device="cuda"), near.N_BINS,
                       near.BIN_LO, near.BIN_W, blob)
    du = torch.empty(te.n, dtype=torch.float64, device="cuda")
    dv = torch.empty_like(du)
    for name, m in (("upsampled", near.S2D_NEAR_UPSAMPLE), ("learned", near.S2D_NEAR_MLP)):
        for r in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            te.correct(m, blob, 0.0, du, dv)
            torch.cuda.synchronize()
            print(f"{name} route {r}: {(time.perf_counter() - t0) * 1e3:.3f} ms", flush=True)


def load_problem(cfg: int):
    import synth
    t0 = time.time()
    prob = synth.make_config(cfg)
    log(f"config {cfg}: {prob.ves.n_nodes} vesicle nodes, {prob.wall.n_nodes} wall nodes, "
        f"{prob.trg.n} targets ({time.time() - t0:.1f}s)")
    return prob


def run_mode(prob, mode, steps, warmup):
    import torch
    import paper_1510_05616_amd as s2d
    t = prob.trg
    ves, wall = s2d.Curves(prob.ves), s2d.Curves(prob.wall)
    tv = s2d.Targets(t.x, t.y, t.ves_curve, t.ves_node)
    tw = s2d.Targets(t.x, t.y, t.wall_curve, t.wall_node)
    u = torch.zeros(t.n, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(u)
    nws = max(s2d.stokes2d_workspace_size(s2d.S2D_OP_SLP, mode, ves, tv),
              s2d.stokes2d_workspace_size(s2d.S2D_OP_DLP, mode, wall, tw))
    ws = torch.empty(nws, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        s2d.stokes2d_slp_eval(mode, ves, tv, prob.d, -1, 1, prob.mu, u, v, 0, ws, stream)
        s2d.stokes2d_dlp_eval(mode, wall, tw, prob.d, -1, 1, u, v, 1, ws, stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    s2d.stokes2d_profile_read(s2d.S2D_OP_SLP)       # drop anything recorded earlier
    s2d.stokes2d_profile_read(s2d.S2D_OP_DLP)
    s2d.stokes2d_profile_enable(True)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for i in range(steps):
        step()
    end.record(stream)
    torch.cuda.synchronize()
    s2d.stokes2d_profile_enable(False)
    ms = start.elapsed_time(end)
    slp_ms, slp_n = s2d.stokes2d_profile_read(s2d.S2D_OP_SLP)
    dlp_ms, dlp_n = s2d.stokes2d_profile_read(s2d.S2D_OP_DLP)
    return dict(ms_total=ms, slp_ms=slp_ms / max(slp_n, 1), dlp_ms=dlp_ms / max(dlp_n, 1),
                u=u.cpu().numpy(), v=v.cpu().numpy(), ws_bytes=nws)


def _time(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


# algorithmic flops per pair (FMA = 2, reciprocal = 1) of the pressure and
# traction terms: r (2), |r|^2 (3), 1/|r|^2 (1), then
#   single-layer pressure: r.g (3), accumulate (2)                          = 11
#   double-layer pressure: r.nu, r.tau (6), 2 (r.nu)(r.tau) (2), two FMAs (4) = 18
#   single-layer traction: r.g, r.m (6), products (3), accumulate (4)       = 19
F1_FLOPS = {"slp_pressure": 11, "dlp_pressure": 18, "slp_traction": 19}


def f1_section(prob, reps=5):
    """Pressure and traction at the free targets of the 128k channel: 128,000
    seeded fluid points plus the 64 side-wall points (single-layer pressure
    and traction from the 96,000 vesicle nodes, double-layer pressure from
    the 32,000 wall nodes, images -1..1), FP32C and FP64, with the FP64 oracle
    on a seeded sample of 256 targets."""
    import torch
    import oracle
    import synth
    import paper_1510_05616_amd as s2d
    fx, fy = synth.fluid_points(prob, 128000, seed=11)
    side = prob.trg.kind == 2
    x = np.concatenate([fx, prob.trg.x[side]])
    y = np.concatenate([fy, prob.trg.y[side]])
    n = x.shape[0]
    th = np.random.default_rng(12).uniform(0.0, 2 * np.pi, n)
    mxn, myn = np.cos(th), np.sin(th)
    f64 = dict(dtype=torch.float64, device="cuda")
    tg = s2d.Targets(x, y)
    ves, wall = s2d.Curves(prob.ves), s2d.Curves(prob.wall)
    mx, my = torch.as_tensor(mxn, **f64), torch.as_tensor(myn, **f64)
    o1, o2 = torch.zeros(n, **f64), torch.zeros(n, **f64)
    nws = max(s2d.stokes2d_workspace_size(op, mode, src, tg) for mode in (0, 1)
              for op, src in ((s2d.S2D_OP_SLP_PRESSURE, ves), (s2d.S2D_OP_DLP_PRESSURE, wall),
                              (s2d.S2D_OP_SLP_TRACTION, ves)))
    ws = torch.empty(nws, dtype=torch.uint8, device="cuda")
    nv, nw = prob.ves.n_nodes, prob.wall.n_nodes
    ops = {
        "slp_pressure": (s2d.S2D_OP_SLP_PRESSURE, n * nv * 3,
                         lambda m: s2d.stokes2d_slp_pressure_eval(m, ves, tg, prob.d, -1, 1, o1, 0, ws)),
        "dlp_pressure": (s2d.S2D_OP_DLP_PRESSURE, n * nw * 3,
                         lambda m: s2d.stokes2d_dlp_pressure_eval(m, wall, tg, prob.d, -1, 1, prob.mu, o1, 0, ws)),
        "slp_traction": (s2d.S2D_OP_SLP_TRACTION, n * nv * 3,
                         lambda m: s2d.stokes2d_slp_traction_eval(m, ves, tg, mx, my, prob.d, -1, 1, o1, o2, 0, ws)),
    }
    idx = np.random.default_rng(13).choice(n, 256, replace=False)
    xs, ys = x[idx], y[idx]
    t0 = time.time()
    ref = {"slp_pressure": (oracle.slp_pressure(prob.ves, xs, ys, prob.d, -1, 1),),
           "dlp_pressure": (oracle.dlp_pressure(prob.wall, xs, ys, prob.d, -1, 1, prob.mu),),
           "slp_traction": oracle.slp_traction(prob.ves, xs, ys, mxn[idx], myn[idx], prob.d, -1, 1)}
    t_oracle = time.time() - t0
    res = {"workload": "128,000 fluid points + 64 side-wall points of the 128k channel (free targets), "
                       "vesicle single-layer pressure and traction, wall double-layer pressure, images -1..1",
           "n_targets": n, "flops_per_pair": F1_FLOPS,
           "oracle_sample": {"targets": 256, "seconds": t_oracle, "threads": oracle.num_threads()}}
    for name, mode in (("f32", s2d.S2D_FP32C), ("f64", s2d.S2D_FP64)):
        out = {}
        for op, (code, pairs, fn) in ops.items():
            fn(mode)
            torch.cuda.synchronize()
            s2d.stokes2d_profile_read(code)
            s2d.stokes2d_profile_enable(True)
            ms = _time(lambda: fn(mode), reps=reps)
            s2d.stokes2d_profile_enable(False)
            kms, kn = s2d.stokes2d_profile_read(code)
            kms /= max(kn, 1)
            got = [o1.cpu().numpy()[idx]] + ([o2.cpu().numpy()[idx]] if op == "slp_traction" else [])
            e = max(float(np.abs(g - r).max()) for g, r in zip(got, ref[op])) / \
                max(float(np.abs(r).max()) for r in ref[op])
            tf = F1_FLOPS[op] * pairs / (kms * 1e-3) / 1e12
            out[op] = {"ms": ms, "kernel_ms": kms, "pairs": pairs, "value": pairs / (ms * 1e-3),
                       "unit": "pair-evals/s", "achieved_tflops": tf, "peak_tflops": PEAK[name] / 1e12,
                       "frac": tf * 1e12 / PEAK[name], "rel_err_vs_oracle": e}
            log(f"f1 {name} {op}: {ms:.3f} ms ({pairs / (ms * 1e-3):.3e} pairs/s), kernel {kms:.3f} ms, "
                f"{tf:.1f} TFLOP/s, E={e:.2e}")
        res[name] = out
    pairs_sample = 256 * (2 * nv + nw) * 3
    res["cpu_baseline"] = {"value": pairs_sample / t_oracle, "unit": "pair-evals/s", "kind": "oracle",
                           "cores": oracle.num_threads(), "sample": "256 seeded targets x the three operators "
                           "x all sources x 3 images (FP64)"}
    return res


# algorithmic flops of the wall upsampling sums: per (fine point, mode k) the
# four values Re(V_k e^{ik th}) (4 each), the two derivatives Re(i k V_k
# e^{ik th}) (5 each) and the twiddle rotation (6); per (mode, node) of the
# coefficient sums 4 complex-by-real products (16), the shift of x (2) and
# the rotation (6)
WALL_SYNTH_FLOPS, WALL_DFT_FLOPS = 32, 24


def wall_section(prob, n_trg=20000, P=8, reps=5):
    """Near-wall correction of the walls' double layer on the 128k channel:
    its two walls of 16,000 nodes (smooth seeded densities) refined P = 8
    times by the library, Delta = D_P - D_1 over images -1..1 at 20,000
    seeded points 0.05..3 node spacings inside the fluid; FP64.  The dominant
    kernel is the double-layer pair kernel over the 256,000 refined nodes."""
    import torch
    import oracle
    import synth
    import paper_1510_05616_amd as s2d
    from oracle import near as onear
    from paper_1510_05616_amd import near as pn
    walls_np = synth.wall_densities(prob.wall, 21)
    tx, ty = synth.near_wall_points(walls_np, n_trg, seed=22)
    walls, tg = s2d.Curves(walls_np), s2d.Targets(tx, ty)
    f64 = dict(dtype=torch.float64, device="cuda")
    du, dv = torch.zeros(n_trg, **f64), torch.zeros(n_trg, **f64)
    ws = torch.empty(pn.near_wall_workspace_size(walls, tg, P), dtype=torch.uint8, device="cuda")
    corr = lambda: pn.near_wall_correct_eval(walls, tg, prob.d, -1, 1, P, du, dv, ws=ws)
    ms_corr = _time(corr, reps)
    fine = pn.stokes2d_wall_upsample(walls, prob.d, P)
    ms_up = _time(lambda: pn.stokes2d_wall_upsample(walls, prob.d, P), reps)
    u, v = torch.zeros(n_trg, **f64), torch.zeros(n_trg, **f64)
    pws = torch.empty(s2d.stokes2d_workspace_size(s2d.S2D_OP_DLP, s2d.S2D_FP64, fine, tg), dtype=torch.uint8,
                      device="cuda")
    dlp = lambda: s2d.stokes2d_dlp_eval(s2d.S2D_FP64, fine, tg, prob.d, -1, 1, u, v, 0, pws)
    dlp()
    torch.cuda.synchronize()
    s2d.stokes2d_profile_read(s2d.S2D_OP_DLP)
    s2d.stokes2d_profile_enable(True)
    _time(dlp, reps)
    s2d.stokes2d_profile_enable(False)
    kms, kn = s2d.stokes2d_profile_read(s2d.S2D_OP_DLP)
    kms /= max(kn, 1)
    corr()
    torch.cuda.synchronize()
    gu, gv = du.cpu().numpy(), dv.cpu().numpy()
    nw, nf = prob.wall.n_nodes, P * prob.wall.n_nodes
    pairs_fine = n_trg * nf * 3
    tf = FLOPS_PER_PAIR * pairs_fine / (kms * 1e-3) / 1e12
    half = nw // 2                                  # nodes per wall
    up_flops = 2 * (P * half * (half // 2 - 1) * WALL_SYNTH_FLOPS + (half // 2 + 1) * half * WALL_DFT_FLOPS)

    # the oracle: refined walls by FFT, both double layers by direct sums,
    # on a seeded sample of the targets
    ns = 200
    idx = np.random.default_rng(23).choice(n_trg, ns, replace=False)
    t0 = time.time()
    parts = []
    for c in range(walls_np.n_curves):
        sl = slice(walls_np.curve_off[c], walls_np.curve_off[c + 1])
        r = onear.wall_upsample(walls_np.x[sl], walls_np.y[sl], walls_np.nx[sl], walls_np.ny[sl],
                                walls_np.fx[sl], walls_np.fy[sl], prob.d, P)
        parts.append((r[0], r[1], r[2], r[3], r[4], np.zeros_like(r[0]), r[5], r[6]))
    fine_np = synth.concat_curves(parts)
    uP, vP = oracle.dlp(fine_np, tx[idx], ty[idx], None, None, prob.d, -1, 1)
    u1, v1 = oracle.dlp(walls_np, tx[idx], ty[idx], None, None, prob.d, -1, 1)
    t_or = time.time() - t0
    e = max(np.abs(gu[idx] - (uP - u1)).max(), np.abs(gv[idx] - (vP - v1)).max()) / np.hypot(uP, vP).max()
    log(f"walls: correction {ms_corr:.3f} ms for {n_trg} targets (upsampling {ms_up:.3f} ms, refined DLP pair "
        f"kernel {kms:.3f} ms = {tf:.1f} TFLOP/s), E={e:.2e}; oracle {t_or:.1f}s for {ns} targets")
    return {"workload": "2 walls x 16,000 nodes of the 128k channel refined 8x, Delta = D_P - D_1 at 20,000 "
                        "near-wall points (0.05..3 spacings), images -1..1, FP64",
            "ms": ms_corr, "value": n_trg / (ms_corr * 1e-3), "unit": "corrected targets/s",
            "upsample_ms": ms_up, "upsample_tflops": up_flops / (ms_up * 1e-3) / 1e12,
            "roofline": {"bound": "alu", "kernel": "pair_kernel<DLP> over the refined walls", "achieved": tf,
                         "peak": PEAK["f64"] / 1e12, "unit": "TFLOP/s", "frac": tf * 1e12 / PEAK["f64"],
                         "traffic": None, "flops_per_pair": FLOPS_PER_PAIR, "pairs_per_launch": pairs_fine,
                         "kernel_ms": kms},
            "rel_err_vs_oracle": float(e),
            "cpu_baseline": {"value": ns / t_or, "unit": "corrected targets/s", "kind": "oracle",
                             "cores": oracle.num_threads(),
                             "sample": f"{ns} seeded targets: FFT refinement of both walls plus the refined and "
                                       "given double layers by direct FP64 sums"}}


def wall_learned_section(prob, n_train=200000, n_test=1000000, steps=200000):
    """The learned route for the walls on the 128k channel's walls (2 x
    16,000 nodes, smooth densities, images -1..1): the network trained on
    200,000 targets at log-uniform distances 0.05..5 spacings (labels from
    the 8x refined walls) for 200,000 steps, calibrated on 1,000,000, then on
    1,000,000 test targets the refined quadrature (every target against all
    256,000 refined nodes), the learned route alone, and AUTO at per-wall
    tolerances of 1e-4 and 1e-3 of each wall's largest |D_P|.  Errors are
    normalised per wall by that largest |D_P|."""
    import torch
    import synth
    from paper_1510_05616_amd import near as pn
    walls = synth.wall_densities(prob.wall, 41)
    d = prob.d
    t0 = time.time()
    tr = pn.WallNearData(walls, d, *synth.near_wall_dataset(walls, n_train, 42))
    torch.cuda.synchronize()
    t_data = time.time() - t0
    t0 = time.time()
    params, hist = pn.train(tr, steps=steps, batch=1024, lr=2e-3, log_every=steps)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    del tr
    va = pn.WallNearData(walls, d, *synth.near_wall_dataset(walls, 1000000, 43))
    blob, bound, bound0, count = pn.calibrate(va, params, margin=1.5, count_margin=2.0)
    del va
    te = pn.WallNearData(walls, d, *synth.near_wall_dataset(walls, n_test, 44))
    du = torch.empty(te.n, dtype=torch.float64, device="cuda")
    dv = torch.empty_like(du)
    fb = torch.zeros(te.n, dtype=torch.int32, device="cuda")
    ws = {m: torch.empty(pn.near_wall_workspace_size(te.curves, te.trg, 8, m), dtype=torch.uint8, device="cuda")
          for m in (pn.S2D_NEAR_UPSAMPLE, pn.S2D_NEAR_MLP, pn.S2D_NEAR_AUTO)}
    tols = {rel: te.curve_tolerance(rel) for rel in (1e-4, 1e-3)}
    run = {
        "upsampled": lambda: pn.near_wall_correct_eval(te.curves, te.trg, d, -1, 1, 8, du, dv,
                                                       ws=ws[pn.S2D_NEAR_UPSAMPLE]),
        "learned": lambda: pn.near_wall_correct_eval(te.curves, te.trg, d, -1, 1, 8, du, dv,
                                                     method=pn.S2D_NEAR_MLP, trg_curve=te.tc, blob=blob,
                                                     ws=ws[pn.S2D_NEAR_MLP]),
    }
    for rel, tol in tols.items():
        run[f"auto_{rel:g}"] = (lambda tol=tol: pn.near_wall_correct_eval(
            te.curves, te.trg, d, -1, 1, 8, du, dv, method=pn.S2D_NEAR_AUTO, trg_curve=te.tc, blob=blob,
            used_fallback=fb, ws=ws[pn.S2D_NEAR_AUTO], curve_tol=tol))
    out = {"workload": "learned wall correction: 128k channel walls (2 x 16,000 nodes), 1,000,000 test targets "
                       "at 0.05..5 spacings, images -1..1, refined 8x; trained on 200,000 targets, calibrated on "
                       "1,000,000",
           "train_s": t_train, "data_s": t_data, "train_steps": steps, "loss": [hist[0][1], hist[-1][1]]}
    for name, fn in run.items():
        ms = _time(fn, reps=2)
        fn()
        torch.cuda.synchronize()
        e = te.scaled_errors(du, dv)
        out[name] = {"ms": ms, "max_normalised_error": e.max().item(),
                     "max_scaled_error_pi_over_d0": (torch.hypot(du - te.du, dv - te.dv) * math.pi
                                                     / te.frame[:, 9:11].abs().sum(1)).max().item()}
        if name.startswith("auto"):
            out[name]["fractions_learned_quadrature_none"] = [(fb == k).float().mean().item() for k in range(3)]
    base = out["upsampled"]["ms"]
    for name in out:
        if isinstance(out[name], dict) and name != "upsampled":
            out[name]["speedup_vs_upsampled"] = base / out[name]["ms"]
    log(f"walls learned: train {t_train:.1f}s; upsampled {base:.1f} ms; learned {out['learned']['ms']:.2f} ms "
        f"(E={out['learned']['max_normalised_error']:.2e}); " + "; ".join(
            f"{k}: {v['ms']:.2f} ms E={v['max_normalised_error']:.2e} fractions "
            + "/".join(f"{x:.2f}" for x in v["fractions_learned_quadrature_none"])
            for k, v in out.items() if k.startswith("auto")))
    return out


def step_section(prob, steps=3, dt=1e-4, kappa_b=1.0):
    """Vesicle time steps (Algorithm 1, steps 6-9) of the 128k channel's
    1,000 vesicles x 96 nodes in the periodic free-space setting (single
    layer over images -1..1, d = 64 pi; no wall response): the step system
    solved by GMRES (right-preconditioned by the factored per-vesicle self
    blocks), update, area correction, reparameterization; solved to 1e-10
    with FP64 single-layer sums, and by iterative refinement with FP32C sums
    (FP64 right-hand side and residuals, FP32C corrections).  The oracle
    times one step of 4 of the vesicles on the host."""
    import torch
    import oracle
    import paper_1510_05616_amd as s2d
    from oracle import vesicle as ov
    from paper_1510_05616_amd import vesicle as pv
    ves = prob.ves
    n = ves.n_nodes
    out = {"workload": "1,000 vesicles x 96 nodes of the 128k channel, images -1..1 (d = 64 pi), "
                       f"dt = {dt}, kappa_B = {kappa_b}, mu = {prob.mu}: one step = GMRES solve of the "
                       "288,000-unknown step system + update + area correction + reparameterization",
           "n_nodes": n}
    out["near_pairs"] = _near_pair_count(ves, prob.d, 5.0)
    for name, mode, tol, near in (("f64", s2d.S2D_FP64, 1e-10, 0), ("f32", s2d.S2D_FP32C, 1e-10, 0),
                                  ("f32_near", s2d.S2D_FP32C, 1e-10, 1)):
        V = pv.Vesicles(ves.x, ves.y, ves.curve_off)
        L0, A0 = V.measure()
        p = pv.params(mode=mode, dt=dt, kappa_b=kappa_b, mu=prob.mu, d=prob.d, img_lo=-1, img_hi=1, L0=L0,
                      tol=tol, restart=64, max_iter=500, nmax=96, near=near, near_P=8, near_band=5.0,
                      near_max=1 << 22)
        ws = V.workspace(p)
        V.time_step(p, A0=A0, ws=ws)                     # warm-up
        torch.cuda.synchronize()
        s2d.stokes2d_profile_read(s2d.S2D_OP_SLP)
        s2d.stokes2d_profile_enable(True)
        its = []
        t0 = time.time()
        for _ in range(steps):
            it, res = V.time_step(p, A0=A0, ws=ws)
            its.append((it, res))
        torch.cuda.synchronize()
        ms = (time.time() - t0) * 1e3 / steps
        s2d.stokes2d_profile_enable(False)
        kms, kn = s2d.stokes2d_profile_read(s2d.S2D_OP_SLP)
        pairs = n * n * 3
        avg = kms / max(kn, 1)
        tf = FLOPS_PER_PAIR * pairs / (avg * 1e-3) / 1e12
        peak = PEAK["f64" if mode == s2d.S2D_FP64 else "f32"]
        out[name] = {"ms_per_step": ms, "value": 1e3 / ms, "unit": "time steps/s", "gmres": its,
                     "single_layer_launches_per_step": kn / steps, "slp_ms_per_step": kms / steps}
        if name == "f64":
            out[name]["roofline"] = {"bound": "alu", "kernel": "pair_kernel<SLP> (on-curve, Kress self terms)",
                                     "achieved": tf, "peak": peak / 1e12, "unit": "TFLOP/s",
                                     "frac": tf * 1e12 / peak, "flops_per_pair": FLOPS_PER_PAIR,
                                     "pairs_per_launch": pairs, "kernel_ms": avg, "traffic": None}
            log(f"step {name}: {ms:.1f} ms per time step, GMRES {its}, {kn / steps:.1f} single-layer launches per "
                f"step ({kms / steps:.1f} ms, {avg:.2f} ms each = {tf:.1f} TFLOP/s)")
        else:
            # FP64 right-hand side and residuals, FP32C corrections: the
            # launches are of both precisions
            what = ("close evaluation of %d near pairs (8x), " % out["near_pairs"]) if near else ""
            log(f"step {name} ({what}FP32C corrections, FP64 residuals): {ms:.1f} ms per time step, GMRES {its}, "
                f"{kn / steps:.1f} single-layer launches per step ({kms / steps:.1f} ms)")
    # the oracle: one step of 4 vesicles (dense solve of the 1,152-unknown system)
    off = ves.curve_off
    s = slice(0, int(off[4]))
    sub_off = off[:5] - off[0]
    x, y = ves.x[s].copy(), ves.y[s].copy()
    g = ov.geometry(x, y, sub_off)
    t0 = time.time()
    ov.time_step(x, y, np.zeros(x.shape[0]), sub_off, dt, kappa_b, prob.mu, L0=ov.arc_lengths(g),
                 A0=ov.areas(x, y, sub_off), d=prob.d, img_lo=-1, img_hi=1)
    t_or = time.time() - t0
    out["cpu_baseline"] = {"value": 1.0 / t_or, "unit": "time steps/s", "kind": "oracle",
                           "cores": oracle.num_threads(),
                           "sample": "one step of 4 of the 1,000 vesicles (384 nodes, dense FP64 solve)"}
    log(f"step oracle: {t_or:.2f} s for one step of 4 vesicles")
    return out


def _near_pair_count(ves, d, band):
    """(node, vesicle, image) pairs of the close evaluation: nodes within band
    times the vesicle's largest spacing of one of its nodes (images -1..1,
    the own vesicle at image 0 excluded), counted on the host with a k-d tree."""
    from scipy.spatial import cKDTree
    off = np.asarray(ves.curve_off)
    x, y = np.asarray(ves.x), np.asarray(ves.y)
    n, nc = x.shape[0], off.shape[0] - 1
    own = np.repeat(np.arange(nc), np.diff(off))
    h = np.zeros(nc)
    for c in range(nc):
        xs, ys = x[off[c]:off[c + 1]], y[off[c]:off[c + 1]]
        # the largest trapezoid weight, from the spectral speed of the node curve
        N = xs.shape[0]
        k = np.fft.fftfreq(N, 1.0 / N)
        k[N // 2] = 0.0
        xa = np.fft.ifft(1j * k * np.fft.fft(xs)).real
        ya = np.fft.ifft(1j * k * np.fft.fft(ys)).real
        h[c] = (2 * np.pi / N) * np.hypot(xa, ya).max()
    tree = cKDTree(np.stack([x, y], 1))
    count = 0
    for kimg in (-1, 0, 1):
        pts = np.stack([x - kimg * d, y], 1)
        hits = tree.query_ball_point(pts, band * h.max())
        for i, js in enumerate(hits):
            if not js:
                continue
            js = np.asarray(js)
            cs = own[js]
            r2 = (pts[i, 0] - x[js]) ** 2 + (pts[i, 1] - y[js]) ** 2
            ok = r2 < (band * h[cs]) ** 2
            near = set(cs[ok].tolist())
            if kimg == 0:
                near.discard(own[i])
            count += len(near)
    return count


def channel_section(prob, steps=2, dt=1e-4, kappa_b=1.0, p_drive=10.0, n_proxy=128, wall_nodes=16000):
    """Algorithm 1 in the 128k channel: its walls at 2 x 16,000 nodes with
    the 32 Gauss-Legendre side heights and 128 proxies factored once
    (step 1: the dense 64,256-unknown periodization system, a blocked LU in
    four panels), then time steps of the 1,000 vesicles: total membrane force
    (step 2), the channel's response (steps 3-5: single layer on the walls
    and side walls, cell solve, wall double layer and proxies at the 96,000
    vesicle nodes), the preconditioned step, update, area correction and
    reparameterization (steps 6-9); FP64."""
    import torch
    import synth
    from paper_1510_05616_amd import vesicle as pv
    from paper_1510_05616_amd.cell import Cell
    h, hp, hpp = synth.wall_profile("sin13")
    side_y = synth._side_targets(h, prob.d, 32)[1][:32]
    walls = synth.concat_curves([(*synth._wall(h, hp, hpp, prob.d, wall_nodes, up)[:6], np.zeros(wall_nodes),
                                  np.zeros(wall_nodes)) for up in (True, False)])
    cell = Cell(walls, side_y, prob.d, n_proxy, prob.mu)
    torch.cuda.synchronize()
    t0 = time.time()
    cell.factor()
    torch.cuda.synchronize()
    t_factor = time.time() - t0
    ves = prob.ves
    out = {"workload": f"Algorithm 1 in the 128k channel: walls at 2 x {wall_nodes:,} nodes, K = 32, M = 128 (cell factored "
                       "once), 1,000 vesicles x 96 nodes, dt = %g, kappa_B = %g, p_drive = %g per period; "
                       "response in FP64, the step solved to 1e-10 with FP64 sums (f64) or by FP32C corrections "
                       "with FP64 residuals (f32; f32_near: with close evaluation of near vesicle pairs, 8x "
                       "upsampled, band 5 spacings)" % (dt, kappa_b, p_drive),
           "cell_factor_s": t_factor}
    for name, mode, near in (("f64", 0, 0), ("f32", 1, 0), ("f32_near", 1, 1)):
        V = pv.Vesicles(ves.x, ves.y, ves.curve_off)
        L0, A0 = V.measure()
        ws = None
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        resp_ms, step_ms, its = [], [], []
        for k in range(steps + 1):                   # step 0 is the warm-up
            torch.cuda.synchronize()
            t0 = time.time()
            fx, fy = V.total_force(kappa_b)
            ev[0].record()
            ur = V.channel_response(cell, fx, fy, p_drive)
            ev[1].record()
            p = pv.params(mode=mode, dt=dt, kappa_b=kappa_b, mu=prob.mu, d=prob.d, img_lo=-1, img_hi=1, L0=L0,
                          u_resp=ur, tol=1e-10, nmax=96, near=near, near_P=8, near_band=5.0, near_max=1 << 22)
            ws = V.workspace(p) if ws is None else ws
            it, res = V.time_step(p, A0=A0, ws=ws)
            torch.cuda.synchronize()
            if k > 0:
                step_ms.append((time.time() - t0) * 1e3)
                resp_ms.append(ev[0].elapsed_time(ev[1]))
                its.append((it, res))
        ms = sum(step_ms) / len(step_ms)
        log(f"channel {name}: cell factor {t_factor:.1f} s ({4 * wall_nodes + 2 * n_proxy:,} unknowns); Algorithm 1 step {ms:.1f} ms "
            f"(response {sum(resp_ms) / len(resp_ms):.1f} ms), GMRES {its}")
        out[name] = {"ms_per_step": ms, "value": 1e3 / ms, "unit": "time steps/s",
                     "response_ms": sum(resp_ms) / len(resp_ms), "gmres": its}
    return out


def cell_section(n_wall=4000, K=32, M=128, reps=5):
    """Periodization system of an empty channel cell at the paper's sizes
    (y = +-(1 + 0.3 sin x), d = 2 pi, 4000 nodes per wall, K = 32 side
    heights, M = 128 proxies, mu = 0.7): factor (block fill, blocked LU of
    the 16,000 x 16,000 wall block, A^-1 B, Schur complement, SVD) and solve
    times, the Poiseuille test errors at (0.8, 0), (3.2, 0), (4.8, 0), and
    the FP64 oracle's dense solve at 500 nodes per wall for scale."""
    import torch
    import synth
    from paper_1510_05616_amd.cell import Cell
    alpha, mu = 0.2, 0.7
    walls, sy, d = synth.make_channel(n_wall, K)
    cell = Cell(walls, sy, d, M, mu)
    cell.factor()                       # first call: library handle and scratch set-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cell.factor()
    t_factor = time.perf_counter() - t0
    v, g = synth.poiseuille_cell_data(walls, sy, d, alpha, mu)
    f64 = dict(dtype=torch.float64, device="cuda")
    vt, gt = torch.as_tensor(v, **f64), torch.as_tensor(g, **f64)
    tau, c = cell.solve(vt, gt)
    ms_solve = _time(lambda: cell.solve(vt, gt, tau, c), reps=reps)
    X, Y = np.array([0.8, 3.2, 4.8]), np.zeros(3)
    u, w, p = cell.flow(tau, c, X, Y)
    ue, pe = synth.poiseuille(X, Y, alpha, mu)
    un = np.stack([u.cpu().numpy(), w.cpu().numpy()], 1)
    pn = p.cpu().numpy()
    eu = float(np.abs(un - ue).max() / (alpha * 1.3 ** 2))
    ep = float(np.abs((pn - pn[0]) - (pe - pe[0])).max() / (2 * alpha * mu * d))
    n, nc, mr = 4 * n_wall, 2 * M, 4 * K
    # LU (2/3 n^3) + A^-1 B (two triangular sweeps) + C A^-1 B
    flops = 2.0 / 3.0 * n ** 3 + 2.0 * n * n * nc + 2.0 * mr * n * nc
    tf = flops / t_factor / 1e12
    res = {"workload": f"empty channel y = +-(1 + 0.3 sin x), d = 2 pi, {n_wall} nodes per wall "
                       f"(system {n} + {nc} unknowns), K = {K}, M = {M}, Poiseuille data",
           "factor_s": t_factor, "solve_ms": ms_solve,
           "factor_flops": flops, "factor_tflops": tf, "peak_tflops": 78.6, "frac": tf / 78.6,
           "poiseuille_error": {"velocity": eu, "pressure": ep}}
    log(f"cell: factor {t_factor * 1e3:.1f} ms ({tf:.1f} TFLOP/s FP64: blocked LU), solve {ms_solve:.3f} ms, "
        f"Poiseuille error velocity {eu:.2e} pressure {ep:.2e}")
    return res


def cell_cpu_baseline(n_wall=500, K=32, M=128):
    """The oracle's dense numpy assembly and solve at 500 nodes per wall."""
    import synth
    from oracle import els
    walls, sy, d = synth.make_channel(n_wall, K)
    t0 = time.perf_counter()
    A, B, C, Q, _ = els.assemble(walls, sy, d, M, 0.7)
    v, g = synth.poiseuille_cell_data(walls, sy, d, 0.2, 0.7)
    els.solve(A, B, C, Q, v, g)
    t = time.perf_counter() - t0
    n = 4 * n_wall
    flops = 2.0 / 3.0 * n ** 3 + 2.0 * n * n * 2 * M + 2.0 * 4 * K * n * 2 * M
    return {"seconds": t, "n_wall": n_wall, "tflops": flops / t / 1e12, "kind": "oracle",
            "sample": f"{n_wall} nodes per wall (system {n} + {2 * M}), numpy/LAPACK"}


def batch_section():
    """Config 4: 256 independent channel instances (1-40 vesicles of
    32-256 nodes, 256-4096 wall nodes per wall) evaluated by one batched call
    (persistent work-list kernel recorded in a HIP graph, tile shape from the
    autotuner), FP32C, against the same instances as sequential single calls."""
    import torch
    import synth
    import paper_1510_05616_amd as s2d
    t0 = time.time()
    probs = synth.make_batch(256)
    log(f"batch: 256 instances generated ({time.time() - t0:.1f}s)")
    mode = s2d.S2D_FP32C
    insts = []
    for p in probs:
        t = p.trg
        u = torch.zeros(t.n, dtype=torch.float64, device="cuda")
        insts.append(s2d.BatchInstance(s2d.Curves(p.ves), s2d.Curves(p.wall),
                                       s2d.Targets(t.x, t.y, t.ves_curve, t.ves_node),
                                       s2d.Targets(t.x, t.y, t.wall_curve, t.wall_node), p.d, p.mu, u,
                                       torch.zeros_like(u)))
    pairs = sum(p.trg.n * (p.ves.n_nodes + p.wall.n_nodes) * 3 for p in probs)
    ws = torch.empty(s2d.stokes2d_batch_workspace_size(mode, insts), dtype=torch.uint8, device="cuda")
    t0 = time.time()
    s2d.stokes2d_batch_eval(mode, insts, ws)          # plans, tunes, records the graph
    torch.cuda.synchronize()
    t_first = time.time() - t0
    ms_batch = _time(lambda: s2d.stokes2d_batch_eval(mode, insts, ws), reps=5)
    wss = torch.empty(max(max(s2d.stokes2d_workspace_size(0, mode, b.ves, b.trg_ves),
                              s2d.stokes2d_workspace_size(1, mode, b.wall, b.trg_wall)) for b in insts),
                      dtype=torch.uint8, device="cuda")

    def singles():
        for b in insts:
            s2d.stokes2d_slp_eval(mode, b.ves, b.trg_ves, b.d, -1, 1, b.mu, b.u, b.v, 0, wss)
            s2d.stokes2d_dlp_eval(mode, b.wall, b.trg_wall, b.d, -1, 1, b.u, b.v, 1, wss)
    ms_single = _time(singles, reps=3)
    shape = s2d.stokes2d_batch_tuned(mode, insts)
    s2d.stokes2d_batch_release()
    res = {"workload": "256 instances, 1-40 vesicles x {32,64,128,256} nodes, 256-4096 nodes per wall, "
                       "images -1..1, FP32C", "pairs": pairs, "ms": ms_batch,
           "value": pairs / (ms_batch * 1e-3), "unit": "pair-evals/s", "first_call_s": t_first,
           "sequential_single_calls_ms": ms_single, "speedup_vs_single_calls": ms_single / ms_batch,
           "tile_shape": shape}
    log(f"batch: {ms_batch:.2f} ms per batched call ({pairs / (ms_batch * 1e-3):.3e} pairs/s), "
        f"{ms_single:.2f} ms as 512 single calls, first call {t_first:.2f}s, shape {shape}")
    return res


def near_section(steps=400000):
    """Learned near-field correction on the near-target workload: train on
    200k targets (400,000 steps of 1024 on the GPU), calibrate on 2M, test on
    1M (targets at log-uniform normal distances 0.05 h .. 5 h from ellipses
    of 64-128 nodes).  Errors are normalised per curve by the largest |u| of
    the 8x upsampled single layer over that curve's test targets; AUTO takes
    per-curve tolerances of rel times that scale."""
    import torch
    import synth
    from paper_1510_05616_amd import near
    t0 = time.time()
    tr = near.NearData(*synth.make_near_dataset(200000, 5)[:4], mu=1.0, upsample=8)
    torch.cuda.synchronize()
    log(f"near: training data ready ({time.time() - t0:.1f}s)")
    t0 = time.time()
    params, hist = near.train(tr, steps=steps, batch=1024, lr=2e-3, log_every=steps)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    del tr
    va = near.NearData(*synth.make_near_dataset(2000000, 6)[:4], mu=1.0, upsample=8)
    blob, bound, bound0, count = near.calibrate(va, params, margin=1.5, count_margin=2.0)
    del va
    log(f"near: trained {steps} steps in {t_train:.1f}s, loss {hist[0][1]:.3e} -> {hist[-1][1]:.3e}")
    te = near.NearData(*synth.make_near_dataset(1000000, 7)[:4], mu=1.0, upsample=8)
    n = te.n
    du, dv = (torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(2))
    fb = torch.zeros(n, dtype=torch.int32, device="cuda")
    ws_up = near._empty(near.near_workspace_size(near.S2D_NEAR_UPSAMPLE, te.curves, te.trg, 8))
    ws_ml = near._empty(near.near_workspace_size(near.S2D_NEAR_AUTO, te.curves, te.trg, 8))
    run = lambda m, th=0.0, flag=None, ws=ws_ml, tol=None: near.near_correct_eval(
        m, te.curves, te.trg, te.tc, 8, blob, th, 1.0, du, dv, flag, ws, curve_tol=tol)
    err = lambda: te.scaled_errors(du, dv).max().item()
    ms_up = _time(lambda: run(near.S2D_NEAR_UPSAMPLE, ws=ws_up))
    ms_mlp = _time(lambda: run(near.S2D_NEAR_MLP))
    run(near.S2D_NEAR_MLP)
    torch.cuda.synchronize()
    e_mlp = err()
    err_mlp = te.scaled_errors(du, dv).cpu().numpy()
    auto = {}
    for rel in (1e-5, 3e-5, 1e-4):
        tol = te.curve_tolerance(rel)
        ms = _time(lambda: run(near.S2D_NEAR_AUTO, 0.0, fb, tol=tol))
        run(near.S2D_NEAR_AUTO, 0.0, fb, tol=tol)
        torch.cuda.synchronize()
        auto[f"{rel:g}"] = {"ms": ms, "speedup_vs_upsampled8": ms_up / ms, "err": err(),
                            "fractions_learned_quadrature_none": [float((fb == k).double().mean()) for k in range(3)]}
    # one scalar tolerance for every curve: 1e-5 of the smallest curve scale
    thr = 1e-5 * te.curve_scale.min().item()
    ms_s = _time(lambda: run(near.S2D_NEAR_AUTO, thr, fb))
    run(near.S2D_NEAR_AUTO, thr, fb)
    torch.cuda.synchronize()
    auto_scalar = {"threshold": thr, "ms": ms_s, "speedup_vs_upsampled8": ms_up / ms_s, "err": err(),
                   "fractions_learned_quadrature_none": [float((fb == k).double().mean()) for k in range(3)]}
    e_plain = te.scaled_errors(torch.zeros_like(du), torch.zeros_like(dv))
    err_plain = e_plain.cpu().numpy()
    # 32x upsampled quadrature as context for the 8x reference (64-node curves,
    # the largest that 32x upsampling supports)
    c64 = synth.make_near_dataset(100000, 8, sizes=(64,))
    d64 = near.NearData(*c64[:4], mu=1.0, upsample=8, labels=False)
    a8, b8, a1, b1 = (torch.empty(d64.n, dtype=torch.float64, device="cuda") for _ in range(4))
    a32, b32 = torch.empty_like(a8), torch.empty_like(a8)
    near.near_upsampled_slp(d64.curves, d64.trg, d64.tc, 8, 1.0, a8, b8, a1, b1)
    near.near_upsampled_slp(d64.curves, d64.trg, d64.tc, 32, 1.0, a32, b32, a1, b1)
    t64 = d64.tc.long()
    s64 = torch.zeros(d64.curves.n_curves, dtype=torch.float64, device="cuda").scatter_reduce(
        0, t64, torch.hypot(a32, b32), reduce="amax", include_self=False)[t64]
    e_8v32 = float((torch.hypot(a8 - a32, b8 - b32) / s64).max())
    b = te.b.cpu().numpy()
    gain = {}
    for lo, hi in ((0.05, 0.2), (0.2, 0.5), (0.5, 1.0), (1.0, 2.0), (2.0, 5.1)):
        m = (b >= lo) & (b < hi)
        gain[f"b {lo}-{hi}"] = {"plain_median": float(np.median(err_plain[m])),
                                "learned_median": float(np.median(err_mlp[m])),
                                "learned_q999": float(np.quantile(err_mlp[m], 0.999)),
                                "learned_max": float(err_mlp[m].max())}
    a5 = auto["1e-05"]
    res = {"workload": "1e6 targets at 0.05h..5h from 5000 ellipses of 64/96/128 nodes; network 14-64-64-64-20 "
                       "trained on the GPU on 2e5 8x-upsampled labels (400,000 steps of 1024), calibrated on 2e6",
           "err_vs_upsampled8": {"learned": e_mlp, "auto_1e-5_per_curve": a5["err"],
                                 "no_correction": float(err_plain.max())},
           "err_upsampled8_vs_32_on_64_node_curves": e_8v32, "error_by_normal_offset": gain,
           "ms": {"upsampled8": ms_up, "learned": ms_mlp, "auto_1e-5_per_curve": a5["ms"]},
           "speedup_vs_upsampled8": {"learned": ms_up / ms_mlp, "auto_1e-5_per_curve": a5["speedup_vs_upsampled8"]},
           "auto_per_curve": auto, "auto_scalar_1e-5_of_smallest_curve_scale": auto_scalar,
           "train_s": t_train, "train_steps": steps, "loss": [hist[0][1], hist[-1][1]]}
    log(f"near: upsampled {ms_up:.3f} ms, learned {ms_mlp:.3f} ms (E={e_mlp:.2e}); AUTO per curve " + "; ".join(
        f"{k}: {v['ms']:.3f} ms ({v['speedup_vs_upsampled8']:.2f}x, E={v['err']:.2e}, learned/quadrature/none "
        + "/".join(f"{x:.3f}" for x in v["fractions_learned_quadrature_none"]) + ")" for k, v in auto.items())
        + f"; scalar {ms_s:.3f} ms (E={auto_scalar['err']:.2e}); plain E={err_plain.max():.2e}, 8x vs 32x {e_8v32:.2e}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=65536,
                    help="targets of the workload the FP64 oracle evaluates on the host (0: skip)")
    ap.add_argument("--near", type=int, default=1, help="run the near-field correction section (0: skip)")
    ap.add_argument("--batch", type=int, default=1, help="run the batched-instances section (0: skip)")
    ap.add_argument("--f1", type=int, default=1, help="run the pressure/traction section (0: skip)")
    ap.add_argument("--cell", type=int, default=1, help="run the periodization-system section (0: skip)")
    ap.add_argument("--walls", type=int, default=1, help="run the near-wall correction sections (0: skip)")
    ap.add_argument("--walls-learned", type=int, default=1,
                    help="with --walls, also run the learned near-wall section (0: skip)")
    ap.add_argument("--step", type=int, default=1, help="run the vesicle time-step section (0: skip)")
    ap.add_argument("--channel", type=int, default=1,
                    help="run Algorithm 1 in the channel, with the cell factored once (0: skip)")
    ap.add_argument("--copy-probe", action="store_true", help="only copy 1 GiB on the device and exit")
    ap.add_argument("--issue-probe", action="store_true",
                    help="only run the VALU issue-rate probes, print their rates and exit")
    ap.add_argument("--near-probe", action="store_true",
                    help="only run the upsampled and learned near-field routes on 1e6 targets and exit")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.near_probe:
        near_probe()
        return
    if args.issue_probe:
        import torch
        import paper_1510_05616_amd as s2d
        s2d.stokes2d_init(0)
        print(json.dumps(issue_probe()), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; a single-GPU run "
              "measures one GPU's share of a target-sharded evaluation", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1510_05616_amd as s2d
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    s2d.stokes2d_init(0)
    prob = load_problem(args.config)
    n_trg, n_v, n_w = prob.trg.n, prob.ves.n_nodes, prob.wall.n_nodes
    n_img = 3
    pairs_slp = n_trg * n_v * n_img
    pairs_dlp = n_trg * n_w * n_img
    pairs = pairs_slp + pairs_dlp

    probe = issue_probe()
    log("VALU issue probe: " + ", ".join(f"{k} {v['wave_instr_per_s']:.3e} wave-instr/s ({v['tflops']:.1f} TFLOP/s)"
                                         for k, v in probe.items()))
    res = {}
    for name, mode in (("f32", s2d.S2D_FP32C), ("f64", s2d.S2D_FP64)):
        r = run_mode(prob, mode, args.steps, args.warmup)
        ms_step = r["ms_total"] / args.steps
        ach = FLOPS_PER_PAIR * pairs_slp / (r["slp_ms"] * 1e-3)
        kern = SLP_KERNEL[name]
        valu = measured_valu(kern)
        # the kernel's VALU wave-instruction rate (instructions per pair from
        # the committed counters) over the probe's all-VGPR rate of its type
        ceiling = probe["f32_vgpr" if name == "f32" else "f64"]["wave_instr_per_s"]
        rate = valu["valu_per_pair"] * pairs_slp / 64 / (r["slp_ms"] * 1e-3) if valu else None
        res[name] = dict(ms_per_step=ms_step, value=pairs / (ms_step * 1e-3),
                         slp_pair_ms=r["slp_ms"], dlp_pair_ms=r["dlp_ms"],
                         roofline={"bound": "alu", "kernel": kern,
                                   "achieved": ach / 1e12, "peak": PEAK[name] / 1e12,
                                   "unit": "TFLOP/s", "frac": ach / PEAK[name],
                                   "traffic": measured_traffic(kern),
                                   "valu_counters": valu,
                                   "issue_ceiling_wave_instr_per_s": ceiling,
                                   "issue_ceiling_frac": rate / ceiling if rate else None,
                                   "issue_probe": probe,
                                   "flops_per_pair": FLOPS_PER_PAIR, "pairs_per_launch": pairs_slp},
                         u=r["u"], v=r["v"])
        log(f"{name}: {ms_step:.3f} ms/step, {pairs / (ms_step * 1e-3):.4e} pairs/s, "
            f"SLP pair kernel {r['slp_ms']:.3f} ms, DLP pair kernel {r['dlp_ms']:.3f} ms")

    cpu = None
    errs = {}
    if args.cpu_sample > 0:
        import oracle
        rng = np.random.default_rng(12345)
        idx = np.sort(rng.choice(n_trg, min(args.cpu_sample, n_trg), replace=False))
        t = prob.trg
        oracle.build(force=False)
        t0 = time.time()
        us, vs = oracle.slp(prob.ves, t.x[idx], t.y[idx], t.ves_curve[idx], t.ves_node[idx],
                            prob.d, -1, 1, prob.mu)
        ud, vd = oracle.dlp(prob.wall, t.x[idx], t.y[idx], t.wall_curve[idx], t.wall_node[idx],
                            prob.d, -1, 1)
        dt = time.time() - t0
        sp = len(idx) * (n_v + n_w) * n_img
        cpu = {"value": sp / dt, "unit": "pair-evals/s", "cores": oracle.num_threads(),
               "kind": "oracle", "seconds": dt,
               "sample": f"{len(idx)} seeded targets of the same workload x all "
                         f"{n_v + n_w} sources x 3 images = {sp:.4e} FP64 pairs"}
        ru, rv = us + ud, vs + vd
        sc = np.hypot(ru, rv).max()
        for name in ("f32", "f64"):
            gu, gv = res[name]["u"][idx], res[name]["v"][idx]
            errs[name] = float(np.hypot(gu - ru, gv - rv).max() / sc)
        log(f"oracle: {dt:.1f}s on {cpu['cores']} threads, {cpu['value']:.3e} pairs/s; "
            f"rel err f32={errs['f32']:.2e} f64={errs['f64']:.2e}")

    f1_res = f1_section(prob) if args.f1 and args.config == 3 else None
    wall_res = wall_section(prob) if args.walls and args.config == 3 else None
    wall_learned = (wall_learned_section(prob) if args.walls and args.walls_learned and args.config == 3
                    else None)
    step_res = step_section(prob) if args.step and args.config == 3 else None
    chan_res = channel_section(prob) if args.channel and args.config == 3 else None
    cell_res = cell_section() if args.cell else None
    if cell_res is not None and args.cpu_sample > 0:
        cell_res["cpu_baseline"] = cell_cpu_baseline()
    near_res = near_section() if args.near else None
    batch_res = batch_section() if args.batch else None

    f32, f64 = res["f32"], res["f64"]
    line = {
        "metric": "Stokes pair-evals/s at N=128k, FP32 vs FP64 on GPU, at 1e-6 rel err vs FP64 oracle",
        "value": f32["value"], "unit": "pair-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": f32["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "periodic channel, 1000 vesicles x 96 nodes (SLP) + 2 walls x 16000 "
                               "nodes (DLP) + 64 side targets, d=64pi, images -1..1, all 128064 targets",
                   "n_targets": n_trg, "n_sources": n_v + n_w, "images": n_img,
                   "pairs_per_step": pairs, "parallelism": "single GPU"},
        "roofline": f32["roofline"],
        "cpu_baseline": cpu,
        "rel_err_vs_oracle": errs or None,
        "fp64": {"value": f64["value"], "unit": "pair-evals/s", "ms_per_step": f64["ms_per_step"],
                 "dtype": "f64", "roofline": f64["roofline"]},
        "kernel_ms": {"f32_slp_pair": f32["slp_pair_ms"], "f32_dlp_pair": f32["dlp_pair_ms"],
                      "f64_slp_pair": f64["slp_pair_ms"], "f64_dlp_pair": f64["dlp_pair_ms"]},
        "pressure_traction": f1_res,
        "periodization_cell": cell_res,
        "near_wall": wall_res,
        "near_wall_learned": wall_learned,
        "time_step": step_res,
        "algorithm1_channel": chan_res,
        "near": near_res,
        "batch": batch_res,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
