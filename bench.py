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
targets of the same workload on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--cpu-sample T]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 19          # algorithmic flops per pair, SLP and DLP alike
PEAK = {"f32": 157.3e12, "f64": 78.6e12}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=8192,
                    help="targets of the workload the FP64 oracle evaluates on the host (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the target-sharded design is described in DESIGN.md)", file=sys.stderr)
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

    res = {}
    for name, mode in (("f32", s2d.S2D_FP32C), ("f64", s2d.S2D_FP64)):
        r = run_mode(prob, mode, args.steps, args.warmup)
        ms_step = r["ms_total"] / args.steps
        ach = FLOPS_PER_PAIR * pairs_slp / (r["slp_ms"] * 1e-3)
        res[name] = dict(ms_per_step=ms_step, value=pairs / (ms_step * 1e-3),
                         slp_pair_ms=r["slp_ms"], dlp_pair_ms=r["dlp_ms"],
                         roofline={"bound": "alu", "kernel": "pair_kernel<SLP>",
                                   "achieved": ach / 1e12, "peak": PEAK[name] / 1e12,
                                   "unit": "TFLOP/s", "frac": ach / PEAK[name], "traffic": None,
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
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
