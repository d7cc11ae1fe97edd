#!/usr/bin/env python3
"""Throughput of the guided linear upsampling hot path on one MI355X.

One step = the pair search (Eq. 3-4, every pair of the 3 x 3 window) plus the
apply step (Eq. 1) over one 3840 x 2160 RGB float32 frame downsampled x8
(480 x 270), eps = 1e-3, launched as the two kernels glu_search and
glu_apply.  Inputs are seeded synthetic Voronoi frames (the 4K x8 workload:
1000 cells, 400 dots of 1-3 px, sigma 0.01, regular-grid downsampling, LR
operator f1) already resident in HBM; five buffer sets (about 1.2 GB) are
rotated so the 256 MB last-level cache cannot serve repeats.

Prints ONE JSON line (see the keys below).  Extra per-kernel timings (search,
apply, fused search+apply, the fast search of Algorithm 1) and the roofline
of the dominant kernel are measured live with HIP events on the stream the
kernels run on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

# the CPU baseline is the oracle on one thread
for _v in ("OMP_NUM_THREADS", "MKL_NUM_THREADS", "OPENBLAS_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

H, W, S, K, EPS = 2160, 3840, 8, 3, 1e-3
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3

# Algorithmic float32 operations per HR pixel of the search, k = 3 (9 cells,
# 36 pairs).  Exhaustive: 27 (I - L_j for 9 cells) + 5 (|d_0|^2) + 36 x 17
# (dot 5, weight 1, residual 6, squared norm 5).  Fast (Algorithm 1):
# 9 x (3 + 5 + 1 sqrt) for the distances, then 9 x (1 + 1 + 1 division
# + 1 + 6 + 6 + 5) for the partners.
FLOPS_PER_PX = {"exhaustive": 27 + 5 + 36 * 17, "fast": 9 * 9 + 9 * 21}
# Algorithmic HBM bytes per HR pixel (C = 3, float32): search reads I (12)
# and writes Theta (6); apply reads Theta (6) and writes T_hat (12); fused
# reads I and writes Theta and T_hat.
BYTES_PER_PX = {"search": 18, "apply": 18, "step": 36, "fused": 30, "bwd": 22}


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--mode", choices=["exhaustive", "fast"], default="exhaustive")
    ap.add_argument("--sets", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--only", choices=["all", "step"], default="all",
                    help="'step' times only the headline step (for profiling)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (a known-size reference for HBM counters)")
    return ap.parse_args()


def _kernel_source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2307_09582_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def _traffic(kernel_key: str, n_px: int):
    """HBM bytes per launch from the committed counter summary, or None when
    the kernel sources changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "traffic_4k_x8.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
    except Exception:
        return None
    if t.get("source_hash") != _kernel_source_hash():
        return None
    ent = t.get("kernels", {}).get(kernel_key)
    if not ent:
        return None
    return ent.get("hbm_bytes_per_launch")


def main():
    args = _parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the GLU hot path of this build runs on a single MI355X "
              "(multi-GPU sharding is a design note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2307_09582_amd as glu

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    t0 = time.time()
    scene = synth.make_scene(H, W, 1000, 400, (1, 3), seed=3, canvas_extra=177)
    sets = []
    for t in range(args.sets):
        I = torch.from_numpy(scene.frame(t, sigma=0.01, dtype=np.float32)).to(dev)
        Il = glu.downsample(I, S, "point")
        T = torch.from_numpy(synth.lr_op_f1(Il.cpu().numpy()).astype(np.float32)).to(dev)
        th = glu.empty_theta(H, W, dev)
        out = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
        sets.append(dict(I=I, Il=Il, T=T, th=th, out=out))
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    print("inputs ready in %.1f s" % gen_s, file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    n_px = H * W

    def step(i, mode):
        st = sets[i % len(sets)]
        glu.search(st["I"], st["Il"], S, K, EPS, mode, theta=st["th"])
        glu.apply(st["th"], st["T"], S, K, out=st["out"])

    def search_only(i, mode):
        st = sets[i % len(sets)]
        glu.search(st["I"], st["Il"], S, K, EPS, mode, theta=st["th"])

    def apply_only(i, mode):
        st = sets[i % len(sets)]
        glu.apply(st["th"], st["T"], S, K, out=st["out"])

    def fused(i, mode):
        st = sets[i % len(sets)]
        glu.search_apply(st["I"], st["Il"], st["T"], S, K, EPS, mode, theta=st["th"], out=st["out"])

    def timed(fn, mode, steps, warmup):
        for i in range(warmup):
            fn(i, mode)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(steps):
            fn(i, mode)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps  # ms

    # headline: timed region bracketed by synchronisation on both sides
    for i in range(args.warmup):
        step(i, args.mode)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    e0.record(stream)
    for i in range(args.steps):
        step(i, args.mode)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = e0.elapsed_time(e1) / args.steps
    value = n_px / (ms_step * 1e-3) / 1e6

    kern = {}
    other = "fast" if args.mode == "exhaustive" else "exhaustive"
    if args.only == "all":
        for mode in (args.mode, other):
            kern[mode] = dict(
                search_us=1e3 * timed(search_only, mode, args.steps, 3),
                apply_us=1e3 * timed(apply_only, mode, args.steps, 3),
                fused_us=1e3 * timed(fused, mode, args.steps, 3),
                step_us=1e3 * timed(step, mode, args.steps, 3),
            )
    else:
        kern[args.mode] = dict(search_us=float("nan"))

    bwd = None
    if args.only == "all":
        # backward of the apply step on the same frames (Theta from the search)
        G = torch.randn((H, W, 3), dtype=torch.float32, device=dev, generator=torch.Generator(dev).manual_seed(5))
        ws = torch.empty(glu.apply_backward_workspace(H, W, 3, S, K) // 4 + 1, dtype=torch.float32, device=dev)
        gT = torch.empty((H // S, W // S, 3), dtype=torch.float32, device=dev)
        ga = torch.empty((H, W), dtype=torch.float32, device=dev)

        def backward(i, mode):
            st = sets[i % len(sets)]
            glu.apply_backward(st["th"], st["T"], G, S, K, workspace=ws, out_T_low=gT, out_alpha=ga)

        bwd_ms = timed(backward, args.mode, args.steps, 3)
        bwd = {
            "us": round(1e3 * bwd_ms, 2),
            "Mpx_s": round(n_px / (bwd_ms * 1e-3) / 1e6, 1),
            "bytes_per_px": BYTES_PER_PX["bwd"],
            "hbm_frac": round(BYTES_PER_PX["bwd"] * n_px / (bwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        }

    ks = kern[args.mode]
    roof = None
    if args.only == "all":
        flops = FLOPS_PER_PX[args.mode] * n_px
        achieved = flops / (ks["search_us"] * 1e-6) / 1e12
        traffic = _traffic("search_" + args.mode, n_px)
        roof = {
            "kernel": "search_" + args.mode,
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
            "traffic": traffic,
        }

    cpu = None
    if not args.no_cpu_baseline:
        cpu = _cpu_baseline(scene, args.mode, args.cpu_seconds)

    step_gbs = BYTES_PER_PX["step"] * n_px / (ms_step * 1e-3) / 1e9
    res = {
        "metric": "HR Mpixel/s, GLU search+apply, 4K x8 fp32",
        "value": round(value, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Voronoi frames, inputs resident in HBM)",
        "config": {
            "workload": "3840x2160 RGB fp32, x8 point downsample to 480x270, 3x3 window, eps 1e-3, "
                        "%s pair search + apply (two kernels)" % args.mode,
            "mode": args.mode,
            "H": H, "W": W, "s": S, "k": K,
            "buffer_sets": len(sets),
        },
        "hbm": {
            "bytes_per_px": BYTES_PER_PX["step"],
            "achieved_GBps": round(step_gbs, 1),
            "peak_GBps": HBM_PEAK_GBS,
            "frac": round(step_gbs / HBM_PEAK_GBS, 4),
        },
        "roofline": roof,
        "kernels_us": {m: {k2: round(v, 2) for k2, v in d.items()} for m, d in kern.items()},
        "bwd": bwd,
        "cpu_baseline": cpu,
        "wall_s_timed_region": round(wall, 4),
    }
    if args.only == "all":
        for m, d in kern.items():
            res.setdefault("modes", {})[m] = {
                "step_Mpx_s": round(n_px / d["step_us"], 1),
                "fused_Mpx_s": round(n_px / d["fused_us"], 1),
                "step_hbm_frac": round(BYTES_PER_PX["step"] * n_px / (d["step_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                "fused_hbm_frac": round(BYTES_PER_PX["fused"] * n_px / (d["fused_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                "apply_hbm_frac": round(BYTES_PER_PX["apply"] * n_px / (d["apply_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            }
    if args.calib_copy:
        src = torch.empty(64 * 2**20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        res["calib_copy_bytes"] = 4 * src.numel()
    print(json.dumps(res), flush=True)


def _cpu_baseline(scene, mode, seconds):
    """The float64 oracle, as it stands, on a band of rows of frame 0."""
    import numpy as np

    import oracle as O
    import synth

    I = scene.frame(0, sigma=0.01, dtype=np.float32)
    L = O.downsample_point(I, S)
    T = synth.lr_op_f1(L)

    def run(rows):
        pix = np.arange(rows * W, dtype=np.int64)
        t = time.perf_counter()
        r = O.search(I, L, S, K, EPS, mode, pixels=pix)
        O.apply(r.a, r.b, r.alpha, T)
        return time.perf_counter() - t

    probe_rows = 8
    tp = run(probe_rows)
    rows = int(max(8, min(H, probe_rows * seconds / max(tp, 1e-3))))
    rows = (rows // 8) * 8 or 8
    dt = run(rows)
    n = rows * W
    return {
        "value": round(n / dt / 1e6, 4),
        "unit": "Mpixel/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "%s search + apply of rows 0..%d of the 3840x2160 frame (%d px, %.1f s), float64 NumPy, "
                  "one thread" % (mode, rows - 1, n, dt),
    }


if __name__ == "__main__":
    main()
