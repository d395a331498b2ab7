#!/usr/bin/env python3
"""Benchmark of the renderer's hot path on one MI355X.

One step = one dm_render_vjp call on the single-cell workload (deformed
icosphere, 5120 triangles, 128 x 128 x 64 grid of 0.2 x 0.2 x 0.5 um voxels,
Gaussian PSF sigma = (0.15, 0.15, 0.45) um, band OTF > 1e-3): mesh prep,
forward sweep over the band, OTF multiply and scatter, inverse FFT to the
image, FFT of dL/dI, adjoint weights and PSF gradient, gradient sweep and the
per-vertex reduction.  Inputs are resident in HBM before timing starts.

value = triangles x band entries / step time (each frequency-triangle pair is
evaluated once by the forward sweep and once by the gradient sweep per step).

Prints ONE JSON line.  Synthetic data (seeded); no dataset.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "tri·freq pairs/s fwd+VJP (5k tris, 128²×64) vs plain; p50/p99 render latency"

# Peak of the FP32 vector ALU of one MI355X: 256 CUs x 4 SIMDs x 32 lanes x
# 2 flops (FMA) x 2.4 GHz = 157.3 TFLOP/s.  Transcendentals (v_sin, v_cos,
# v_rcp) issue at a quarter of the FMA rate, so one costs the issue slots of
# 4 FMAs = 8 flops.
PEAK_TFLOPS = 157.3
TRANS_FLOP_EQ = 8.0
# Algorithmic work per frequency-triangle pair, counted from the closed forms
# (Eq. 7-8 forward; Eq. 9-10 and the indicator shape derivative for the
# gradient): FP32 flops (FMA = 2) and transcendentals.
ALG = {
    "fwd": {"flops": 36.0, "trans": 7.0},
    "vjp_volume": {"flops": 50.0, "trans": 9.0},
    "vjp_surface": {"flops": 80.0, "trans": 9.0},
}


def flop_eq(kind: str) -> float:
    a = ALG[kind]
    return a["flops"] + TRANS_FLOP_EQ * a["trans"]


def cpu_baseline(case, grid, sigma, mode, seconds: float):
    """The FP64 oracle (C direct sums, OpenMP) timed on a bounded sample of
    the same workload: all triangles against a random subset of the band's
    frequencies, forward and gradient."""
    from oracle import reference as ref
    ref.build()
    xi, h, band = ref.otf_and_band(grid, sigma)
    xb = xi[band]
    rng = np.random.default_rng(0)
    V = case.V.astype(np.float64) - np.asarray(grid.origin)
    F = case.F
    nt = F.shape[0]

    def run(nf):
        idx = rng.choice(len(xb), size=nf, replace=False)
        x = xb[idx]
        W = rng.standard_normal(nf) + 1j * rng.standard_normal(nf)
        t0 = time.perf_counter()
        ref.mesh_ft_raw(V, F, x, mode)
        t1 = time.perf_counter()
        ref.mesh_ft_vjp_raw(V, F, x, W, mode)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    run(8)   # warm-up (thread pool, page faults)
    nf, n_tot, tf_tot, tv_tot = 16, 0, 0.0, 0.0
    while tf_tot + tv_tot < seconds:
        per = (tf_tot + tv_tot) / n_tot if n_tot else None
        if per:   # grow towards the remaining budget, at most doubling
            nf = int(min(2 * nf, max(16, (seconds - tf_tot - tv_tot) / per)))
        nf = min(nf, len(xb))
        tf, tv = run(nf)
        n_tot, tf_tot, tv_tot = n_tot + nf, tf_tot + tf, tv_tot + tv
    pairs = n_tot * nt
    rate = pairs / (tf_tot + tv_tot)
    return {"value": rate, "unit": "pairs/s", "cores": ref.num_threads(), "kind": "oracle",
            "sample": f"{n_tot} of {len(xb)} band frequencies (random) x {nt} triangles, forward + gradient, "
                      f"{tf_tot + tv_tot:.1f} s (fwd {pairs / tf_tot:.3g} pairs/s, grad {pairs / tv_tot:.3g} pairs/s)"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["volume", "surface"], default="volume")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(each mesh or request is independent; see the design notes on sharding).", file=sys.stderr)
        return 2

    import torch

    import paper_2303_10440_amd as dm
    from workloads import configs

    mode = configs.VOLUME if args.mode == "volume" else configs.SURFACE
    case = configs.cfg3(mode)
    g = case.grid
    sigma = case.sigma
    dev = torch.device("cuda:0")
    h = dm.Handle(0)
    topo = h.topology(case.F, n_verts=len(case.V))
    V = torch.tensor(case.V, device=dev)
    G = torch.tensor(np.random.default_rng(0).standard_normal(g.n).astype(np.float32), device=dev)
    n_band = dm.band_size(h, g, sigma)
    nt = case.F.shape[0]
    pairs = float(n_band) * nt

    for _ in range(args.warmup):
        dm.render_vjp(h, V, topo, sigma, g, G, want_image=True)
    torch.cuda.synchronize()

    h.timing(True)
    h.timing_read(reset=True)
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for i in range(args.steps):
        evs[i][0].record(stream)
        dm.render_vjp(h, V, topo, sigma, g, G, want_image=True)
        evs[i][1].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    h.timing(False)
    kt = h.timing_read(reset=True)
    total_ms = t_start.elapsed_time(t_end)
    ms_step = total_ms / args.steps
    lat = np.array([a.elapsed_time(b) for a, b in evs])

    fwd_launch, fwd_ms, fwd_pairs = kt["fwd"]
    vjp_launch, vjp_ms, vjp_pairs = kt["vjp"]
    vkind = "vjp_volume" if mode == configs.VOLUME else "vjp_surface"
    sweeps = {
        "fwd": {"avg_ms": fwd_ms / max(fwd_launch, 1), "pairs_per_s": fwd_pairs / (fwd_ms * 1e-3),
                "flop_eq_per_pair": flop_eq("fwd")},
        "vjp": {"avg_ms": vjp_ms / max(vjp_launch, 1), "pairs_per_s": vjp_pairs / (vjp_ms * 1e-3),
                "flop_eq_per_pair": flop_eq(vkind)},
    }
    dom = "fwd" if fwd_ms >= vjp_ms else "vjp"
    dkind = "fwd" if dom == "fwd" else vkind
    launches = fwd_launch if dom == "fwd" else vjp_launch
    dms = (fwd_ms if dom == "fwd" else vjp_ms) / max(launches, 1)
    per_launch_pairs = (fwd_pairs if dom == "fwd" else vjp_pairs) / max(launches, 1)
    achieved = per_launch_pairs * flop_eq(dkind) / (dms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS, "traffic": None,
                "kernel": "k_fwd_sweep" if dom == "fwd" else "k_vjp_sweep",
                "avg_launch_ms": dms, "pairs_per_launch": per_launch_pairs,
                "flop_eq_per_pair": flop_eq(dkind)}

    out = {
        "metric": METRIC,
        "value": pairs / (ms_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single cell: SH-deformed icosphere-4 (2562 v, 5120 t), 128x128x64 grid, "
                               "0.2x0.2x0.5 um voxels, Gaussian PSF sigma (0.15, 0.15, 0.45) um, band OTF > 1e-3",
                   "mode": args.mode, "n_triangles": nt, "band_entries": n_band, "pairs_per_step": pairs,
                   "step": "dm_render_vjp: image + dL/dverts + dL/dSigma"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "min": float(lat.min())},
        "sweeps": sweeps,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, g, sigma, mode, args.cpu_seconds)
        out["cpu_baseline"]["gpu_over_cpu"] = out["value"] / out["cpu_baseline"]["value"]
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
