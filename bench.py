#!/usr/bin/env python3
"""Benchmark of the renderer's hot path on one MI355X.

One step = one dm_render_vjp call on the single-cell workload (deformed
icosphere, 5120 triangles, 128 x 128 x 64 grid of 0.2 x 0.2 x 0.5 um voxels,
Gaussian PSF sigma = (0.15, 0.15, 0.45) um, band OTF > 1e-3): mesh prep,
forward sweep over the band, OTF multiply and scatter, inverse FFT to the
image, FFT of dL/dI, adjoint weights and PSF gradient, gradient sweep and the
per-vertex reduction.  Inputs are resident in HBM before timing starts.

value = triangles x band entries / step time (each frequency-triangle pair is
evaluated once forward and once for the gradient per step; with dL/dI given
and the image wanted, dm_render_vjp does both in one fused sweep).

Besides the headline step the default run measures the 64-cell batch against
64 single calls (--no-batch skips it) and a short serving comparison of the
batched server against one call per mesh at a saturating arrival rate
(--no-serve-quick skips it); profiler runs of the headline kernels pass both.

Prints ONE JSON line.  Synthetic data (seeded); no dataset.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "tri·freq pairs/s fwd+VJP (5k tris, 128²×64) vs plain; p50/p99 render latency"

# Published peak of the FP32 vector ALU of one MI355X: 256 CUs x 4 SIMDs x
# 32 lanes x 2 flops (FMA) x 2.4 GHz = 157.3 TFLOP/s.
PEAK_TFLOPS = 157.3
TRANS_KINDS = ("sin", "cos", "rcp")
# Algorithmic work per frequency-triangle pair, counted from the closed forms
# as written (Eq. 7-8 forward: three vertex phase factors and one reciprocal;
# Eq. 9-10 and the indicator shape derivative for the gradient): FP32 flops
# (FMA = 2) and transcendentals by kind.  The sweeps share phase factors along
# triangle strips and so execute fewer transcendentals than this count; the
# count is the algorithm's, not the implementation's.
ALG = {
    "fwd": {"flops": 36.0, "sin": 3, "cos": 3, "rcp": 1},
    "vjp_volume": {"flops": 50.0, "sin": 3, "cos": 3, "rcp": 3},
    "vjp_surface": {"flops": 80.0, "sin": 3, "cos": 3, "rcp": 3},
}
# The fused sweep evaluates both per pair: its algorithmic work is the sum.
for _m in ("volume", "surface"):
    ALG["fused_" + _m] = {k: ALG["fwd"][k] + ALG["vjp_" + _m][k] for k in ALG["fwd"]}


# HBM traffic of the dominant kernel from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) over this benchmark, each
# divided by what the same counter reads for a plain device-to-device copy of
# known size.  Valid only for the kernel source it was measured on: if the
# hash of the kernel file differs, the benchmark reports traffic as null.
TRAFFIC = {
    "kernel": "k_fused_lanes<0>",
    "source_sha256": "4e39ea4322236879130b5040bfb8bfffc65d6c301a0794c01d8778abf2f487f0",
    # FETCH_SIZE 1,339,149 KiB x 2.000 (a 256 MiB copy reads 131,090 KiB) and
    # WRITE_SIZE 205,847 KiB x 1.000 (the copy writes 262,144 KiB), per launch
    # (mean of three launches each)
    "read_bytes": 1339149.0 * 1024 * 2.0,
    "write_bytes": 205846.7 * 1024 * 1.0,
    "profile": "profiles/k_fused_lanes_cfg3_volume.md",
}
TRAFFIC["bytes_per_launch"] = TRAFFIC["read_bytes"] + TRAFFIC["write_bytes"]


def kernel_source_sha256() -> str:
    import hashlib
    path = os.path.join(ROOT, "paper_2303_10440_amd", "csrc", "dm_kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel: str):
    if TRAFFIC is None or TRAFFIC["kernel"] != kernel or TRAFFIC["source_sha256"] != kernel_source_sha256():
        return None
    return TRAFFIC["bytes_per_launch"]


def flop_eq(kind: str, rates: dict) -> float:
    """FP32 flop-equivalents of one pair: its flops plus each transcendental
    priced at the measured cost of its kind, PEAK / (measured lane rate), so
    that pairs/s x flop_eq / PEAK is the fraction of the pair rate the ALU
    allows when flops and transcendentals share it (times add)."""
    a = ALG[kind]
    return a["flops"] + sum(a[t] * PEAK_TFLOPS * 1e12 / rates[t] for t in TRANS_KINDS)


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
    cores = ref.num_threads()
    # the same sample on one thread, for a fixed fraction of the budget
    ref.set_num_threads(1)
    try:
        n1 = max(2, int(n_tot * 0.25 / max(cores, 1)))
        t1f, t1v = run(n1)
    finally:
        ref.set_num_threads(cores)
    return {"value": rate, "unit": "pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_tot} of {len(xb)} band frequencies (random) x {nt} triangles, forward + gradient, "
                      f"{tf_tot + tv_tot:.1f} s (fwd {pairs / tf_tot:.3g} pairs/s, grad {pairs / tv_tot:.3g} pairs/s)",
            "one_thread": {"value": n1 * nt / (t1f + t1v), "unit": "pairs/s",
                           "sample": f"{n1} band frequencies x {nt} triangles, {t1f + t1v:.1f} s"},
            "cpu_model": cpu_model(), "affinity": len(os.sched_getaffinity(0))}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_sweeps(dm, reps: int = 10) -> dict:
    """The paper's mesh-transform benchmark shapes (its Sec. 5 figure), on the
    whole spectrum (band threshold 0, the exact transform), forward render
    only: (a) the 80-triangle icosphere over images of 32^3 ... 256^3 voxels,
    time and library memory; (b) a 100^3 image over icospheres of 320 ...
    20480 triangles, time against the triangle count."""
    import torch
    from workloads import configs
    h = dm.Handle(0)

    def time_render(case):
        topo = h.topology(case.F, n_verts=len(case.V))
        V = torch.tensor(case.V, device="cuda:0")
        dm.render(h, V, topo, case.sigma, case.grid)
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(s)
            dm.render(h, V, topo, case.sigma, case.grid)
            b.record(s)
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        n_band = float(dm.band_size(h, case.grid, case.sigma))
        return ms, n_band, case.F.shape[0]

    by_size = []
    for n in (32, 64, 128, 256):
        c = configs.sphere_case(sub=1, radius=0.3 * n, n=(n, n, n), tau=0.0)
        ms, nb, nt = time_render(c)
        by_size.append({"n": n, "n_triangles": nt, "entries": nb, "ms": ms, "pairs_per_s": nb * nt / (ms * 1e-3),
                        "library_bytes_cumulative": h.memory_in_use()})
    by_tris = []
    for sub in (2, 3, 4, 5):
        c = configs.sphere_case(sub=sub, radius=30.0, n=(100, 100, 100), tau=0.0)
        ms, nb, nt = time_render(c)
        by_tris.append({"n_triangles": nt, "entries": nb, "ms": ms, "pairs_per_s": nb * nt / (ms * 1e-3)})
    t = np.array([r["n_triangles"] for r in by_tris], float)
    m = np.array([r["ms"] for r in by_tris])
    slope, icpt = np.polyfit(t, m, 1)
    resid = float(np.max(np.abs(m - (slope * t + icpt)) / m))
    return {"workload": "icosphere (80 triangles) over cubic images 32^3..256^3, and a 100^3 image over "
                        "icospheres of 320..20480 triangles; unit voxels, sigma (1, 1, 2.5), full spectrum "
                        "(tau = 0), forward render, median of 10",
            "by_image_size": by_size, "by_triangles": by_tris,
            "linear_fit_ms": {"per_1k_triangles": slope * 1e3, "intercept": icpt, "max_rel_residual": resid}}


def bench_batch(dm, h, reps: int = 2) -> dict:
    """cfg4: 64 independent deformed cells (1k-20k triangles, grids 64^3 /
    96^3 / 128x128x64, sigma_z ~ U[1.5, 3]): one dm_batch_run for all of them
    against 64 dm_render_vjp calls in a row on the same stream."""
    import torch
    from workloads import configs
    cases = configs.cfg4()
    rng = np.random.default_rng(1)
    reqs, pairs = [], 0.0
    for c in cases:
        topo = h.topology(c.F, n_verts=len(c.V))
        V = torch.tensor(c.V, device="cuda:0")
        G = torch.tensor(rng.standard_normal(c.grid.n).astype(np.float32), device="cuda:0")
        reqs.append((V, topo, c.sigma, c.grid, G))
        pairs += float(dm.band_size(h, c.grid, c.sigma)) * c.F.shape[0]
    out_b = dm.batch_run(h, reqs)
    out_l = [dm.render_vjp(h, *r, want_image=True) for r in reqs]
    torch.cuda.synchronize()
    worst = max(float(((a[0] - b[2]).norm() / b[2].norm()).item()) for a, b in zip(out_b, out_l))
    s = torch.cuda.current_stream()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(s)
    for _ in range(reps):
        dm.batch_run(h, reqs)
    e1.record(s)
    for _ in range(reps):
        for r in reqs:
            dm.render_vjp(h, *r, want_image=True)
    e2.record(s)
    torch.cuda.synchronize()
    tb, tl = e0.elapsed_time(e1) / reps, e1.elapsed_time(e2) / reps
    # sweep-kernel pair rates: the persistent launch over all 64 cells against
    # the single calls' fused sweeps (launch events around each)
    h.timing(True)
    h.timing_read(reset=True)
    dm.batch_run(h, reqs)
    torch.cuda.synchronize()
    kb = h.timing_read(reset=True)["batch"]
    for r in reqs:
        dm.render_vjp(h, *r, want_image=True)
    torch.cuda.synchronize()
    kf = h.timing_read(reset=True)["fused"]
    h.timing(False)
    return {"workload": "64 deformed cells, n_t log-uniform [1k, 20k], grids {64^3, 96^3, 128x128x64}, "
                        "sigma_xy = 1, sigma_z ~ U[1.5, 3] voxels, forward + gradient, all in one persistent "
                        "launch per density",
            "pairs": pairs, "batched_ms": tb, "looped_ms": tl, "batched_pairs_per_s": pairs / (tb * 1e-3),
            "looped_pairs_per_s": pairs / (tl * 1e-3), "speedup": tl / tb, "max_image_rel_diff": worst,
            "persistent_sweep": {"launches": kb[0], "ms": kb[1], "pairs_per_s": kb[2] / (kb[1] * 1e-3)},
            "single_call_sweeps": {"launches": kf[0], "ms": kf[1], "pairs_per_s": kf[2] / (kf[1] * 1e-3)}}


def bench_fit(dm, h, case, mode, shape_steps: int = 10, psf_steps: int = 4) -> dict:
    """Staggered fitting on the single-cell workload: the target is the cell
    rendered with sigma (0.15, 0.15, 0.45) um; the fit starts from the cell
    shrunk by 3% about its centroid and a PSF 20% too wide, and times shape
    steps (narrow band, weighted L2, Adam on the vertices) and PSF steps
    (full spectrum, plain L2, Adam on (sigma_xy, sigma_z))."""
    import torch
    from paper_2303_10440_amd import fit
    g = case.grid
    s_xy, s_z = float(np.sqrt(case.sigma[0])), float(np.sqrt(case.sigma[2]))
    dev = torch.device("cuda:0")
    topo = h.topology(case.F, n_verts=len(case.V))
    target = dm.render(h, torch.tensor(case.V, device=dev), topo, case.sigma, g)
    c = case.V.mean(0)
    V = torch.tensor((c + 0.97 * (case.V - c)).astype(np.float32), device=dev)
    F = fit.StaggeredFit(h, topo, V, 1.2 * s_xy, 1.2 * s_z, g, target,
                         fit.FitConfig(lr_shape=0.005, lr_psf=0.005))
    F.shape_step()
    F.psf_step()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(s)
    for _ in range(shape_steps):
        F.shape_step()
    e1.record(s)
    for _ in range(psf_steps):
        F.psf_step()
    e2.record(s)
    torch.cuda.synchronize()
    # the paper's vertex update: uniform Adam on the Laplacian-filtered gradient
    Vs = torch.tensor((c + 0.97 * (case.V - c)).astype(np.float32), device=dev)
    Fs = fit.StaggeredFit(h, topo, Vs, s_xy, s_z, g, target,
                          fit.FitConfig(lr_shape=0.005, optimizer="adam_uniform", smooth_lambda=50.0))
    Fs.shape_step()
    torch.cuda.synchronize()
    e3, e4 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e3.record(s)
    for _ in range(shape_steps):
        Fs.shape_step()
    e4.record(s)
    torch.cuda.synchronize()
    n_band = float(dm.band_size(h, g, case.sigma))
    n_full = float(dm.band_size(h, dataclasses.replace(g, tau=0.0), case.sigma))
    ts, tp = e0.elapsed_time(e1) / shape_steps, e1.elapsed_time(e2) / psf_steps
    losses = [l for k, l in F.history]
    return {"workload": "single-cell fit: shape steps on the band OTF > 1e-3, PSF steps on the full "
                        "spectrum (tau = 0), start 3% shrunk and PSF 20% wide",
            "shape_step_ms": ts, "psf_step_ms": tp,
            "shape_step_smoothed_uniform_adam_ms": e3.elapsed_time(e4) / shape_steps,
            "shape_pairs_per_s": n_band * case.F.shape[0] / (ts * 1e-3),
            "psf_pairs_per_s": n_full * case.F.shape[0] / (tp * 1e-3),
            "band_entries": n_band, "full_spectrum_entries": n_full,
            "first_shape_loss": losses[0], "last_shape_loss": [l for k, l in F.history if k == "shape"][-1],
            "psf": [float(x) for x in F.psf]}


def bench_foam(dm, steps: int = 20) -> dict:
    """The multi-cell workload: a cluster of 8 cells sharing their walls
    (4608 faces, 2169 vertices) in the single-cell grid (128 x 128 x 64 of
    0.2 x 0.2 x 0.5 um, sigma (0.15, 0.15, 0.45) um, band OTF > 1e-3), as the
    paper's double-membrane surface density and as a piecewise-constant
    indicator density (cell densities U[0.5, 1.5]); one dm_render_vjp per
    step."""
    import torch
    from workloads import configs
    h = dm.Handle(0)
    out = {}
    for mode, key in ((configs.SURFACE, "surface"), (configs.VOLUME, "volume")):
        c = configs.foam_case(mode)
        topo = h.topology(c.F, n_verts=len(c.V))
        topo.set_weights(c.extra["tri_w"])
        V = torch.tensor(c.V, device="cuda:0")
        G = torch.tensor(np.random.default_rng(0).standard_normal(c.grid.n).astype(np.float32), device="cuda:0")
        for _ in range(3):
            dm.render_vjp(h, V, topo, c.sigma, c.grid, G, want_image=True)
        torch.cuda.synchronize()
        s_ = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s_)
        for _ in range(steps):
            dm.render_vjp(h, V, topo, c.sigma, c.grid, G, want_image=True)
        e1.record(s_)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        pairs = float(dm.band_size(h, c.grid, c.sigma)) * c.F.shape[0]
        out[key] = {"ms_per_step": ms, "pairs_per_step": pairs, "pairs_per_s": pairs / (ms * 1e-3)}
    out["workload"] = ("8-cell cluster (cube foam 2x2x2, 8x8 squares per cell face, rounded), 4608 faces, "
                       "walls once; 128x128x64 grid, 0.2x0.2x0.5 um, sigma (0.15, 0.15, 0.45) um, fwd + gradient")
    return out


def bench_otf(dm, case, steps: int = 20) -> dict:
    """The single-cell workload with a tabulated PSF instead of the Gaussian:
    an aberrated OTF table (envelope widths 0.3 / 0.9 um, a defocus-like
    phase and a missing cone), band |OTF| > 1e-3 rebuilt on every call; one
    dm_render_otf_vjp (image + dL/dverts) per step."""
    import torch
    from workloads import psfs
    h = dm.Handle(0)
    g = case.grid
    otf_full = psfs.aberrated_otf(g, 0.3, 0.9, defocus=0.8, cone=1.5)
    otf = torch.tensor(psfs.half_spectrum(otf_full), device="cuda:0")
    topo = h.topology(case.F, n_verts=len(case.V))
    V = torch.tensor(case.V, device="cuda:0")
    G = torch.tensor(np.random.default_rng(0).standard_normal(g.n).astype(np.float32), device="cuda:0")
    for _ in range(3):
        dm.render_otf_vjp(h, V, topo, otf, g, G, want_image=True)
    torch.cuda.synchronize()
    s_ = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s_)
    for _ in range(steps):
        dm.render_otf_vjp(h, V, topo, otf, g, G, want_image=True)
    e1.record(s_)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    re, im = otf.real.double(), otf.imag.double()
    n_pos = int(((re * re + im * im) > float(np.float32(g.tau)) ** 2).sum().item())
    return {"workload": "single cell, tabulated aberrated OTF (defocus phase, missing cone), fwd + gradient",
            "ms_per_step": ms, "band_positions": n_pos, "n_triangles": int(case.F.shape[0]),
            "pairs_per_s": n_pos * case.F.shape[0] / (ms * 1e-3)}


def bench_smooth(dm, reps: int = 20) -> dict:
    """The shape step's Laplacian filter (I + 50 L)^{-2} g (dm_laplace_smooth)
    on the single-cell mesh (2562 vertices) and a 20252-vertex geodesic
    sphere, random gradient, relative residual 1e-6 per solve; the FP64
    oracle (two sparse direct solves per column, scipy) timed beside it."""
    import torch
    from oracle import smoothing as S
    from workloads import configs, meshes
    h = dm.Handle(0)
    out = []
    c3 = configs.cfg3()
    Vg, Fg = meshes.geodesic_sphere(45)
    for name, F, nv in (("cfg3 cell", c3.F, len(c3.V)), ("geodesic-45 sphere", Fg, len(Vg))):
        topo = h.topology(F, n_verts=nv)
        g = torch.tensor(np.random.default_rng(0).standard_normal((nv, 3)).astype(np.float32), device="cuda:0")
        o, info = dm.laplace_smooth(h, topo, g, lam=50.0, tol=1e-6, with_info=True)
        torch.cuda.synchronize()
        s_ = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s_)
        for _ in range(reps):
            dm.laplace_smooth(h, topo, g, lam=50.0, tol=1e-6, out=o)
        e1.record(s_)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gd = g.cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        want = S.laplace_smooth(F, nv, gd, 50.0)
        t_cpu = time.perf_counter() - t0
        err = float(np.linalg.norm(o.cpu().numpy() - want) / np.linalg.norm(want))
        its = info["iters"][0] + info["iters"][1]
        out.append({"mesh": name, "n_verts": nv, "ms": ms,
                    "solver": "CG, one workgroup" if nv <= 3072 else "Chebyshev, one launch per step",
                    "iterations": list(info["iters"]), "residuals": list(info["residual"]),
                    "us_per_iteration": ms * 1e3 / max(its, 1), "rel_err_vs_oracle": err,
                    "oracle_ms": t_cpu * 1e3})
    return {"workload": "(I + 50 L)^{-2} g, L the edge-graph Laplacian, random g, relative residual 1e-6 per "
                        "solve: Jacobi-preconditioned CG in one workgroup up to 3072 vertices, Chebyshev "
                        "iteration with a priori step counts above", "cases": out}


def bench_serve(dm, rate: float, count: int, warmup: int, max_batch: int, max_inflight: int, pool: int = 32,
                seed: int = 0, abba: bool = False) -> dict:
    """cfg5: Poisson arrivals of forward + gradient requests on resident cells
    (n_t log-uniform [500, 40k], grids {64^3, 128^3, 256x256x128}); latency is
    submission to completion as seen by the server.  With abba the trace is
    replayed batched, plain, plain, batched and each mode reports the mean of
    its two replays (slow drifts of the device's clocks cancel)."""
    import torch
    from workloads import configs
    cases, t_arr, idx, widx = configs.cfg5_pooled(seed, count, rate, pool, warmup)
    h = dm.Handle(0)
    rng = np.random.default_rng(2)
    Gs = [torch.tensor(rng.standard_normal(c.grid.n).astype(np.float32), device="cuda:0") for c in cases]
    pairs_of = [float(dm.band_size(h, c.grid, c.sigma)) * c.F.shape[0] for c in cases]

    def run(mb, mi):
        srv = dm.Server(0, max_batch=mb, max_inflight=mi)
        ids = [srv.mesh_add(c.V, c.F) for c in cases]

        def submit(i):
            c = cases[i]
            img = torch.empty(c.grid.n, device="cuda:0")
            dv = torch.empty((len(c.V), 3), device="cuda:0")
            ds = torch.empty(6, device="cuda:0")
            return srv.submit(ids[i], c.sigma, c.grid, Gs[i], img, dv, ds), (img, dv, ds)

        keep = [submit(int(i)) for i in widx]
        for t, _ in keep:
            srv.poll(t)
        torch.cuda.synchronize()
        subs, keep, t0 = [], [], time.perf_counter()
        for k in range(count):
            while time.perf_counter() - t0 < t_arr[k]:
                pass
            ts = time.perf_counter() - t0
            tk, bufs = submit(int(idx[k]))
            subs.append((tk, ts))
            keep.append(bufs)
        res = [(srv.poll(tk), ts) for tk, ts in subs]
        st = srv.stats()
        srv.close()
        lat = np.array([r["total_ms"] for r, _ in res])
        done = max(ts * 1e3 + r["total_ms"] for r, ts in res)
        span_s = (done - subs[0][1] * 1e3) * 1e-3
        pairs = sum(pairs_of[int(i)] for i in idx)
        late = max(ts - t_arr[k] for k, (_, ts) in enumerate(subs))
        return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "throughput_rps": count / span_s, "pairs_per_s": pairs / span_s,
                "mean_batch": float(st["mean_batch"]), "batches": int(st["batches"]),
                "max_submit_lateness_ms": 1e3 * float(late),
                "ok": all(r["status"] == 0 for r, _ in res)}

    out = {"workload": f"{count} Poisson requests at {rate:g}/s on a pool of {pool} resident cells "
                       "(n_t log-uniform [500, 40k], grids {64^3, 128^3, 256x256x128}, own PSF per cell), "
                       "forward + gradient each",
           "rate": rate, "offered_pairs_per_s": rate * float(np.mean([pairs_of[int(i)] for i in idx]))}
    order = ("batched", "plain", "plain", "batched") if abba else ("batched", "plain")
    runs = {"batched": [], "plain": []}
    for mode in order:
        r = run(max_batch, max_inflight) if mode == "batched" else run(1, 1)
        runs[mode].append(r)
        print(f"serve {rate:g}/s {mode}: {r}", file=sys.stderr, flush=True)
    for mode, rs in runs.items():
        if len(rs) == 1:
            out[mode] = rs[0]
        else:
            m = {k: float(np.mean([r[k] for r in rs])) for k in ("p50_ms", "p99_ms", "mean_ms", "throughput_rps",
                                                                  "pairs_per_s", "mean_batch")}
            m["ok"] = all(r["ok"] for r in rs)
            m["replays"] = rs
            out[mode] = m
    out["throughput_gain"] = out["batched"]["throughput_rps"] / out["plain"]["throughput_rps"]
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["volume", "surface"], default="volume")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", action=argparse.BooleanOptionalAction, default=True,
                    help="the 64-cell batched vs looped comparison (on by default)")
    ap.add_argument("--serve-quick", action=argparse.BooleanOptionalAction, default=True,
                    help="a short serving comparison at a saturating rate: 300 requests at 100/s "
                         "(on by default; --serve gives the full per-rate sweep)")
    ap.add_argument("--sweeps", action="store_true",
                    help="add the paper's mesh-transform benchmark shapes (image size, triangle count)")
    ap.add_argument("--otf", action="store_true",
                    help="add the single-cell workload with a tabulated (aberrated) PSF")
    ap.add_argument("--foam", action="store_true",
                    help="add the 8-cell cluster (per-face density weights) in both densities")
    ap.add_argument("--smooth", action="store_true",
                    help="add the shape step's Laplacian filter on the cell and a 20k-vertex sphere")
    ap.add_argument("--fit", action="store_true",
                    help="add the staggered shape / PSF fitting steps on the single-cell workload")
    ap.add_argument("--serve", type=float, nargs="*", default=None,
                    help="add the serving comparison at these arrival rates (req/s)")
    ap.add_argument("--serve-count", type=int, default=1000)
    ap.add_argument("--serve-warmup", type=int, default=50)
    ap.add_argument("--serve-abba", action="store_true",
                    help="replay each serving trace batched, plain, plain, batched and report per-mode means")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device-to-device copy (reference for HBM byte counters)")
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
    from paper_2303_10440_amd import probe
    rates = probe.alu_rates()

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

    msuf = "volume" if mode == configs.VOLUME else "surface"
    kinds = {"fwd": ("k_fwd_lanes", "fwd"), "vjp": ("k_vjp_lanes", "vjp_" + msuf),
             "fused": ("k_fused_lanes", "fused_" + msuf)}
    sweeps = {}
    for key, (kn, alg) in kinds.items():
        n_l, ms_sum, prs = kt[key]
        if n_l == 0:
            continue
        sweeps[key] = {"kernel": kn + ("<0>" if mode == configs.VOLUME else "<1>"), "launches_per_step": n_l / args.steps,
                       "avg_ms": ms_sum / n_l, "pairs_per_s": prs / (ms_sum * 1e-3),
                       "flop_eq_per_pair": flop_eq(alg, rates),
                       "frac": prs / (ms_sum * 1e-3) * flop_eq(alg, rates) / (PEAK_TFLOPS * 1e12)}
    # the dominant kernel: the sweep with the largest share of the step
    dom = max(sweeps, key=lambda k: kt[k][1])
    dkind = kinds[dom][1]
    launches, dms_sum, dpairs = kt[dom]
    dms = dms_sum / launches
    per_launch_pairs = dpairs / launches
    achieved = per_launch_pairs * flop_eq(dkind, rates) / (dms * 1e-3) / 1e12
    kname = sweeps[dom]["kernel"]
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS, "traffic": measured_traffic(kname),
                "kernel": kname,
                "avg_launch_ms": dms, "pairs_per_launch": per_launch_pairs,
                "flop_eq_per_pair": flop_eq(dkind, rates),
                "algorithmic_per_pair": ALG[dkind],
                "measured_lane_rates_per_s": {k: rates[k] for k in ("fma",) + TRANS_KINDS},
                "mix_time_over_sum": rates["mix_over_sum"]}

    # The two sweeps apart, as autograd runs them (dm_render with the band
    # spectrum, then dm_render_vjp reusing it: forward sweep, then the
    # gradient sweep alone), timed by the same launch events.
    n_sep = max(3, min(10, args.steps))
    h.timing(True)
    h.timing_read(reset=True)
    for _ in range(n_sep):
        _, spec = dm.render(h, V, topo, sigma, g, spectrum=True)
        dm.render_vjp(h, V, topo, sigma, g, G, spectrum_in=spec)
    torch.cuda.synchronize()
    h.timing(False)
    kt2 = h.timing_read(reset=True)
    separate = {}
    for key in ("fwd", "vjp"):
        kn, alg = kinds[key]
        n_l, ms_sum, prs = kt2[key]
        if n_l:
            separate[key] = {"kernel": kn + ("<0>" if mode == configs.VOLUME else "<1>"), "launches": n_l,
                             "avg_ms": ms_sum / n_l, "pairs_per_s": prs / (ms_sum * 1e-3),
                             "flop_eq_per_pair": flop_eq(alg, rates),
                             "frac": prs / (ms_sum * 1e-3) * flop_eq(alg, rates) / (PEAK_TFLOPS * 1e12)}

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
        "separate_sweeps": separate,
        "roofline": roofline,
    }
    if args.copy_calibration:
        x = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 256 << 20
    if args.batch:
        out["batched"] = bench_batch(dm, h)
    if args.fit:
        out["fit"] = bench_fit(dm, h, case, mode)
    if args.sweeps:
        out["sweeps_paper_shapes"] = bench_sweeps(dm)
    if args.smooth:
        out["smooth"] = bench_smooth(dm)
    if args.foam:
        out["foam"] = bench_foam(dm)
    if args.otf:
        out["otf"] = bench_otf(dm, case)
    if args.serve_quick:
        out["serving_quick"] = bench_serve(dm, 100.0, 300, 30, 16, 2)
    if args.serve is not None:
        out["serving"] = [bench_serve(dm, r, args.serve_count, args.serve_warmup, 16, 2, abba=args.serve_abba)
                          for r in (args.serve or [200.0])]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, g, sigma, mode, args.cpu_seconds)
        out["cpu_baseline"]["gpu_over_cpu"] = out["value"] / out["cpu_baseline"]["value"]
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
