#!/usr/bin/env python3
"""Throughput of the micromagnetic Monte Carlo hot path on one MI355X.

A step is one full MMC sweep (paper Sec. II: one compound trial move per cell,
red then black colour pass), each colour pass preceded by a demag refresh
(FFT convolution with the cell-averaged tensor, Sec. III, Eq. 14), on the
1024x1024x4 grid of 5 nm cells at T = 0.9 Tc with 1 T applied along z.
Prints one JSON line: cell-updates/s, the roofline figure of the dominant
kernel (algorithmic bytes / HIP-event-timed launch duration) and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
KINDS = ["demag_xfwd", "demag_ypass", "demag_xinv", "colour_pass", "end_of_sweep"]


def pad_pow2(n, minimum=1):
    p = 1
    while p < 2 * n - 1:
        p *= 2
    return max(p, minimum)


def algorithmic_bytes(grid, demag, kind):
    """Minimum HBM bytes one launch of `kind` must move (FP32 data)."""
    nx, ny, nz = grid
    N = nx * ny * nz
    Px, Py = pad_pow2(nx, 2), pad_pow2(ny)
    L, S = Px // 2, 3 * nz
    spec = L * S * ny * 8                           # x-spectrum, complex FP32 (bins 0 and L share row 0)
    tensor = (L + 1) * (Py // 2 + 1) * 6 * nz * 4   # tensor spectrum, FP32
    if kind == "demag_xfwd":
        return 12 * N + spec                        # read m, write spectrum
    if kind == "demag_ypass":
        return 2 * spec + tensor                    # read + write spectrum, read tensor
    if kind == "demag_xinv":
        return spec + 12 * N // 2                   # read spectrum, write h of one colour
    if kind == "colour_pass":
        per = 12 + 12 + 12 + (12 if demag else 0)   # own m, other m, own write, own h
        return per * N // 2
    return 0


TRAFFIC_SOURCES_NOTE = "profiles/loop_1024x1024x4_traffic.json"


def counted_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, TRAFFIC_SOURCES_NOTE)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for p in rec["sources"]:
        fp = os.path.join(ROOT, p)
        if not os.path.exists(fp):
            return None
        h.update(open(fp, "rb").read())
    if h.hexdigest() != rec["source_sha256"] or kernel not in rec["bytes_per_launch"]:
        return None
    return rec["bytes_per_launch"][kernel]["total"]


def cpu_baseline(seconds_target=15.0):
    """The FP64 oracle (as it stands) on a 256x256x4 section of the same workload."""
    from oracle import oracle as O
    wl = workloads.WORKLOADS["loop_1024x1024x4"]
    mat = workloads.BASE_MATERIAL
    grid = (256, 256, 4)
    S = O.System(grid, wl["cell"], Ms0=mat["Ms0"], A0=mat["A0"], K1=mat["K1"], Tc=mat["Tc"], T=wl["T"],
                 B=wl["B"], demag=True, mf=mat["mf"])
    m = S.init_state("uniform")
    _ = S.plan                                       # tensor setup, not timed (as on the GPU side)
    S.run(m, 1, cone_deg=30, adapt_every=100)        # warm-up sweep
    n, t = 0, 0.0
    while t < seconds_target and n < 200:
        t0 = time.perf_counter()
        S.run(m, 2, sweep0=1 + n, cone_deg=30, adapt_every=100)
        t += time.perf_counter() - t0
        n += 2
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cells = int(np.prod(grid))
    return {"value": cells * n / t, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": "%d sweeps of a 256x256x4 section (same cell, material, T, field, demag on), %.1f s" % (n, t)}


def batched_leg(n_chains=64, sweeps=100, seed=0):
    """Independent chains of uneven size, T and field: one HIP-graph launch per
    call (batched) against the same chains run one after another (plain)."""
    import torch
    from paper_2106_05593_amd import Batch, Chain
    mat = workloads.BASE_MATERIAL
    params = workloads.batch_chain_params(n_chains, seed)

    def make():
        return [Chain(p["grid"], (5e-9,) * 3, Ms0=mat["Ms0"], A0=mat["A0"], K1=mat["K1"], Tc=mat["Tc"], T=p["T"],
                      B=p["B"], mf=mat["mf"], mu=mat["mu"], demag=True, adapt_every=100, seed=seed,
                      chain_id=p["chain_id"], init=0) for p in params]
    chains = make()
    cells = sum(int(np.prod(p["grid"])) for p in params)
    for c in chains:                                   # warm-up, one at a time
        c.sweep(2)
    for c in chains:
        c.sync()
    t0 = time.perf_counter()
    for c in chains:
        c.sweep(sweeps)
    for c in chains:
        c.sync()
    t_plain = time.perf_counter() - t0
    b = Batch(chains)
    b.sweep(sweeps)                                    # captures the graph (first call)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.sweep(sweeps)
    b.sync()
    t_batch = time.perf_counter() - t0
    b.close()
    for c in chains:
        c.close()
    scale = 1000.0 / sweeps                            # chains of 1000 sweeps each
    return {"chains": n_chains, "cells": cells, "timed_sweeps_per_chain": sweeps,
            "chains_per_s_batched": n_chains / (t_batch * scale), "chains_per_s_plain": n_chains / (t_plain * scale),
            "cell_updates_per_s_batched": cells * sweeps / t_batch, "cell_updates_per_s_plain": cells * sweeps / t_plain,
            "speedup": t_plain / t_batch}


def fe_film_leg(sweeps=100, warmup=5, every=10, seed=0):
    """The granular Fe film with cubic anisotropy (paper Fig. 5 problem, at 8
    of its 10 layers): per-cell colour pass with grain classes and the cubic
    term, demag refreshed once per sweep as in the paper.  Cell-updates/s and
    the HIP-event time of each kernel kind over the sampled sweeps."""
    import torch
    from paper_2106_05593_amd import Chain
    p = workloads.FE_FILM
    grid = p["grid"]
    N = int(np.prod(grid))
    gid, ng = workloads.voronoi_grains(grid, p["cell"], p["grain_spacing"], seed=7)
    ch = Chain(grid, p["cell"], Ms0=p["Ms0"], A0=p["A0"], K1=0.0, Tc=p["Tc"], T=p["T"], B=p["B"], demag=True,
               refresh_per_sweep=1, adapt_every=100, seed=seed, init=0, init_dir=p["init_dir"])
    ch.set_grains(gid, np.tile([0.0, 0.0, 1.0], (ng, 1)), np.zeros(ng), np.zeros(ng), np.full(ng, p["Tc"]),
                  p["bscale"])
    ch.set_anisotropy("cubic", np.array(p["cubic_axes"]), p["K1c"], p["K2c"], me_scaling=True)
    ch.sweep(warmup)
    ch.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms, cnt = ch.sweep_timed(sweeps, every=every)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ch.stats()
    assert st["sweeps"] == warmup + sweeps and np.isfinite(st["m2_mean"])
    kern = {}
    for k, name in enumerate(KINDS):
        if cnt[k]:
            avg = 1e3 * ms[k] / cnt[k]
            b = algorithmic_bytes(grid, True, name)
            if name == "colour_pass":
                b += 4 * N                                # class ids: the pass's cells and the other colour's
            kern[name] = {"launches": int(cnt[k]), "avg_us": round(avg, 3), "alg_bytes": b,
                          "GBs": round(b / (avg * 1e-6) / 1e9, 1)}
    ch.close()
    return {"workload": "fe_film_400x400x8", "grid": list(grid), "cell_nm": 2, "grains": int(ng),
            "demag_refresh_per_sweep": 1, "sweeps": sweeps, "ms_per_sweep": 1e3 * wall / sweeps,
            "cell_updates_per_s": N * sweeps / wall, "kernels": kern}


def profile_leg(sweeps=50, warmup=5, every=10, seed=0):
    """The benchmark grid under a Gaussian in-plane temperature profile (paper
    Sec. IV, laser heating): 16 temperature classes from 0.9 Tc at the rim to
    1.1 Tc at the centre (2 um between the 1/e points), each cell's move judged at
    its class's temperature; per-cell colour pass with class ids."""
    import torch
    from paper_2106_05593_amd import Chain
    wl = workloads.WORKLOADS["loop_1024x1024x4"]
    mat = workloads.BASE_MATERIAL
    grid = wl["grid"]
    N = int(np.prod(grid))
    cls, T_of = workloads.gaussian_temperature_classes(grid, wl["cell"], 2e-6, 1.1 * mat["Tc"], 0.9 * mat["Tc"], 16)
    n = len(T_of)
    ch = Chain(grid, wl["cell"], Ms0=mat["Ms0"], A0=mat["A0"], K1=mat["K1"], Tc=mat["Tc"], T=wl["T"], B=wl["B"],
               mf=mat["mf"], mu=mat["mu"], demag=True, adapt_every=wl["adapt_every"], seed=seed, init=0)
    ch.set_grains(cls, np.tile(mat["easy_axis"], (n, 1)), np.full(n, mat["K1"]), np.zeros(n), np.full(n, mat["Tc"]),
                  1.0)
    ch.set_grain_temperatures(T_of)
    ch.sweep(warmup)
    ch.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms, cnt = ch.sweep_timed(sweeps, every=every)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert np.isfinite(ch.stats()["m2_mean"])
    kern = {name: {"launches": int(cnt[k]), "avg_us": round(1e3 * ms[k] / cnt[k], 3)}
            for k, name in enumerate(KINDS) if cnt[k]}
    ch.close()
    return {"workload": "loop_1024x1024x4 + Gaussian temperature profile (16 classes, 0.9-1.1 Tc)",
            "sweeps": sweeps, "ms_per_sweep": 1e3 * wall / sweeps, "cell_updates_per_s": N * sweeps / wall,
            "kernels": kern}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-fe-film", action="store_true")
    ap.add_argument("--no-profile-leg", action="store_true")
    ap.add_argument("--profile-every", type=int, default=10,
                    help="bracket every kernel of one timed sweep in this many with HIP events")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 5}))
        return

    from paper_2106_05593_amd import Chain

    wl = workloads.WORKLOADS["loop_1024x1024x4"]
    mat = workloads.BASE_MATERIAL
    grid = wl["grid"]
    N = int(np.prod(grid))
    print("bench: creating %s chain (demag on)" % (grid,), file=sys.stderr, flush=True)
    ch = Chain(grid, wl["cell"], Ms0=mat["Ms0"], A0=mat["A0"], K1=mat["K1"], Tc=mat["Tc"], T=wl["T"], B=wl["B"],
               mf=mat["mf"], mu=mat["mu"], demag=True, adapt_every=wl["adapt_every"], cone_deg=wl["cone_deg"],
               seed=0, init=0)
    ch.sweep(args.warmup)
    ch.sync()
    torch.cuda.synchronize()
    print("bench: warm-up done, timing %d sweeps" % args.steps, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    # HIP events around each launch of every profile_every-th sweep (on the
    # chain's stream); the other sweeps run without instrumentation
    ms, cnt = ch.sweep_timed(args.steps, every=args.profile_every)   # synchronises the stream
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ch.stats()
    assert st["sweeps"] == args.warmup + args.steps and np.isfinite(st["m2_mean"])
    value = N * args.steps / wall

    per_kernel = {}
    for k, name in enumerate(KINDS):
        if cnt[k] == 0:
            continue
        avg_us = 1e3 * ms[k] / cnt[k]
        b = algorithmic_bytes(grid, True, name)
        per_kernel[name] = {"launches": int(cnt[k]), "avg_us": round(avg_us, 3), "total_ms": round(float(ms[k]), 3),
                            "alg_bytes": b, "GBs": round(b / (avg_us * 1e-6) / 1e9, 1) if b else None}
    dom = max(per_kernel, key=lambda n: per_kernel[n]["total_ms"])
    ach = per_kernel[dom]["GBs"]
    roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": counted_traffic(dom), "kernel": dom}
    sampled = (args.steps + args.profile_every - 1) // args.profile_every
    roofline["event_sampled_sweeps"] = sampled
    sweep_bytes = sum(algorithmic_bytes(grid, True, n) * int(cnt[k]) for k, n in enumerate(KINDS)) / sampled
    out = {
        "metric": "MC cell-updates/s at 1024x1024x4 w/ demag; batched chains/s vs plain, FP32",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "loop_1024x1024x4", "grid": list(grid), "cell_nm": 5, "T_K": wl["T"],
                   "mu0H_T": wl["B"][2], "demag_refresh_per_sweep": 2, "sweep_alg_bytes_per_cell": round(sweep_bytes / N, 1)},
        "roofline": roofline,
        "kernels": per_kernel,
    }
    if not args.no_batched:
        print("bench: batched chains leg", file=sys.stderr, flush=True)
        out["batched"] = batched_leg()
    if not args.no_fe_film:
        print("bench: granular Fe film leg (cubic anisotropy)", file=sys.stderr, flush=True)
        out["fe_film"] = fe_film_leg()
    if not args.no_profile_leg:
        print("bench: temperature-profile leg", file=sys.stderr, flush=True)
        out["temperature_profile"] = profile_leg()
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
