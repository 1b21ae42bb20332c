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
KINDS = ["demag_xfwd", "demag_ypass", "demag_xinv", "colour_pass", "end_of_sweep", "fused_pass"]


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
    if kind == "fused_pass":
        return 2 * spec + 12 * N + 6 * N            # spectrum in and out, m read, own colour written
    if kind == "fused_pass_half":
        return spec + 12 * N + 6 * N                # spectrum in, m read, own colour written
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


def host_cpu():
    """CPU model, logical CPUs and physical cores of this host (from /proc/cpuinfo)."""
    model, cores, logical = None, set(), 0
    phys = core = None
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "processor":
                logical += 1
            elif k == "model name" and model is None:
                model = v
            elif k == "physical id":
                phys = v
            elif k == "core id":
                core = v
            elif not k and phys is not None and core is not None:
                cores.add((phys, core))
                phys = core = None
        if phys is not None and core is not None:
            cores.add((phys, core))
    except OSError:
        pass
    return {"model": model, "logical_cpus": logical or os.cpu_count(), "physical_cores": len(cores) or None}


def _omp_threads(n):
    """Set the OpenMP thread count of the oracle library (it links libgomp)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except OSError:
        return False


def cpu_baseline(seconds_target=15.0):
    """The FP64 oracle (as it stands) on a 256x256x4 section of the same
    workload (same cell, material, T, field, demag), timed with all host
    threads and with one thread."""
    from oracle import oracle as O
    wl = workloads.WORKLOADS["loop_1024x1024x4"]
    mat = workloads.BASE_MATERIAL
    grid = (256, 256, 4)
    S = O.System(grid, wl["cell"], Ms0=mat["Ms0"], A0=mat["A0"], K1=mat["K1"], Tc=mat["Tc"], T=wl["T"],
                 B=wl["B"], demag=True, mf=mat["mf"])
    m = S.init_state("uniform")
    _ = S.plan                                       # tensor setup, not timed (as on the GPU side)
    cells = int(np.prod(grid))
    cpu = host_cpu()
    threads_all = int(os.environ.get("OMP_NUM_THREADS", cpu["logical_cpus"] or 1))

    def rate(threads, budget, sweep0):
        _omp_threads(threads)
        S.run(m, 1, sweep0=sweep0, cone_deg=30, adapt_every=100)        # warm-up sweep
        n, t = 0, 0.0
        while t < budget and n < 200:
            t0 = time.perf_counter()
            S.run(m, 2, sweep0=sweep0 + 1 + n, cone_deg=30, adapt_every=100)
            t += time.perf_counter() - t0
            n += 2
        return cells * n / t, n, t
    v_all, n_all, t_all = rate(threads_all, seconds_target, 0)
    v_one, n_one, t_one = rate(1, max(2.0, seconds_target / 3), 1000)
    _omp_threads(threads_all)
    return {"value": v_all, "unit": "cell-updates/s", "cores": threads_all, "kind": "oracle",
            "sample": "%d sweeps of a 256x256x4 section (same cell, material, T, field, demag on) in %.1f s with %d "
                      "threads; %d sweeps in %.1f s with 1 thread" % (n_all, t_all, threads_all, n_one, t_one),
            "value_1thread": v_one, "cpu_model": cpu["model"], "logical_cpus": cpu["logical_cpus"],
            "physical_cores": cpu["physical_cores"]}


def cpu_batched(n_chains=64, sweeps=1000, seed=0):
    """The FP64 oracle on the batched workload's chains: for each chain shape,
    one chain of that shape (its own T and field) timed over 2 sweeps after a
    warm-up sweep with all host threads (tensor setup not timed), then every
    chain's `sweeps` sweeps extrapolated linearly from its shape's time per
    sweep."""
    from oracle import oracle as O
    mat = workloads.BASE_MATERIAL
    params = workloads.batch_chain_params(n_chains, seed)
    cpu = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", cpu["logical_cpus"] or 1))
    _omp_threads(threads)
    per_sweep, timed = {}, 0.0
    for p in params:
        g = tuple(p["grid"])
        if g in per_sweep:
            continue
        S = O.System(g, (5e-9,) * 3, Ms0=mat["Ms0"], A0=mat["A0"], K1=mat["K1"], Tc=mat["Tc"], T=p["T"], B=p["B"],
                     demag=True, mf=mat["mf"], chain_id=p["chain_id"], seed=seed)
        m = S.init_state("uniform")
        _ = S.plan
        S.run(m, 1, sweep0=0, cone_deg=30, adapt_every=100)
        t0 = time.perf_counter()
        S.run(m, 2, sweep0=1, cone_deg=30, adapt_every=100)
        dt = time.perf_counter() - t0
        timed += dt
        per_sweep[g] = dt / 2
    total = sum(per_sweep[tuple(p["grid"])] for p in params) * sweeps
    cells = sum(int(np.prod(p["grid"])) for p in params)
    return {"chains_per_s": n_chains / total, "cell_updates_per_s": cells * sweeps / total, "threads": threads,
            "kind": "oracle", "seconds_per_sweep": {"x".join(map(str, g)): round(t, 4) for g, t in per_sweep.items()},
            "sample": "2 sweeps of one chain per shape (%.1f s with %d threads), every chain's %d sweeps extrapolated "
                      "linearly" % (timed, threads, sweeps)}


def batched_leg(n_chains=64, sweeps=1000, seed=0):
    """Independent chains of uneven size, T and field (64 chains drawn from
    64^2x1, 128^2x1, 256^2x2, 512^2x2 cells of 5 nm, T in [0.2, 1.2] Tc, Hz in
    [-0.5, 0.5] T, demag on), `sweeps` sweeps each: one batch call (one HIP
    graph launch) against the same chains run one at a time (each chain's
    sweeps, then a synchronisation, then the next chain)."""
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
        c.sync()
    t0 = time.perf_counter()
    for c in chains:
        c.sweep(sweeps)
        c.sync()
    t_plain = time.perf_counter() - t0
    b = Batch(chains)
    b.sweep(sweeps)                                    # schedule choice and graph capture (first call)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.sweep(sweeps)
    b.sync()
    t_batch = time.perf_counter() - t0
    used, trial = b.schedule()
    b.close()
    for c in chains:
        c.close()
    return {"chains": n_chains, "cells": cells, "sweeps_per_chain": sweeps, "schedule": used,
            "chains_per_s_batched": n_chains / t_batch, "chains_per_s_plain": n_chains / t_plain,
            "cell_updates_per_s_batched": cells * sweeps / t_batch, "cell_updates_per_s_plain": cells * sweeps / t_plain,
            "speedup": t_plain / t_batch}


def granular_leg(sweeps=5000, warmup=5, every=100, seed=0):
    """Granular medium (512x512x8 cells of 3 nm; 3-D Voronoi grains of 10 nm
    mean seed spacing; per-grain easy axis within 10 deg of z, Ku 0.7 MJ/m^3,
    Tc ~ N(700 K, 35 K); exchange across grain boundaries x0.1; 600 K; demag
    before each colour pass) with the y-direction DFT stages in FP32 and as
    split BF16 / FP16 matrix products: cell-updates/s per precision, the
    y-pass time, the relative L2 difference of the demag field of one state
    from the FP32 field, and <m> after the timed sweeps."""
    import torch
    from paper_2106_05593_amd import Chain
    wl = workloads.WORKLOADS["granular_512x512x8"]
    mat = workloads.BASE_MATERIAL
    grid, cell = wl["grid"], wl["cell"]
    N = int(np.prod(grid))
    gid, ng = workloads.voronoi_grains(grid, cell, 10e-9, seed=4)
    ea, K1, K2, Tc = workloads.grain_properties(ng, seed=5)
    m_probe = workloads.random_state(N, seed=6)
    out = {"workload": "granular_512x512x8", "grains": int(ng), "sweeps": sweeps, "modes": {}}
    h_ref = None
    for mode in ("fp32", "split_bf16", "split_fp16"):
        ch = Chain(grid, cell, Ms0=mat["Ms0"], A0=mat["A0"], K1=0.0, Tc=mat["Tc"], T=wl["T"], B=wl["B"],
                   mf=mat["mf"], mu=mat["mu"], demag=mode, adapt_every=100, seed=seed, init=1)
        ch.set_grains(gid, ea, K1, K2, Tc, 0.1)
        state = ch.get_m()
        ch.set_m(m_probe)
        h = ch.demag_field().astype(np.float64)
        if h_ref is None:
            h_ref = h
        ch.set_m(state)
        ch.sweep(warmup)
        ch.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms, cnt = ch.sweep_timed(sweeps, every=every)
        wall = time.perf_counter() - t0
        st = ch.stats()
        out["modes"][mode] = {"cell_updates_per_s": N * sweeps / wall, "ms_per_sweep": 1e3 * wall / sweeps,
                              "ypass_us": round(1e3 * ms[1] / cnt[1], 2),
                              "field_rel_l2_vs_fp32": float(np.linalg.norm(h - h_ref) / np.linalg.norm(h_ref)),
                              "m_mean": [round(v, 6) for v in st["m_mean"]], "m2_mean": round(st["m2_mean"], 6)}
        ch.close()
    return out


def dmi_film_leg(sweeps=10000, seed=0):
    """DMI thin film with demag (256x256x1 cells of 4x4x2 nm, D0 1.5 mJ/m^2,
    T 0.5 Tc, zero field, random start): `sweeps` sweeps, wall time and
    cell-updates/s."""
    import torch
    from paper_2106_05593_amd import Chain
    wl = workloads.WORKLOADS["film_256x256x1"]
    mat = workloads.BASE_MATERIAL
    grid = wl["grid"]
    N = int(np.prod(grid))
    ch = Chain(grid, wl["cell"], Ms0=mat["Ms0"], A0=mat["A0"], K1=mat["K1"], D0=wl["D0"], Tc=mat["Tc"], T=wl["T"],
               B=wl["B"], mf=mat["mf"], mu=mat["mu"], demag=True, adapt_every=100, seed=seed, init=1)
    ch.sweep(5)
    ch.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.sweep(sweeps)
    ch.sync()
    wall = time.perf_counter() - t0
    st = ch.stats()
    ch.close()
    return {"workload": "film_256x256x1", "sweeps": sweeps, "wall_s": wall, "cell_updates_per_s": N * sweeps / wall,
            "m2_mean": st["m2_mean"]}


def loop_leg(temperatures=(630.0, 770.0), sweeps_per_point=200, seed=0):
    """The hysteresis-loop workload as a whole: 1024x1024x4 cells of 5 nm with
    demag, field along z from +1 T to -1 T in 0.01 T steps and back (401
    points), 200 sweeps per point, the point's value the mean of sweeps
    101-200 (FP64 means of every sweep), at each temperature: loop wall time
    and cell-updates/s over the whole loop."""
    import torch
    from paper_2106_05593_amd import Chain
    wl = workloads.WORKLOADS["loop_1024x1024x4"]
    mat = workloads.BASE_MATERIAL
    grid = wl["grid"]
    N = int(np.prod(grid))
    fields = np.concatenate([np.linspace(1.0, -1.0, 201), np.linspace(-0.99, 1.0, 200)])
    out = {"workload": "loop_1024x1024x4", "points": len(fields), "sweeps_per_point": sweeps_per_point, "runs": {}}
    for T in temperatures:
        ch = Chain(grid, wl["cell"], Ms0=mat["Ms0"], A0=mat["A0"], K1=mat["K1"], Tc=mat["Tc"], T=T, B=(0, 0, 1.0),
                   mf=mat["mf"], mu=mat["mu"], demag=True, adapt_every=100, seed=seed, init=0)
        ch.sweep(2)
        ch.sync()
        torch.cuda.synchronize()
        half = sweeps_per_point // 2
        mz = []
        t0 = time.perf_counter()
        for i, b in enumerate(fields):
            ch.set_field((0.0, 0.0, float(b)))
            ch.sweep(half)
            ch.take_averages()                   # drops the first half
            ch.sweep(sweeps_per_point - half)
            avg, n = ch.take_averages()
            mz.append(avg[2])
            if i % 50 == 0:
                print("bench: loop T=%.0f K point %d/%d" % (T, i, len(fields)), file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        ch.close()
        sweeps = len(fields) * sweeps_per_point
        out["runs"]["%.0f K" % T] = {"wall_s": wall, "sweeps": sweeps, "cell_updates_per_s": N * sweeps / wall,
                                     "mz_at_+1T": mz[0], "mz_at_-1T": mz[200], "mz_at_0T_down": mz[100],
                                     "mz_at_0T_up": mz[300]}
    return out


def fe_film_leg(sweeps=100, warmup=5, every=10, seed=0, nz=10):
    """The granular Fe film with cubic anisotropy (paper Fig. 5 problem: 400 x
    400 cells of 2 nm, nz layers, 10 of them in the paper): per-cell colour
    pass with grain classes and the cubic term, demag refreshed once per sweep
    as in the paper.  Cell-updates/s and the HIP-event time of each kernel kind
    over the sampled sweeps."""
    import torch
    from paper_2106_05593_amd import Chain
    p = workloads.FE_FILM
    grid = (p["grid"][0], p["grid"][1], nz)
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
    return {"workload": "fe_film_400x400x%d" % nz, "grid": list(grid), "cell_nm": 2, "grains": int(ng),
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
    ap.add_argument("--no-granular", action="store_true")
    ap.add_argument("--granular-sweeps", type=int, default=5000,
                    help="sweeps per precision in the granular leg")
    ap.add_argument("--no-dmi-film", action="store_true")
    ap.add_argument("--loop-leg", action="store_true", help="also run the whole 401-point loop at 630 K and 770 K")
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

    def make_chain():
        return Chain(grid, wl["cell"], Ms0=mat["Ms0"], A0=mat["A0"], K1=mat["K1"], Tc=mat["Tc"], T=wl["T"], B=wl["B"],
                     mf=mat["mf"], mu=mat["mu"], demag=True, adapt_every=wl["adapt_every"], cone_deg=wl["cone_deg"],
                     seed=0, init=0)
    # one-time set-up, outside the timed sweeps: the first chain of a shape
    # computes the tensor spectrum and runs the tile and colour-pass tuners; a
    # second one reuses both (cached per shape in the process)
    t0 = time.perf_counter()
    ch = make_chain()
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    make_chain().close()
    t_second = time.perf_counter() - t0
    setup = {"create_s": round(t_first, 3), "create_same_shape_s": round(t_second, 3),
             "what": "first chain: mean field, Newell tensor and its spectrum (FP64, host), device buffers, initial "
                     "state, x-tile and colour-pass tuners; a second chain of the shape reuses the spectrum and the "
                     "tuners' choices"}
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
    form = ch.tuning()[2]                       # colour-pass form chosen at creation (0, 1 or 2)
    kinds = KINDS[:5] + (["fused_pass_half"] if form == 2 else ["fused_pass"])
    for k, name in enumerate(kinds):
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
    if roofline["traffic"]:                     # counted bytes over the same launch time
        tg = roofline["traffic"] / (per_kernel[dom]["avg_us"] * 1e-6) / 1e9
        roofline["traffic_GBs"], roofline["traffic_frac"] = round(tg, 1), round(tg / HBM_PEAK_GBS, 4)
    sampled = (args.steps + args.profile_every - 1) // args.profile_every
    roofline["event_sampled_sweeps"] = sampled
    sweep_bytes = sum(algorithmic_bytes(grid, True, n) * int(cnt[k]) for k, n in enumerate(kinds)) / sampled
    out = {
        "metric": "MC cell-updates/s at 1024x1024x4 w/ demag; batched chains/s vs plain, FP32",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "loop_1024x1024x4", "grid": list(grid), "cell_nm": 5, "T_K": wl["T"],
                   "mu0H_T": wl["B"][2], "demag_refresh_per_sweep": 2, "sweep_alg_bytes_per_cell": round(sweep_bytes / N, 1)},
        "roofline": roofline,
        "kernels": per_kernel,
        "tuning": {"x_rows_per_thread": list(ch.tuning()[0]), "colour_pass_form": form},
        "setup": setup,
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
    if not args.no_granular:
        print("bench: granular 512x512x8 leg (FP32 and split demag stages)", file=sys.stderr, flush=True)
        out["granular"] = granular_leg(sweeps=args.granular_sweeps)
    if not args.no_dmi_film:
        print("bench: DMI film leg", file=sys.stderr, flush=True)
        out["dmi_film"] = dmi_film_leg()
    if args.loop_leg:
        print("bench: whole-loop leg", file=sys.stderr, flush=True)
        out["loop"] = loop_leg()
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        if "batched" in out:
            print("bench: timing the CPU oracle on the batched chains", file=sys.stderr, flush=True)
            out["batched"]["cpu_oracle"] = cpu_batched()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
