#!/usr/bin/env python3
"""Throughput of the hot path on one MI355X: cutoff pair-interactions/s.

One step = pi_bin (cell ids, counts, prefix sum, stable scatter) followed by
pi_interact (27-cell sweep, compensated FP32, with the FP64 invariant
reductions) over a system already resident in HBM.  The default workload is
2^24 uniform particles in the unit cube, r_c = 1/256, 256^3 cells (one
particle per cell).  value = ordered cutoff pairs per step / step time.

    python bench.py [--steps K] [--warmup W] [--workload scale_1ppc]

Prints one JSON line.  Per-kernel device times come from the library's own
hipEvent timing (pi_timing_*), recorded on the launch stream: first a
breakdown run of min(K, 20) steps with every launch timed (the per-kernel
table and the stage times; it also names the dominant kernel), then the K
timed steps with events around the dominant kernel's launches only, since
each timed launch adds two event records to the stream (about 0.1 ms per
step over the 13 launches of a step).  The roofline's duration is that
kernel's mean over the timed steps.  The CPU baseline is the FP64 oracle
(oracle/) timed on the host.

The same line carries the rest of the metric: `batch` (512 independent
systems in one captured graph launch against one launch per system) and
`serve` (the request server: saturation and one-at-a-time rates, and
p50/p99 latency under Poisson arrivals at fixed rates); --no-batch and
--no-serve skip them.
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

METRIC = "cutoff pair-interactions/s at 1 ppc (16.8M particles); p99 latency at fixed QPS"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3

# Algorithmic FLOPs of the sweep (FMA = 2; add, mul, sqrt, rcp, rsq = 1;
# compares and integer work not counted): every candidate pays 3 sub + 1 mul
# + 2 FMA = 8; every accepted pair pays about 22 on the plain path (sqrt, q,
# W, W' with a reciprocal, the weighted terms and 1 + 3 accumulating FMAs),
# 12 more with compensated accumulation (3 per accumulator), and about 19
# more where q > 1/2 for the cancellation-free 1 - q, which is 7/8 of the
# pairs of a uniform distribution (the shell volume beyond half the cutoff).
FLOP_PER_CANDIDATE = 8.0
FLOP_PER_PAIR = {"plain": 22.0, "compensated": 34.0 + 19.0 * 7.0 / 8.0,
                 "fp64acc": 34.0 + 19.0 * 7.0 / 8.0}

WORKLOADS = {
    "scale_1ppc": ("uniform 2^24 particles, unit cube, r_c=1/256, 256^3 cells (1 ppc)", "scale_1ppc"),
    "scale_8ppc": ("uniform 2^24 particles, unit cube, r_c=1/128, 128^3 cells (8 ppc)", "scale_8ppc"),
    "clustered": ("2^23 particles, 64 Gaussian blobs + 10% uniform, r_c=1/128, 128^3 cells", "clustered"),
    "tiny": ("uniform 32768 particles, unit cube, r_c=1/32, 32^3 cells", "tiny"),
    "dense_64ppc": ("uniform 2^21 particles, unit cube, r_c=1/32, 32^3 cells (64 ppc)", "dense_64ppc"),
}


def algorithmic_bytes(name: str, n: int, nc: int, orig_order: bool) -> float:
    """Compulsory HBM bytes of one launch: every input read once, every output
    written once, at 4 bytes per int32/float32 element."""
    if name == "k_fill_i32":
        return 4.0 * nc
    if name == "k_radix_hist":
        return 4.0 * n                                # one key per particle (12 B on the first pass)
    if name == "k_radix_scatter":
        return 48.0 * n                               # records in and out (40 B on the first pass)
    if name == "k_cell_ranges":
        return 4.0 * n + 8.0 * nc                     # sorted ids in; counts and offsets out
    if name.startswith("k_sweep"):
        # sorted x, y, z, w in (16 B), rho, G and count out (20 B), one
        # offset per cell (4 B); the original-order scatter reads perm
        return 36.0 * n + 4.0 * nc + (4.0 * n if orig_order else 0.0)
    return 0.0


def kernel_key(name: str) -> str:
    """Common key for a kernel's library timing name and its rocprofv3 name:
    the base name plus the first three template arguments, if any."""
    import re
    m = re.search(r"(k_[a-z0-9_]+)(?:<([^>]*)>)?", name)
    if not m:
        return name
    base, targs = m.group(1), m.group(2)
    if targs:
        return base + "<" + ",".join(t.strip() for t in targs.split(",")[:3]) + ">"
    return base


def source_hash() -> str:
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2406_16091_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _profile_value(tag: str, pattern: str, kernel: str, inv: bool):
    """Value of the `tag` line for `kernel` in the committed summaries
    profiles/`pattern`, or None if none matches the current kernel sources.
    Among the template instances that match, the one with the invariant
    reduction on (and not the batch form) is preferred when `inv` is set,
    since that is the instance the timed step launches."""
    import glob
    want, cur = kernel_key(kernel), source_hash()
    found = []
    for p in sorted(glob.glob(os.path.join(ROOT, "profiles", pattern))):
        with open(p) as f:
            for line in f:
                if line.startswith(tag + " "):
                    parts = line.split()
                    name, val, h = " ".join(parts[1:-2]), parts[-2], parts[-1]
                    key = kernel_key(name)
                    # (a timing name without template arguments matches
                    # every instance of its kernel)
                    if (key == want or ("<" not in want and key.split("<")[0] == want)) and h == cur:
                        found.append((name, float(val)))
    if not found:
        return None
    if inv:
        for name, val in found:
            if name.replace(" ", "").endswith(",true,false>"):
                return val
    return found[0][1]


def measured_traffic(kernel: str, inv: bool = True):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summaries (profiles/traffic_*.md: FETCH_SIZE and WRITE_SIZE scaled by a
    copy kernel's), or None if none matches the current kernel sources."""
    return _profile_value("TRAFFIC", "traffic_*.md", kernel, inv)


def measured_valu_issue(kernel: str, inv: bool = True):
    """Microseconds of VALU issue per launch of `kernel` (SQ_INSTS_VALU x 4
    cycles over the 1024 SIMDs at 2.4 GHz) from the committed counter
    summaries (profiles/sqcounters_*.md), or None."""
    return _profile_value("VALUISSUE", "sqcounters_*.md", kernel, inv)


def candidates_from_counts(counts: np.ndarray, dims) -> int:
    """Sum over targets of sources in the clipped 27-cell stencil, minus self
    (measurement bookkeeping for the FLOP count)."""
    from scipy import ndimage
    c = counts.reshape(dims[2], dims[1], dims[0]).astype(np.int64)
    nb = ndimage.convolve(c, np.ones((3, 3, 3), np.int64), mode="constant", cval=0)
    return int((c * nb).sum() - c.sum())


def cpu_baseline(system, budget_s: float = 30.0):
    import oracle
    t0 = time.perf_counter()
    b = oracle.bin_particles(system.x, system.y, system.z, system.w, system.origin, system.dims,
                             system.cell_w, system.rc)
    t_bin = time.perf_counter() - t0
    n = system.n
    # sweep over all targets if the estimate fits the budget, else a subsample
    from paper_2406_16091_amd import synth
    probe = synth.subsample(n, min(n, 200_000), seed=20)
    t0 = time.perf_counter()
    oracle.sweep(system.x, system.y, system.z, system.w, system.dims, system.rc, b, targets=probe)
    t_probe = time.perf_counter() - t0
    est = t_probe * n / max(len(probe), 1)
    if t_bin + est <= budget_s:
        targets, label = None, f"full workload: bin + sweep of all {n} targets"
    else:
        m = int(len(probe) * (budget_s - t_bin) / max(t_probe, 1e-9))
        m = max(10_000, min(n, m))
        targets = synth.subsample(n, m, seed=20)
        label = f"bin all {n} + sweep of {m} sampled targets (pairs scaled by {n}/{m})"
    t0 = time.perf_counter()
    o = oracle.sweep(system.x, system.y, system.z, system.w, system.dims, system.rc, b, targets=targets)
    t_sweep = time.perf_counter() - t0
    pairs = float(o.count.sum())
    if targets is not None:
        # time per full step = bin + sweep scaled to all targets
        frac = len(targets) / n
        t_sweep /= frac
        pairs /= frac
    value = pairs / (t_bin + t_sweep)
    return {"value": value, "unit": "pairs/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": label, "bin_s": round(t_bin, 3), "sweep_s": round(t_sweep, 3)}


def bench_batch(steps: int, warmup: int, sweep: str = "auto"):
    """512 independent systems (N log-uniform in [1e3, 2e5], 1-4 per cell):
    one pi_batch_run (one captured hipGraph launch per step) against the
    plain path of pi_bin + pi_interact per system on the same stream."""
    import torch
    from paper_2406_16091_amd import device, pi, synth

    systems = synth.batch_systems()
    n_total = sum(s.n for s in systems)
    stream = torch.cuda.Stream()
    # plain path: one resident system object per system
    singles = [device.DeviceSystem(s) for s in systems]
    torch.cuda.synchronize()

    def plain_step():
        for d in singles:
            d.bin(stream=stream)
            d.interact(sweep=sweep, invariants=True, stream=stream)

    for _ in range(warmup):
        plain_step()
    stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plain_step()
    stream.synchronize()
    t_plain = (time.perf_counter() - t0) / steps
    pairs_plain = sum(d.invariants()["pairs"] for d in singles)
    del singles

    db = device.DeviceBatch(systems)
    torch.cuda.synchronize()
    stream.wait_stream(torch.cuda.current_stream())
    for _ in range(max(warmup, 1)):
        db.run(sweep=sweep, stream=stream)   # the first call captures the graph
    stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        db.run(sweep=sweep, stream=stream)
    stream.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    db.sync(stream)
    pairs = sum(v["pairs"] for v in db.invariants())
    assert pairs == pairs_plain, "batched and per-system pair totals differ"
    return {"systems": len(systems), "particles": n_total, "pairs_per_step": pairs,
            "batched_ms_per_step": round(t_batch * 1e3, 4),
            "batched_pairs_per_s": round(pairs / t_batch, 1),
            "one_system_per_launch_ms_per_step": round(t_plain * 1e3, 4),
            "one_system_per_launch_pairs_per_s": round(pairs / t_plain, 1),
            "speedup": round(t_plain / t_batch, 2)}


def _fresh_requests(pool, count, rng, sweeps, first_seed):
    """`count` requests drawn from the pool of distinct systems, each a fresh
    particle set: a random one of the 48 symmetries of its cube (axis
    permutation and mirror images v -> (g - 2^-16) - v, exact on the 2^-16
    lattice), and its own displacement seed."""
    from paper_2406_16091_amd import pi, synth
    lat = 2.0 ** -16
    out = []
    for k in range(count):
        s = pool[int(rng.integers(len(pool)))]
        axes = [s.x, s.y, s.z]
        order = rng.permutation(3)
        flip = rng.random(3) < 0.5
        top = np.float32(s.dims[0] - lat)
        v = [(top - axes[a]).astype(np.float32) if f else axes[a] for a, f in zip(order, flip)]
        t = synth.System(s.name, v[0], v[1], v[2], s.w, s.origin, s.dims, s.cell_w, s.rc)
        out.append(pi.make_request(t, n_sweeps=sweeps, jitter_sigma=0.1 * s.rc, lattice=lat,
                                   seed=first_seed + k))
    return out


def bench_serve(n_pool: int = 48, sweeps: int = 8, seconds: float = 3.0, loads=(0.5, 0.8), seed: int = 5,
                n_closed: int = 24, n_lo: float = 1e4, n_hi: float = 4e6, max_slots: int = 64, n_streams: int = 4):
    """Serving: requests of N log-uniform in [n_lo, n_hi] particles (uniform or
    8-blob clustered, 1/2/4/8 per cell), each swept `sweeps` times with
    Gaussian displacements of 0.1 r_c between sweeps.  Every submission is a
    fresh particle set (_fresh_requests); no request is submitted twice.
    Measures the saturation rate (n_closed requests submitted at once), the
    one-request-at-a-time rate on the same requests, and p50/p99 latency
    (submit to results in host memory) under Poisson arrivals at fractions of
    the saturation rate.  AUTO requests take the tuner's cached choice for
    their class or the static rule; the server never runs timed trials."""
    import torch
    from paper_2406_16091_amd import device, pi, synth

    pool = synth.serve_requests(n_pool, seed=seed, n_lo=n_lo, n_hi=n_hi)
    rng = np.random.default_rng(seed)
    ctx = device.Context.get(0).handle
    torch.cuda.synchronize()
    next_seed = [100_000]

    def fresh(count, systems=None):
        r = _fresh_requests(systems or pool, count, rng, sweeps, next_seed[0])
        next_seed[0] += count
        return r

    # a server is warmed once with the largest systems it may see, one per
    # slot, so that its device buffers and pinned staging have their final
    # sizes before anything is measured (a serving engine sizes its slots
    # for the largest admissible request)
    largest = [max(pool, key=lambda t: t.n)]

    def run_all(server, reqs):
        t0 = time.perf_counter()
        tickets = [pi.pi_submit(server, r) for r in reqs]
        pairs = 0
        for t in tickets:
            r = pi.pi_wait(server, t, copy=False)
            pairs += r["pairs_total"]
            pi.pi_release(server, t)
        return time.perf_counter() - t0, pairs

    # the closed-loop comparison: the same fresh requests through a one-slot
    # server (one request at a time) and through the full server
    closed = fresh(n_closed)
    one = pi.pi_server_create(ctx, max_slots=1, n_streams=1)
    run_all(one, fresh(2, largest))
    t_seq, pairs_seq = run_all(one, closed)
    pi.pi_server_destroy(one)

    server = pi.pi_server_create(ctx, max_slots=max_slots, n_streams=n_streams)
    run_all(server, fresh(n_streams, largest))
    run_all(server, fresh(n_closed))
    t_sat, pairs_sat = run_all(server, closed)
    assert pairs_sat == pairs_seq, "a request's results depend on what runs beside it"
    rate_sat = len(closed) / t_sat
    out = {"request_particles": [n_lo, n_hi], "max_slots": max_slots, "lanes": n_streams,
           "distinct_systems": n_pool, "fresh_request_sets": True, "closed_loop_requests": n_closed,
           "sweeps_per_request": sweeps, "mean_particles": float(np.mean([s.n for s in pool])),
           "saturation_requests_per_s": round(rate_sat, 2),
           "saturation_pairs_per_s": round(pairs_sat / t_sat, 1),
           "one_at_a_time_requests_per_s": round(len(closed) / t_seq, 2),
           "one_at_a_time_pairs_per_s": round(pairs_seq / t_seq, 1),
           "speedup_over_one_at_a_time": round(t_seq / t_sat, 2), "loads": []}
    del closed
    for f in loads:
        lam = f * rate_sat
        reqs = fresh(int(lam * seconds * 1.3) + 8)
        t_start = time.perf_counter()
        next_t = t_start
        k = 0
        pending = {}
        lat, pairs, refused = [], 0, 0
        waits, runs, sizes = [], [], []
        while True:
            now = time.perf_counter()
            if now - t_start < seconds and now >= next_t and k < len(reqs):
                t_client = time.perf_counter()
                st, tk = pi.pi_submit_status(server, reqs[k])
                if st == pi.PI_OK:
                    pending[tk] = (t_client, int(reqs[k].n))
                else:
                    refused += 1
                k += 1
                next_t += rng.exponential(1.0 / lam)
                continue
            for tk in list(pending):
                r = pi.pi_poll(server, tk, copy=False)
                if r["done"]:
                    t_client, nk = pending.pop(tk)
                    lat.append(time.perf_counter() - t_client)
                    waits.append(r["t_start"] - r["t_submit"])
                    runs.append(r["t_done"] - r["t_start"])
                    sizes.append(nk)
                    pairs += r["pairs_total"]
                    pi.pi_release(server, tk)
            if (now - t_start >= seconds or k >= len(reqs)) and not pending:
                break
            time.sleep(0.0002)
        wall = time.perf_counter() - t_start
        lat_ms = np.array(lat) * 1e3

        def pct(v_ms, q):
            return round(float(np.percentile(v_ms, q)), 3) if len(v_ms) else None
        wait_ms, run_ms = np.array(waits) * 1e3, np.array(runs) * 1e3
        small = lat_ms[np.array(sizes) <= np.median(sizes)] if len(sizes) else lat_ms
        out["loads"].append({"load": f, "offered_requests_per_s": round(lam, 2), "completed": len(lat),
                             "refused": refused, "p50_ms": pct(lat_ms, 50), "p99_ms": pct(lat_ms, 99),
                             "p50_admission_wait_ms": pct(wait_ms, 50), "p99_admission_wait_ms": pct(wait_ms, 99),
                             "p50_on_gpu_ms": pct(run_ms, 50), "p99_on_gpu_ms": pct(run_ms, 99),
                             "p99_ms_smaller_half": pct(small, 99),
                             "pairs_per_s": round(pairs / wall, 1)})
        del reqs
    pi.pi_server_destroy(server)
    return out


# Table 1 of the paper (Sec. 7.2): seconds per call of its Lennard-Jones
# kernel (21 FLOP per interaction as Sec. 7.1 counts it) for the no-LDS
# sweep (Par-Part-NoLoop) and the X-pencil on an A100 and an MI210, per
# (d, particles per cell).  Context only: other GPUs.
PAPER_TABLE1_S = {
    (2, 1): (1.0e-05, 1.1e-05, 8.6e-06, 6.9e-06), (4, 1): (2.0e-05, 1.2e-05, 2.9e-05, 1.9e-05),
    (8, 1): (2.8e-05, 1.9e-05, 4.3e-05, 4.1e-05), (16, 1): (3.7e-05, 2.0e-05, 1.4e-04, 9.8e-05),
    (32, 1): (4.2e-05, 3.8e-05, 6.3e-04, 2.3e-04), (2, 10): (3.4e-05, 1.8e-05, 3.2e-05, 4.2e-05),
    (4, 10): (7.2e-05, 4.6e-05, 1.4e-04, 7.8e-05), (8, 10): (9.1e-05, 5.6e-05, 4.6e-04, 4.6e-04),
    (16, 10): (1.0e-04, 8.1e-05, 2.2e-03, 1.8e-04), (32, 10): (4.2e-04, 4.0e-04, 9.2e-04, 1.2e-03),
    (2, 100): (1.6e-04, 1.2e-04, 4.2e-04, 2.7e-04), (4, 100): (5.2e-04, 3.7e-04, 3.9e-03, 2.1e-03),
    (8, 100): (6.1e-04, 6.1e-04, 7.8e-03, 5.3e-03), (16, 100): (3.2e-03, 3.2e-03, 1.2e-02, 8.0e-03),
    (32, 100): (2.5e-02, 2.5e-02, 5.1e-02, 5.3e-02),
}
# FLOP per interaction of the three kernels as this library evaluates them
# (FMA = 2; rcp = 1): Lennard-Jones: differences 3, softened s^2 6 (three
# FMA), rcp 1, times sigma^2 1, u^3 2, 4 e0 (u^6 - u^3) 3, accumulation 1 =
# 17; low-FLOP: 3 sub, 2 add, accumulation 1 = 6; high-FLOP: 17 + 150.
PAIRFN_FLOP = {"lj": 17.0, "lowflop": 6.0, "highflop": 167.0}


def bench_table1(calls: int = 200, min_s: float = 0.05, kernels=("lj", "lowflop", "highflop")):
    """The paper's timing experiment on MI355X: d^3 cells (d = 2 .. 32) with
    1, 10 or 100 particles per cell, uniform in the unit cube, cell width =
    r_c = 1/d; every candidate pair of the 27-cell stencil evaluated with the
    Lennard-Jones kernel (plain FP32 sums, no invariants, as the paper times
    it) and the low-/high-FLOP kernels of Fig. 8.  Time per call = wall time
    of `calls` back-to-back asynchronous calls / calls (Sec. 7.1), fewer calls
    (at least 10) once they pass min_s seconds."""
    import torch
    from paper_2406_16091_amd import device, synth

    rows = []
    for p in (1, 10, 100):
        for d in (2, 4, 8, 16, 32):
            s = synth.uniform_unit_cube(d ** 3 * p, -int(round(np.log2(d))), seed=900 + d + p, name=f"t1-{d}-{p}")
            ds = device.DeviceSystem(s)
            ds.bin()
            ds.sync()
            cand = candidates_from_counts(ds.binned()["counts"], s.dims)
            row = {"d": d, "ppc": p, "n": s.n, "candidates_per_particle": round(cand / s.n, 2),
                   "paper_A100_nolds_pencil_s": PAPER_TABLE1_S[(d, p)][:2],
                   "paper_MI210_nolds_pencil_s": PAPER_TABLE1_S[(d, p)][2:]}
            for kind in kernels:
                for sweep in ("nolds", "pencil", "subbox", "auto"):
                    def call():
                        ds.interact_pairfn(kind, "plain", sweep, "sorted", (0, 0, 0), invariants=False)
                    for _ in range(3):
                        call()
                    torch.cuda.synchronize()
                    k = 0
                    t0 = time.perf_counter()
                    while k < calls:
                        call()
                        k += 1
                        if k >= 10 and k % 10 == 0:
                            torch.cuda.synchronize()
                            if time.perf_counter() - t0 >= min_s:
                                break
                    torch.cuda.synchronize()
                    t = (time.perf_counter() - t0) / k
                    row[f"{kind}_{sweep}_s"] = float(f"{t:.4g}")
                    if sweep == "auto":
                        row[f"{kind}_auto_candidate_pairs_per_s"] = float(f"{cand / t:.4g}")
                        row[f"{kind}_auto_tflops"] = round(cand * PAIRFN_FLOP[kind] / t / 1e12, 3)
            ds.sync()
            ds.close()
            rows.append(row)
            print(f"[bench] table1 d={d} ppc={p}: lj auto {row['lj_auto_s']:.3g} s/call", file=sys.stderr,
                  flush=True)
    return rows


def bench_step(system, steps: int = 20, warmup: int = 3):
    """Time stepping on the headline workload: one pi_step = the sweep
    (compensated, AUTO), the symplectic Euler update with the B-spline as a
    soft pair potential, and the incremental re-binning; velocities
    N(0, (0.05 w)^2) per axis, dt = 0.25, kappa = 0.02 r_c^5, positions kept
    on the 2^-24 lattice.  Reports the step time and the kernels' times, the
    re-binning (update + offsets scan + placement) beside a full pi_bin."""
    import torch
    from paper_2406_16091_amd import device, pi

    ds = device.DeviceSystem(system)
    ctx = ds.ctx.handle
    ds.bin()
    rng = np.random.default_rng(77)
    vel = [rng.normal(0, 0.05 * system.cell_w, system.n).astype(np.float32) for _ in range(3)]
    ds.set_velocity(*vel)
    opts = pi.make_step_opts(0.25, 0.02 * system.rc ** 5, 2.0 ** -24)
    for _ in range(warmup):
        pi.pi_step(ctx, ds.cells, opts, ds.inv)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pi.pi_step(ctx, ds.cells, opts, ds.inv)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ds.sync()
    pi.pi_timing_reset(ctx)
    pi.pi_timing_only(ctx, None)
    pi.pi_timing_enable(ctx, True)
    for _ in range(steps):
        pi.pi_step(ctx, ds.cells, opts, ds.inv)
    for _ in range(steps):
        ds.bin()
    torch.cuda.synchronize()
    pi.pi_timing_enable(ctx, False)
    kt = pi.pi_timing_read(ctx)
    ds.close()
    per = {k: round(v[1] * 1e3 / steps, 2) for k, v in kt.items()}
    rebin = sum(v for k, v in per.items() if k.startswith(("k_step_", "k_scan_")))
    full = sum(v for k, v in per.items() if k.startswith(("k_radix", "k_digit", "k_cell_ranges", "k_max")))
    return {"workload": "the headline system, stepped", "ms_per_step": round(ms, 4),
            "update_and_incremental_rebin_us": round(rebin, 2), "full_pi_bin_us": round(full, 2),
            "kernels_us": per}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="scale_1ppc", choices=sorted(WORKLOADS))
    ap.add_argument("--sweep", default="auto")
    ap.add_argument("--tile", default="0,0,0")
    ap.add_argument("--precision", default="compensated")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="do not record per-kernel events")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the request server (saturation, one-at-a-time, Poisson p50/p99)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 512-system batch (graph launch vs one launch per system)")
    ap.add_argument("--no-step", action="store_true",
                    help="skip the time-stepping measurement (sweep + update + incremental re-binning)")
    ap.add_argument("--no-table1", action="store_true",
                    help="skip the paper's timing grid (Lennard-Jones and Fig. 8 kernels on d^3 cells)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes 5 times "
                         "(reference kernel for scaling HBM traffic counters), then exit")
    args = ap.parse_args()

    if args.copy_probe > 0:
        import torch
        a = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "copies": 5}))
        return

    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the library has no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch
    from paper_2406_16091_amd import device, pi, synth

    desc, gen = WORKLOADS[args.workload]
    print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
    system = getattr(synth, gen)()
    ds = device.DeviceSystem(system)
    ctx = ds.ctx.handle
    tile = tuple(int(v) for v in args.tile.split(","))

    def step():
        ds.bin()
        ds.interact(precision=args.precision, sweep=args.sweep, tile=tile, invariants=True)

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    ds.sync()
    torch.cuda.synchronize()

    # breakdown: every launch timed, over a run of its own
    kt, dom_name, nbreak = {}, None, min(args.steps, 20)
    if not args.no_timing:
        pi.pi_timing_reset(ctx)
        pi.pi_timing_only(ctx, None)
        pi.pi_timing_enable(ctx, True)
        for _ in range(nbreak):
            step()
        torch.cuda.synchronize()
        pi.pi_timing_enable(ctx, False)
        kt = pi.pi_timing_read(ctx)
        dom_name = max(kt.items(), key=lambda kv: kv[1][1])[0]
        print(f"[bench] breakdown over {nbreak} steps; dominant kernel {dom_name}", file=sys.stderr, flush=True)

    # timed steps: events around the dominant kernel only
    pi.pi_timing_reset(ctx)
    if dom_name is not None:
        pi.pi_timing_only(ctx, dom_name)
        pi.pi_timing_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pi.pi_timing_enable(ctx, False)
    ds.sync()
    kdom = pi.pi_timing_read(ctx) if dom_name is not None else {}
    pi.pi_timing_only(ctx, None)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.4f} ms/step", file=sys.stderr, flush=True)

    inv = ds.invariants()
    pairs = inv["pairs"]
    b = ds.binned()
    n, nc = system.n, system.n_cells
    cand = candidates_from_counts(b["counts"], system.dims)
    value = pairs / (ms_per_step * 1e-3)

    kernels = {k: {"launches": v[0], "avg_us": round(v[1] * 1e3 / max(v[0], 1), 3)} for k, v in kt.items()}
    roof = None
    stages = {}
    if kt and dom_name in kdom:
        name, (launches, total_ms) = dom_name, kdom[dom_name]
        avg_s = total_ms * 1e-3 / launches
        by = algorithmic_bytes(name, n, nc, False)
        if name.startswith("k_sweep"):
            flops = FLOP_PER_CANDIDATE * cand + FLOP_PER_PAIR[args.precision] * pairs
            t_hbm = by / (HBM_PEAK_GBS * 1e9)
            t_alu = flops / (FP32_PEAK_TFLOPS * 1e12)
            bound = "hbm" if t_hbm >= t_alu else "alu"
        else:
            flops, bound = 0.0, "hbm"
        traffic = measured_traffic(name)
        if bound == "hbm":
            ach = by / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": name,
                    "avg_us": round(avg_s * 1e6, 2), "algorithmic_bytes": by,
                    "algorithmic_flops": flops}
        else:
            ach = flops / avg_s / 1e12
            roof = {"bound": "alu", "achieved": round(ach, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(ach / FP32_PEAK_TFLOPS, 4), "traffic": traffic, "kernel": name,
                    "avg_us": round(avg_s * 1e6, 2), "algorithmic_flops": flops, "algorithmic_bytes": by}
        roof["traffic_over_algorithmic_bytes"] = round(traffic / by, 3) if traffic and by else None
        if flops:
            roof["fp32_frac_of_157TF"] = round(flops / avg_s / 1e12 / FP32_PEAK_TFLOPS, 4)
        # the VALU issue time the committed instruction counters give for the
        # kernel, against its measured time: near 1 means bound by VALU issue
        issue = measured_valu_issue(name)
        roof["valu_issue_us"] = round(issue, 1) if issue else None
        roof["valu_issue_over_time"] = round(issue / (avg_s * 1e6), 3) if issue else None
        bin_us = sum(v[1] for k, v in kt.items() if not k.startswith(("k_sweep", "k_inv"))) * 1e3 / nbreak
        sw = [(k, v) for k, v in kt.items() if k.startswith("k_sweep")]
        sweep_us = sum(v[1] for _, v in sw) * 1e3 / nbreak
        bin_bytes = 40.0 * n + 8.0 * nc
        stages = {"bin_us": round(bin_us, 2), "sweep_us": round(sweep_us, 2),
                  "bin_hbm_frac_algorithmic": round(bin_bytes / (bin_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                  "sweep_fp32_frac": round((FLOP_PER_CANDIDATE * cand + FLOP_PER_PAIR[args.precision] * pairs)
                                           / (sweep_us * 1e-6) / 1e12 / FP32_PEAK_TFLOPS, 4)}

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "n_cells": nc, "rc": system.rc,
                   "layout": "inputs SoA; sorted cell-relative positions kept as one float4 (x, y, z, w) "
                             "record per slot (the SoA view is written on demand, outside the step)",
                   "sweep": args.sweep, "precision": args.precision,
                   "pairs_per_step": pairs, "candidate_pairs_per_step": cand,
                   "candidate_pairs_per_s": round(cand / (ms_per_step * 1e-3), 1)},
        "roofline": roof,
        "stages": stages,
        "kernels": kernels,
        "kernels_breakdown_steps": nbreak if kt else 0,
    }
    if not args.no_step:
        print("[bench] time stepping", file=sys.stderr, flush=True)
        out["step"] = bench_step(system)
    if not args.no_batch:
        print("[bench] batch of 512 systems", file=sys.stderr, flush=True)
        out["batch"] = bench_batch(max(3, args.steps // 10), 2)
    if not args.no_serve:
        print("[bench] serving", file=sys.stderr, flush=True)
        out["serve"] = bench_serve()
        print("[bench] serving small requests", file=sys.stderr, flush=True)
        out["serve_small"] = bench_serve(n_pool=64, n_closed=256, n_lo=2e3, n_hi=1e5, max_slots=256)
    if not args.no_table1:
        print("[bench] table 1 grid", file=sys.stderr, flush=True)
        out["table1"] = bench_table1()
    if rank == 0 and not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(system)
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
