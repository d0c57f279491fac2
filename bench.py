#!/usr/bin/env python3
"""Benchmark of the all-pairs binary-star step on one MI355X.

Default workload: two-star system of N = 262,144 elements (q = 0.3, PCG64 seed 0), FP32 forces with
Kahan-compensated accumulation, dt = 1e-4, donor growth and the L1 count every step. A step is
one full kick-drift-kick leap-frog step (O(N^2) force evaluation plus the O(N) kicks, drift,
growth update and L1 count), all in libnbody's HIP kernels, with the state resident in HBM.

Prints ONE JSON line: interactions/s over the timed steps (N^2 per step), the force kernel's
roofline position (20 flops per interaction, measured with HIP events on the launch stream) and
the FP64 CPU oracle's rate on a bounded row sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload c3|c2|c4] [--mode kahan|plain|fp64]
                    [--serve full|small|none]

The same line carries the serving measurement (by default the 256-request trace: continuous
batching against one-at-a-time solves, sims/s and p50/p99 latency both ways, whether every final
state is bitwise the same both ways, and the step-0 force error against the oracle of one request
per size decile).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pair interactions/s + % FP32 VALU peak at N=256K; served sims/s, p50/p99"
FLOPS_PER_INTERACTION = 20
# MI355X published vector peaks: 157.3 TFLOP/s FP32 and 78.6 TFLOP/s FP64. Over 256 CUs at
# 2.4 GHz the FP32 figure is 256 flops per clock per CU, that is 128 FP32 FMA lane-operations per
# clock per CU (the FP64 figure half of that). The library emits only non-packed FP32
# instructions; how close a stream of them comes to 128 lanes per clock is measured on the part
# itself by the issue-rate probe (nb_valu_probe), reported beside the roofline.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
N_CU, CLOCK_HZ = 256, 2.4e9
FMA_LANES_PER_CLK_CU = PEAK_FP32_TFLOPS * 1e12 / (2 * N_CU * CLOCK_HZ)  # 128
VALU_LANE_ISSUE_PER_S = FMA_LANES_PER_CLK_CU * N_CU * CLOCK_HZ

WORKLOADS = {
    "c3": dict(n=262144, q=0.3, mode="kahan", steps=200, warmup=5),
    "c2": dict(n=65536, q=0.5, mode="kahan", steps=1000, warmup=10),
    "c4": dict(n=131072, q=0.8, mode="kahan", steps=200, warmup=5),
}

# force kernel of each mode; the FP32 Kahan kernels are instantiated per band height (%d)
KERNEL_NAMES = {"kahan": "k_force_sym<%d>", "plain": "k_force_f32", "fp64": "k_force_sym64<0>"}
PAPER_KERNEL_NAMES = {"kahan": "k_force_sym_paper<%d>", "fp64": "k_force_sym64<1>"}
COUNTERS_FILE = os.path.join(ROOT, "profiles", "force_counters.json")
# the sources that decide the kernels' machine code: the kernels and their compile-time knobs
KERNEL_SRCS = [os.path.join(ROOT, "paper_2303_12166_amd", "csrc", f)
               for f in ("nb_internal.h", "nb_kernels.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_text(src: str) -> str:
    """C++ source without its comments and with runs of white space collapsed: what the compiler
    turns into machine code, so that an edit of comments alone keeps the hash below."""
    import re

    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, encoding="utf-8") as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()[:16]


def counter_record(workload: str, mode: str, cfg: dict):
    """The committed rocprofv3 counter record of this workload's force kernel, if it was taken
    with this kernel source and work split (HBM bytes per launch, VALU instructions per pair)."""
    try:
        with open(COUNTERS_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    entry = rec.get("%s:%s" % (workload, mode))
    if not entry or entry.get("kernel_sha") != kernel_source_sha():
        return None
    if entry.get("nsplit") != cfg["nsplit"] or entry.get("rows", 1) != cfg["rows"]:
        return None
    return entry


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(ic, target_seconds: float, law=None):
    """The FP64 oracle on a bounded row sample of the same workload (one force evaluation)."""
    import numpy as np

    import oracle

    p, v = ic.f32_as_f64()
    if law is None:
        def accel(rows):
            return oracle.accel(p, ic.n1, ic.G, ic.m, ic.D1, ic.D2, rows=rows)
    else:
        def accel(rows):
            return oracle.accel_paper(p, v, ic.n1, ic.G, ic.m, ic.D1, ic.D2, law["eps"],
                                      law["gamma"], law["beta"], rows=rows)
    n = ic.n
    cores = oracle.max_threads()
    # calibrate on a short sample (second pass: threads already running)
    cal_rows = np.linspace(0, n - 1, 4 * cores).astype(np.int64)
    for _ in range(2):
        t0 = time.perf_counter()
        accel(cal_rows)
        t_cal = max(time.perf_counter() - t0, 1e-6)
    rate = len(cal_rows) * n / t_cal
    k = int(min(n, max(64, target_seconds * rate / n)))
    rows = np.linspace(0, n - 1, k).astype(np.int64)
    t0 = time.perf_counter()
    ref = accel(rows)
    t = time.perf_counter() - t0
    return {
        "value": k * n / t,
        "unit": "interactions/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "%d of %d rows, each against all %d elements (one FP64 force evaluation "
                  "of the step-0 state, %.1f s)" % (k, n, n, t),
        "cpu": cpu_model(),
        "host_cpus_visible": os.cpu_count(),
        "detail": oracle_scaling(cores) if law is None else None,
    }, rows, ref


def oracle_scaling(cores: int) -> dict:
    """The oracle's force-evaluation rate at the other workload sizes (row samples of about a
    second each; every row at N = 2048), the whole N = 2048, 100-step run, and one core."""
    import numpy as np

    import oracle
    import synth

    out = {"interactions_per_s": {}}
    for n, q in ((2048, 0.5), (65536, 0.5), (131072, 0.8)):
        ic = synth.make_binary(n, q, seed=0)
        p, _ = ic.f32_as_f64()
        k = n if n <= 2048 else max(4 * cores, int(1.0e9 / n))
        rows = np.linspace(0, n - 1, k).astype(np.int64)
        oracle.accel(p, ic.n1, ic.G, ic.m, ic.D1, ic.D2, rows=rows[: 4 * cores])
        t0 = time.perf_counter()
        oracle.accel(p, ic.n1, ic.G, ic.m, ic.D1, ic.D2, rows=rows)
        out["interactions_per_s"][str(n)] = k * n / (time.perf_counter() - t0)
    ic = synth.make_binary(2048, 0.5, seed=0)
    p, v = ic.f32_as_f64()
    run = oracle.Run(p, v, ic.n1, ic.G, ic.m, 1e-4, ic.D1, ic.D2, ic.q, a=ic.a, R2_0=ic.R2)
    t0 = time.perf_counter()
    run.advance(100)
    out["n2048_100_step_run_s"] = time.perf_counter() - t0
    ic = synth.make_binary(65536, 0.5, seed=0)
    p, _ = ic.f32_as_f64()
    rows = np.linspace(0, ic.n - 1, 2048).astype(np.int64)
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.accel(p, ic.n1, ic.G, ic.m, ic.D1, ic.D2, rows=rows)
        out["one_core_interactions_per_s"] = len(rows) * ic.n / (time.perf_counter() - t0)
    finally:
        oracle.set_threads(cores)
    return out


def valu_probe() -> dict:
    """Measured issue rates of single VALU instruction streams (lane-instructions per clock per
    CU at the 2.4 GHz peak clock): 2048 blocks of 256 lanes (eight waves per SIMD), eight
    independent chains per lane. Beside each rate, the shader clock the chip held under that
    stream (s_memtime against the 100 MHz s_memrealtime counter, over one block's run) and the
    rate per cycle of that clock."""
    import torch

    import paper_2303_12166_amd as nb

    sink = torch.zeros(64, dtype=torch.float32, device="cuda")
    blocks = N_CU * 4 * 8 // 4
    out, clocks, per_cycle = {}, {}, {}
    for op, name, iters in ((0, "v_fma_f32", 65536), (1, "v_rsq_f32", 16384),
                            (2, "v_rcp_f32", 16384), (3, "3 v_fma_f32 + 1 v_rsq_f32", 16384),
                            (4, "v_fmac_f32", 65536), (5, "v_add_f32", 65536),
                            (6, "v_mul_f32", 65536), (7, "v_sub_f32 (DPP wave_ror:1 source)", 65536),
                            (8, "v_mul_f32 + v_add_f32 in turn", 65536)):
        nb.nb_valu_probe(op, blocks, 64, sink)
        best = None
        for _ in range(3):
            ms, ops, ratio = nb.nb_valu_probe(op, blocks, iters, sink)
            rate = ops / (ms * 1e-3) / (N_CU * CLOCK_HZ)
            if best is None or rate > best[0]:
                best = (rate, ratio)
        out[name] = round(best[0], 2)
        ghz = 0.1 * best[1]
        clocks[name] = round(ghz, 3)
        per_cycle[name] = round(best[0] * CLOCK_HZ / (ghz * 1e9), 2) if ghz > 0 else None
    out["unit"] = "lane-instructions per clock per CU (2.4 GHz, 256 CUs)"
    out["published_fma_lanes_per_clk_cu"] = FMA_LANES_PER_CLK_CU
    out["shader_clock_ghz"] = clocks
    out["per_cycle_of_shader_clock"] = per_cycle
    return out


def copy_calibration() -> int:
    import torch

    n = 1 << 28  # 2^28 floats = 1 GiB
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "repeats": 3}))
    return 0


def serving_trace(scale: str):
    import synth

    if scale == "full":
        trace = synth.make_trace()  # 256 requests, 20/s, N 4096..131072, q 0.1..1, 500 steps
        desc = "256 requests, Poisson 20/s, N log-uniform 4096..131072 (x64), q U[0.1,1], 500 steps"
    else:
        trace = synth.make_trace(count=48, rate=200.0, n_max=32768, steps=200)
        desc = ("48 requests, Poisson 200/s, N log-uniform 4096..32768 (x64), q U[0.1,1], "
                "200 steps")
    return trace, desc


def served_sample(trace, k: int = 10):
    """One request per size decile of the trace (the median-N request of each tenth)."""
    order = sorted(trace, key=lambda r: (r.n, r.rid))
    out = []
    for d in range(k):
        lo, hi = d * len(order) // k, (d + 1) * len(order) // k
        if hi > lo:
            out.append(order[(lo + hi) // 2])
    return out


def served_reference(sample, rows_per_request: int = 64):
    """CPU-baseline leg: the FP64 oracle's step-0 accelerations on sampled rows of each sampled
    request (the request's own seeded system)."""
    import numpy as np

    import oracle
    import synth

    refs = []
    t0 = time.perf_counter()
    for req in sample:
        ic = synth.make_binary(req.n, req.q, seed=req.seed)
        rows = np.unique(np.concatenate([[0, ic.n1 - 1, ic.n1, ic.n - 1],
                                         np.linspace(0, ic.n - 1, rows_per_request)]
                                        ).astype(np.int64))
        p, _ = ic.f32_as_f64()
        refs.append((rows, oracle.accel(p, ic.n1, ic.G, ic.m, ic.D1, ic.D2, rows=rows)))
    log("oracle reference of %d served requests: %.1f s" % (len(sample), time.perf_counter() - t0))
    return refs


def served_errors(sample, refs) -> dict:
    """Step-0 force error of each sampled request's system on the GPU (the arithmetic the server
    runs: a system's kernels and work split depend on its own size only) against the oracle."""
    import numpy as np

    import paper_2303_12166_amd as nb
    import synth

    rows_out, worst = [], 0.0
    for req, (rows, ref) in zip(sample, refs):
        s = nb.System.from_ic(synth.make_binary(req.n, req.q, seed=req.seed), mode="kahan")
        a = s.accelerations()
        s.close()
        err = float(np.linalg.norm(a[rows] - ref, axis=1).max() / np.linalg.norm(ref, axis=1).max())
        worst = max(worst, err)
        rows_out.append({"rid": req.rid, "n": req.n, "q": round(req.q, 4), "rows": int(len(rows)),
                         "force_error_step0": err})
    return {"metric": "max_i |a_gpu-a_oracle| / max_k |a_oracle| on sampled rows, one request "
                      "per size decile", "requests": rows_out, "max": worst}


def serving(scale: str, sequential: bool = True) -> dict:
    """Continuous batching vs one-at-a-time plain solves on one Poisson request trace (the
    batched run alone with sequential=False, e.g. under a kernel trace)."""
    from paper_2303_12166_amd import serve

    trace, desc = serving_trace(scale)
    budget = 64 << 30
    server = serve.BatchServer(budget_bytes=budget, round_steps=10)
    t0 = time.perf_counter()
    batched = server.run(trace, log=log if scale == "full" else None)
    log("batched run %.1f s (%d rounds, %d graphs)" % (time.perf_counter() - t0, server.rounds,
                                                      server.graphs_built))
    if not sequential:
        return {"trace": desc, "requests": len(trace), "budget_bytes": budget,
                "round_steps": server.round_steps, "rounds": server.rounds,
                "batched": serve.summarize(batched), "evicted_nonfinite": server.evicted}
    t0 = time.perf_counter()
    seq = serve.run_sequential(trace, log=log if scale == "full" else None)
    log("sequential run %.1f s" % (time.perf_counter() - t0))
    sb, ss = serve.summarize(batched), serve.summarize(seq)
    same = all(a.digest == b.digest for a, b in zip(batched, seq))
    return {
        "trace": desc,
        "requests": len(trace),
        "budget_bytes": budget,
        "round_steps": server.round_steps,
        "batched": sb,
        "sequential": ss,
        "sims_per_s_speedup": sb["sims_per_s"] / ss["sims_per_s"],
        "results_identical": same,
        "evicted_nonfinite": server.evicted,
        "memory": {"peak_footprint_bytes": server.peak_footprint_bytes,
                   "peak_allocated_bytes": server.peak_allocated_bytes,
                   "peak_cached_bytes": server.peak_cached_bytes},
    }


def precision_study(steps: int) -> dict:
    import numpy as np
    import torch

    import oracle
    import paper_2303_12166_amd as nb
    import synth

    n, q = 131072, 0.8
    ic = synth.make_binary(n, q, seed=0)
    rng = np.random.default_rng(4)
    rows = np.unique(np.concatenate([[0, ic.n1 - 1, ic.n1, n - 1],
                                     rng.integers(0, n, size=252)])).astype(np.int64)
    p64, _ = ic.f32_as_f64()
    ref = oracle.accel(p64, ic.n1, ic.G, ic.m, ic.D1, ic.D2, rows=rows)
    scale = np.linalg.norm(ref, axis=1).max()
    out = {"workload": "two-star binary, N=131072, q=0.8, dt=1e-4, growth off",
           "steps": steps, "force_error_rows": int(len(rows)), "modes": {}}
    for mode in ("plain", "kahan", "fp64"):
        s = nb.System.from_ic(ic, mode=mode, growth_on=False)
        a0 = s.accelerations()
        err = float(np.linalg.norm(a0[rows] - ref, axis=1).max() / scale)
        d0 = s.diagnostics(with_pe=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            k = min(250, steps - done)
            s.step(k)
            s.synchronize()
            done += k
            log("precision study %s: %d/%d steps" % (mode, done, steps))
        t = time.perf_counter() - t0
        d1 = s.diagnostics(with_pe=True)
        v = s.velocities().astype(np.float64)
        s.close()
        pnorm = ic.m * np.linalg.norm(v, axis=1).sum()
        out["modes"][mode] = {
            "force_error_step0": err,
            "energy_drift": abs(d1["E"] - d0["E"]) / abs(d0["E"]),
            "momentum_drift": float(np.linalg.norm(d1["P"] - d0["P"]) / pnorm),
            "angular_momentum_drift": float(np.linalg.norm(d1["L"] - d0["L"])
                                            / np.linalg.norm(d0["L"])),
            "seconds": t,
            "ms_per_step": t / steps * 1e3,
        }
    return out


def morton_perm(pos, n1: int):
    """A sorted order like the library's creation-time one, for the given positions: each star
    in Morton order of 10-bit coordinates inside its own bounding box (ties by index), star 2
    from slot roundup(n1, 256), padding -1."""
    import numpy as np

    def spread(v):
        v = v.astype(np.uint32) & 0x3FF
        v = (v | (v << 16)) & 0x030000FF
        v = (v | (v << 8)) & 0x0300F00F
        v = (v | (v << 4)) & 0x030C30C3
        v = (v | (v << 2)) & 0x09249249
        return v

    def order(b, e):
        p = pos[b:e].astype(np.float64)
        if p.shape[0] == 0:
            return np.zeros(0, dtype=np.int32)
        lo, hi = p.min(axis=0), p.max(axis=0)
        span = np.where(hi > lo, hi - lo, 1.0)
        q = np.minimum(1023.0, np.clip((p - lo) / span, 0.0, 1.0) * 1024.0).astype(np.uint32)
        key = spread(q[:, 0]) | (spread(q[:, 1]) << 1) | (spread(q[:, 2]) << 2)
        return (b + np.lexsort((np.arange(e - b), key))).astype(np.int32)

    n = pos.shape[0]
    p1 = -(-n1 // 256) * 256
    slots = p1 + -(-(n - n1) // 256) * 256
    perm = np.full(slots, -1, dtype=np.int32)
    perm[:n1] = order(0, n1)
    perm[p1:p1 + n - n1] = order(n1, n)
    return perm


def near_share(nb, s, n1: int, D1: float, D2: float, fresh: bool = False) -> float:
    """Share of the (64-element i block, later j tile) pairs of the symmetric kernel that the
    bounding-box test leaves on the near (contact-law) path, for the system's current positions
    in its sorted order (fresh=False: the library's, fixed when the system was created;
    fresh=True: a Morton order of the current positions, what a re-sort would give)."""
    import numpy as np

    pos = s.positions()
    perm = morton_perm(pos, n1) if fresh else nb.nb_sorted_order(s.handle, s.stream)
    slots = perm.size
    T = slots // 256
    P = np.full((slots, 3), np.nan)
    ok = perm >= 0
    P[ok] = pos[perm[ok]]
    tiles = P.reshape(T, 256, 3)
    waves = P.reshape(T * 4, 64, 3)
    with np.errstate(all="ignore"):
        import warnings

        with warnings.catch_warnings():
            warnings.simplefilter("ignore", RuntimeWarning)
            tlo, thi = np.nanmin(tiles, axis=1), np.nanmax(tiles, axis=1)
            wlo, whi = np.nanmin(waves, axis=1), np.nanmax(waves, axis=1)
    p1 = -(-n1 // 256) * 256
    tstar = (np.arange(T) * 256 >= p1).astype(int)
    Ds = np.array([D1, 0.5 * (D1 + D2), D2])
    far2 = Ds * Ds * (1.0 + 2.0e-5)
    near = total = 0
    for w in range(T * 4):
        I = w // 4
        J = np.arange(I + 1, T)
        if J.size == 0 or np.isnan(wlo[w]).any():
            continue
        gap = np.maximum(0.0, np.maximum(tlo[J] - whi[w], wlo[w] - thi[J]))
        gap2 = np.nansum(gap * gap, axis=1)
        cls = tstar[I] + tstar[J]
        valid = ~np.isnan(tlo[J]).any(axis=1)
        near += int(np.count_nonzero((gap2 < far2[cls]) & valid))
        total += int(np.count_nonzero(valid))
    return near / max(total, 1)


def lobe_fill(extra_steps: int, n: int = 65536, q: float = 0.5, bin_steps: int = 100,
              resort_every: int = 0) -> dict:
    """Grow the donor to its Roche lobe and past the stop; record the per-step L1 flux series
    and, every 500 steps, the accretor-side retention of the transferred elements. With
    resort_every = K (a multiple of 500), the sorted order is rebuilt every K steps."""
    import math

    import numpy as np
    import torch

    import paper_2303_12166_amd as nb
    import synth

    ic = synth.make_binary(n, q, seed=0)
    s = nb.System.from_ic(ic, mode="kahan")
    def shares(D2):
        return {"near_share": near_share(nb, s, ic.n1, ic.D1, D2),
                "near_share_fresh_order": near_share(nb, s, ic.n1, ic.D1, D2, fresh=True)}

    rows, ret, near = [], [], [dict(step=0, **shares(ic.D2))]
    chunk_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, stop_seen = 0, None
    while stop_seen is None or done < stop_seen + extra_steps:
        k = 500 if stop_seen is None else min(500, stop_seen + extra_steps - done)
        tc = time.perf_counter()
        s.step(k)
        s.synchronize()
        chunk_ms.append([done + k, round((time.perf_counter() - tc) / k * 1e3, 4)])
        done += k
        rows.append(s.l1_log(k))
        ret.append({"step": done, "n_past_bound": list(s.retention())})
        d = s.diagnostics()
        if resort_every and done % resort_every == 0:
            s.resort()
        if done % 2000 == 0:
            near.append(dict(step=done, **shares(d["D2"])))
        if stop_seen is None and d["growth_stopped"]:
            stop_seen = done
        log("lobe fill: %d steps, past L1 %d, growth %s" % (done, rows[-1][-1, 1],
                                                          "stopped" if d["growth_stopped"] else "on"))
        if stop_seen is None and done >= 40000:
            break
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    d = s.diagnostics()
    near.append(dict(step=done, **shares(d["D2"])))
    s.close()
    series = np.concatenate(rows)
    assert list(series[:, 0]) == list(range(1, done + 1))
    bins = []
    for b in range(0, done, bin_steps):
        seg = series[b:b + bin_steps]
        bins.append([int(seg[-1, 0]), int(seg[:, 2].sum()), int(seg[:, 3].sum()), int(seg[-1, 1])])
    first_fwd = np.flatnonzero(series[:, 2] > 0)
    return {
        "workload": "two-star binary, N=%d, q=%g, FP32 Kahan, dt=1e-4, donor element diameter "
                    "grown by 1e-4 per step from R2_0 = %.2f until the nominal radius passes "
                    "r_L a (eq. 3), then %d more steps%s" % (
                        n, q, ic.R2, extra_steps,
                        ", sorted order rebuilt every %d steps" % resort_every if resort_every
                        else ""),
        "steps": done,
        "growth_stopped": d["growth_stopped"],
        "growth_steps": int(round(math.log(d["D2"] / ic.D2) / math.log(1.0 + 1e-4))),
        "R2_final": d["R2"],
        "first_forward_crossing_step": int(series[first_fwd[0], 0]) if first_fwd.size else None,
        "forward_crossings": int(series[:, 2].sum()),
        "backward_crossings": int(series[:, 3].sum()),
        "past_L1_at_end": int(series[-1, 1]),
        "bins": {"columns": ["last_step", "forward", "backward", "past_L1_at_end"],
                 "rows": bins},
        "retention": ret,
        "ms_per_step": t / done * 1e3,
        # step time of each 500-step stretch (host-timed, the read-backs between stretches
        # excluded) and the near-path share of the sorted order over the run
        "ms_per_step_by_stretch": chunk_ms,
        "near_share": near,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c3")
    ap.add_argument("--mode", choices=["kahan", "plain", "fp64"], default=None)
    ap.add_argument("--law", choices=["contact", "paper"], default="contact",
                    help="element law: the conservative contact law (default) or the paper's "
                         "eqs. (4)-(6) (velocity-noised start, gamma/eps/beta from "
                         "synth.paper_law_params; Kahan or FP64 only)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--serve", choices=["none", "small", "full"], default="full",
                    help="serving measurement added to the main line: 'full' (default) the "
                         "256-request trace (Poisson 20/s, N 4096..131072, 500 steps), 'small' a "
                         "48-request trace (N 4096..32768, 200 steps), 'none' no serving")
    ap.add_argument("--no-sequential", action="store_true",
                    help="with --serve-only: the batched run alone (no one-at-a-time baseline)")
    ap.add_argument("--serve-only", action="store_true",
                    help="print only the serving measurement (--serve picks the trace)")
    ap.add_argument("--precision-study", action="store_true",
                    help="N=131072, q=0.8: FP32 plain, FP32 Kahan and FP64 runs of --steps steps "
                         "(default 2000), step-0 force error vs the FP64 oracle and FP64 drift of "
                         "E, P and L (donor growth off so that the energy is conserved)")
    ap.add_argument("--lobe-fill", action="store_true",
                    help="grow the donor of an N=--lobe-n, q=--lobe-q system (default 65536, 0.5: "
                         "about 4150 steps) to its Roche lobe and run --steps more after growth "
                         "stops (default 2000); prints the binned L1 flux series and the "
                         "accretor-side retention")
    ap.add_argument("--lobe-n", type=int, default=65536, help="elements of the --lobe-fill run")
    ap.add_argument("--lobe-q", type=float, default=0.5, help="mass ratio of the --lobe-fill run")
    ap.add_argument("--resort-every", type=int, default=0,
                    help="--lobe-fill: rebuild the sorted order every this many steps (multiple "
                         "of 500; 0 never)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (three times), the reference "
                         "for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters to bytes")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.precision_study:
        import torch

        import paper_2303_12166_amd as nb

        nb.load()
        torch.cuda.set_device(0)
        res = precision_study(args.steps or 2000)
        print(json.dumps({"metric": "precision study (force error, E/P/L drift)", "value": None,
                          "n_gpus": 1, "data": "synthetic", "precision_study": res}), flush=True)
        return 0
    if args.lobe_fill:
        import torch

        import paper_2303_12166_amd as nb

        nb.load()
        torch.cuda.set_device(0)
        if args.resort_every % 500:
            ap.error("--resort-every must be a multiple of 500")
        res = lobe_fill(2000 if args.steps is None else args.steps, n=args.lobe_n, q=args.lobe_q,
                        resort_every=args.resort_every)
        print(json.dumps({"metric": "lobe-filling run: L1 flux series and retention",
                          "value": None, "n_gpus": 1, "data": "synthetic", "lobe_fill": res}),
              flush=True)
        return 0
    if args.serve_only:
        import torch

        import paper_2303_12166_amd as nb

        nb.load()
        torch.cuda.set_device(0)
        res = serving("small" if args.serve == "small" else "full",
                      sequential=not args.no_sequential)
        print(json.dumps({
            "metric": METRIC, "value": res["batched"]["sims_per_s"], "unit": "sims/s",
            "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f32",
            "data": "synthetic", "config": {"workload": "serving: " + res["trace"]},
            "serving": res}), flush=True)
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2303_12166_amd as nb
    import synth

    wl = WORKLOADS[args.workload]
    mode = args.mode or wl["mode"]
    steps = wl["steps"] if args.steps is None else args.steps
    warmup = wl["warmup"] if args.warmup is None else args.warmup
    n, q = wl["n"], wl["q"]

    nb.load()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    log("workload %s: N=%d q=%.2f mode=%s steps=%d warmup=%d" % (args.workload, n, q, mode, steps,
                                                                  warmup))
    ic = synth.make_binary(n, q, seed=0)
    law = None
    if args.law == "paper":
        if mode == "plain":
            print("the paper's law has no plain FP32 kernel", file=sys.stderr)
            return 2
        ic = synth.with_velocity_noise(ic, 0.05, 1000)
        law = synth.paper_law_params(ic)
    s = nb.System.from_ic(ic, mode=mode, dt=1e-4, **(law or {}))
    a0 = s.accelerations()
    cfg = nb.nb_tile_config(n, ic.n1, nb.MODES[mode], nb.LAWS[args.law])
    log("tile config", cfg)

    s.step(warmup)
    s.synchronize()
    nb.nb_timing_reset()
    nb.nb_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.step(1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nb.nb_timing_enable(False)
    force_ms, launches = nb.nb_timing_read()
    elapsed = t1 - t0
    d = s.diagnostics(with_pe=False)
    log("timed %d steps in %.3f s; force kernel %.3f ms avg over %d launches" %
        (steps, elapsed, force_ms / max(launches, 1), launches))

    inter = float(n) * float(n)
    value = inter * steps / elapsed
    avg_s = force_ms / max(launches, 1) / 1e3
    peak = PEAK_FP64_TFLOPS if mode == "fp64" else PEAK_FP32_TFLOPS
    counters = counter_record(args.workload + (":paper" if law else ""), mode, cfg)
    achieved = FLOPS_PER_INTERACTION * inter / avg_s / 1e12 if avg_s > 0 else 0.0
    kernel = (PAPER_KERNEL_NAMES if law else KERNEL_NAMES)[mode]
    if "%d" in kernel:
        kernel = kernel % cfg["rows"]
    # pairs the kernel evaluates: N^2 / 2 with the symmetric kernels (each unordered pair once),
    # N^2 one-sided
    evaluated = inter / 2 if kernel.startswith("k_force_sym") else inter
    executed = FLOPS_PER_INTERACTION * evaluated / avg_s / 1e12 if avg_s > 0 else 0.0
    roofline = {
        "bound": "alu",
        "achieved": round(achieved, 3),
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": (counters or {}).get("bytes_per_launch"),
        "kernel": kernel,
        "flops_per_interaction": FLOPS_PER_INTERACTION,
        "avg_launch_ms": round(avg_s * 1e3, 4),
        "launches": launches,
        "flops_per_launch": FLOPS_PER_INTERACTION * inter,
        "kernel_interactions_per_s": inter / avg_s if avg_s > 0 else 0.0,
        # the convention above counts N^2 interactions per evaluation; the symmetric kernel
        # evaluates each unordered pair once, so the work it executes is half that
        "pairs_evaluated_per_launch": evaluated,
        "executed_achieved": round(executed, 3),
        "executed_frac": round(executed / peak, 4),
    }
    probe = None
    try:
        probe = valu_probe()
    except Exception as e:  # a probe failure must not lose the measurement
        log("VALU probe failed: %s" % e)
    roofline["valu_probe"] = probe
    if counters:
        vpp = counters.get("valu_lane_instructions_per_pair")
        roofline["counters"] = {
            "source": "profiles/force_counters.json (rocprofv3, same kernel source and split)",
            "valu_lane_instructions_per_pair": vpp,
            "trans_lane_instructions_per_pair": counters.get("trans_lane_instructions_per_pair"),
            "hbm_bytes_per_launch": counters.get("bytes_per_launch"),
            "algorithmic_bytes_per_launch": counters.get("algorithmic_bytes_per_launch"),
        }
        if vpp and avg_s > 0:
            # achieved VALU issue (every VALU instruction, transcendentals included, live timing)
            # against 128 lane-instructions per clock per CU (the published FP32 peak in FMA
            # lanes) and against the probe's measured non-packed FMA rate
            rate = vpp * evaluated / avg_s
            roofline["counters"]["valu_lane_instructions_per_s"] = rate
            roofline["counters"]["valu_lane_instructions_per_clk_cu"] = round(
                rate / (N_CU * CLOCK_HZ), 2)
            roofline["counters"]["valu_issue_frac"] = round(rate / VALU_LANE_ISSUE_PER_S, 4)
            if probe and probe.get("v_fma_f32"):
                roofline["counters"]["valu_issue_frac_of_probe_fma"] = round(
                    rate / (N_CU * CLOCK_HZ) / probe["v_fma_f32"], 4)
            for key in ("add_f32", "mul_f32", "fma_f32"):
                k = key + "_lane_instructions_per_pair"
                if counters.get(k) is not None:
                    roofline["counters"][k] = counters[k]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if mode == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": "two-star binary, N=%d, q=%g, %s forces%s, dt=1e-4, donor growth + L1 "
                        "count every step" % (n, q, {"kahan": "FP32 Kahan", "plain": "FP32 plain",
                                                       "fp64": "FP64"}[mode],
                                              " under eqs. (4)-(6)" if law else ""),
            "n": n,
            "q": q,
            "mode": mode,
            "law": args.law,
            "seed": 0,
            "tile": cfg,
        },
        "roofline": roofline,
        "state_after": {"step": d["step"], "n_past_L1": d["n_past_L1"], "D2": d["D2"],
                        "nonfinite": d["nonfinite"]},
        # the paper measures nothing on this path; its one performance figure is a vendor peak
        "paper_context": {"hardware": "NVIDIA GeForce RTX 3080", "vendor_fp32_peak_tflops": 29.0,
                          "measured": None,
                          "note": "quoted in the paper's Methodology section as the GPU's "
                                  "processing power; no timing, N or throughput is reported"},
    }
    s.close()

    sample, refs = [], None
    if args.serve != "none":
        sample = served_sample(serving_trace(args.serve)[0])
    if not args.no_cpu:
        base, rows, ref = cpu_baseline(ic, args.cpu_seconds, law)
        out["cpu_baseline"] = base
        err = (np.linalg.norm(a0[rows] - ref, axis=1).max() / np.linalg.norm(ref, axis=1).max())
        out["force_error_step0"] = {"value": float(err), "rows": int(len(rows)),
                                    "metric": "max_i |a_gpu-a_oracle| / max_k |a_oracle|"}
        if sample:
            refs = served_reference(sample)
    else:
        out["cpu_baseline"] = None
    if args.serve != "none":
        out["serving"] = serving(args.serve)
        if refs is not None:
            out["serving"]["oracle_check"] = served_errors(sample, refs)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
