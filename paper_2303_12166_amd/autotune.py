"""Autotuner for the force kernels' work split.

The kernels' compile-time shapes (tile sizes, waves per SIMD) were fixed by measurement. What
depends on the system size is how the pair work is cut into work units: the number of j chunks
(more chunks mean more, shorter units: better balance across the 256 CUs, more partial sums to
combine) and, in the FP32 Kahan mode, the band height (tile rows whose pairs one unit evaluates
together: taller bands store fewer reaction partials and stage each j tile once for more rows,
at fewer waves per SIMD). For each precision mode, element law and size bucket the tuner times
one whole force evaluation (gather, force kernel and combine) for every candidate (rows, chunks)
on a seeded two-star system and keeps the fastest (the candidates within 2 % of the first pass's
best are timed again in five interleaved rounds, and the best median wins); ``apply`` installs
the table through
``nb_tile_override``, so the choice stays a function of the mode, law and system size alone (a
system gets the same split alone and in a batch). A workspace budget can exclude candidates whose
``nb_scratch_bytes`` exceeds it.

    python -m paper_2303_12166_amd.autotune [--out FILE] [--keys kahan,kahan:paper,fp64]  # GPU
"""

from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys

from . import (LAWS, MODES, NbParams, nb_scratch_bytes, nb_tile_config, nb_tile_override,
               nb_version)

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(HERE, "tuning", "gfx950.json")

# bucket edges (inclusive ranges) covering 4096 .. 524288 elements: a factor sqrt(2) apart up to
# 262144 (each bucket is tuned at its geometric middle, so no size is more than 2^(1/4) from the
# size its split was measured at), then one bucket up to 524287 tuned at 262144
EDGES = [int(64 * round(4096 * 2 ** (k / 2) / 64)) for k in range(13)] + [524288]
CHUNKS = (1, 2, 4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256)
REFINE_FRAC, REFINE_ROUNDS = 0.02, 5
ROWS = {"kahan": (1, 2, 4), "fp64": (1,)}
# table keys: "<mode>" for the contact law, "<mode>:paper" for eqs. (4)-(6)
KEYS = ("kahan", "kahan:paper", "fp64", "fp64:paper")


def split_key(key: str):
    mode, _, law = key.partition(":")
    return mode, law or "contact"


def buckets():
    out = [(1, EDGES[0] - 1)]
    for lo, hi in zip(EDGES[:-1], EDGES[1:]):
        out.append((lo, hi - 1))
    out.append((EDGES[-1], (1 << 31) - 1))
    return out


def _entries(table: dict):
    for key, sub in table.get("tables", {}).items():
        mode, law = split_key(key)
        for e in sub.get("buckets", []):
            yield MODES[mode], LAWS[law], e


def apply(table: dict) -> None:
    for mode, law, e in _entries(table):
        nb_tile_override(int(e["n_lo"]), int(e["n_hi"]), mode, int(e["nsplit"]),
                         int(e.get("rows", 1)), law=law)


def clear(table: dict) -> None:
    for mode, law, e in _entries(table):
        nb_tile_override(int(e["n_lo"]), int(e["n_hi"]), mode, 0, 1, law=law)


def load_table(path: str = TABLE_PATH):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def apply_saved(path: str = TABLE_PATH) -> bool:
    """Installs the saved table if it exists and was made for this library version."""
    table = load_table(path)
    if not table or table.get("library_version") != nb_version():
        return False
    apply(table)
    return True


def _time_forces(ic, mode: str, law_kw: dict, repeats: int) -> float:
    """Mean time of one whole force evaluation (gather, force kernel and combine), from events
    on the system's stream."""
    import torch

    from .system import System

    s = System.from_ic(ic, mode=mode, **law_kw)
    s.forces()
    s.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s.stream)
    for _ in range(repeats):
        s.forces()
    b.record(s.stream)
    b.synchronize()
    ms = a.elapsed_time(b)
    s.close()
    return ms / max(repeats, 1)


def _workspace(ic, mode: str, law_kw: dict) -> int:
    p = NbParams(n=ic.n, n1=ic.n1, G=ic.G, m=ic.m, dt=1e-4, D1=ic.D1, D2=ic.D2, q=ic.q, a=ic.a,
                 R2_0=ic.R2, growth_rate=1e-4, growth_on=1, mode=MODES[mode],
                 law=LAWS[law_kw.get("law", "contact")], pad=0, eps=law_kw.get("eps", 0.0),
                 gamma=law_kw.get("gamma", 0.0), beta=law_kw.get("beta", 1.0))
    return nb_scratch_bytes(p)


def tune_key(key: str, q: float = 0.5, repeats: int = 4, max_n: int = 262144,
             budget: int = 0, log=print) -> dict:
    import synth

    mode, law = split_key(key)
    M, W = MODES[mode], LAWS[law]
    out = {"q": q, "budget_bytes": budget, "buckets": []}
    for lo, hi in buckets():
        n = int(64 * round(math.sqrt(max(lo, EDGES[0] // 2) * min(hi, max_n)) / 64))
        if lo > max_n:
            break
        ic = synth.make_binary(n, q, seed=7)
        law_kw = {}
        if law == "paper":
            ic = synth.with_velocity_noise(ic, 0.05, 7)
            law_kw = synth.paper_law_params(ic)
        timings, seen = {}, set()
        for rows in ROWS[mode]:
            for ns in CHUNKS:
                nb_tile_override(n, n, M, ns, rows, law=W)
                try:
                    cfg = nb_tile_config(n, ic.n1, M, W)
                    # requests that give the same work split as an earlier one are skipped
                    split = (cfg["rows"], cfg["nsplit"], cfg["jchunk"])
                    if split in seen or cfg["nsplit"] > ns:
                        continue
                    seen.add(split)
                    if budget and _workspace(ic, mode, law_kw) > budget:
                        continue
                    timings["%d:%d" % (rows, ns)] = _time_forces(ic, mode, law_kw, repeats)
                finally:
                    nb_tile_override(n, n, M, 0, 1, law=W)
        # the candidates within REFINE_FRAC of the fastest are timed again in interleaved rounds
        # (a first pass of a few evaluations each cannot tell splits 1 % apart); the best median
        # over the rounds wins
        first = min(timings.values())
        close = sorted(k for k, v in timings.items() if v <= first * (1.0 + REFINE_FRAC))
        refined = {}
        if len(close) > 1:
            rounds = {k: [] for k in close}
            for _ in range(REFINE_ROUNDS):
                for k in close:
                    rows, ns = (int(v) for v in k.split(":"))
                    nb_tile_override(n, n, M, ns, rows, law=W)
                    try:
                        rounds[k].append(_time_forces(ic, mode, law_kw, 2 * repeats))
                    finally:
                        nb_tile_override(n, n, M, 0, 1, law=W)
            refined = {k: statistics.median(v) for k, v in rounds.items()}
            best = min(refined, key=refined.get)
        else:
            best = close[0]
        rows, ns = (int(v) for v in best.split(":"))
        ms = refined.get(best, timings[best])
        log("%s bucket [%d, %d] tuned at n=%d: rows %d nsplit %d (%.3f ms); %s%s" % (
            key, lo, hi, n, rows, ns, ms,
            " ".join("%s=%.3f" % (k, v) for k, v in sorted(timings.items())),
            "; refined " + " ".join("%s=%.3f" % (k, v) for k, v in sorted(refined.items()))
            if refined else ""))
        out["buckets"].append({"n_lo": lo, "n_hi": hi, "n_tuned": n, "rows": rows, "nsplit": ns,
                               "ms": round(ms, 4),
                               "candidates_ms": {k: round(v, 4) for k, v in timings.items()},
                               "refined_ms": {k: round(v, 4) for k, v in refined.items()}})
    return out


def tune(keys=KEYS, q: float = 0.5, repeats: int = 4, max_n: int = 262144,
         budget: int = 0, log=print) -> dict:
    import torch

    table = {"arch": torch.cuda.get_device_properties(0).gcnArchName.split(":")[0],
             "library_version": nb_version(), "budget_bytes": int(budget), "tables": {}}
    for key in keys:
        table["tables"][key] = tune_key(key, q, repeats, max_n, budget, log)
    return table


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--keys", default=",".join(KEYS))
    ap.add_argument("--repeats", type=int, default=4)
    ap.add_argument("--max-n", type=int, default=262144)
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="skip splits whose workspace exceeds this many GB (0: no limit)")
    args = ap.parse_args()
    keys = [k for k in args.keys.split(",") if k]
    for k in keys:
        mode, law = split_key(k)
        if mode not in ROWS or law not in LAWS:
            ap.error("no tunable split for %r" % k)
    table = tune(keys, repeats=args.repeats, max_n=args.max_n,
                 budget=int(args.budget_gb * 1e9),
                 log=lambda *a: print(*a, file=sys.stderr, flush=True))
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
        f.write("\n")
    print(json.dumps({"written": args.out, "keys": keys}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
