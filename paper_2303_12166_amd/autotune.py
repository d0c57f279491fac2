"""Autotuner for the force kernels' work split.

The kernels' compile-time shapes (tile sizes, waves per SIMD) were fixed by measurement. What
depends on the system size is how many j chunks the work is split into: more chunks mean more,
shorter work units (better balance across the 256 CUs, more partial sums to combine). For each
size bucket the tuner times one whole force evaluation (gather, force kernel and combine) for
every candidate split on a seeded two-star system and keeps the fastest; ``apply`` installs the
table through ``nb_tile_override``, so the choice stays a function of the system size alone (a
system gets the same split alone and in a batch).

    python -m paper_2303_12166_amd.autotune [--out FILE]     # on a GPU
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys

from . import MODES, nb_tile_config, nb_tile_override, nb_version

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(HERE, "tuning", "gfx950.json")

# bucket edges (inclusive ranges) covering 4096 .. 524288 elements, factor 2 apart
EDGES = [4096, 8192, 16384, 32768, 65536, 131072, 262144, 524288]
CANDIDATES = (1, 2, 4, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256)


def buckets():
    out = [(1, EDGES[0] - 1)]
    for lo, hi in zip(EDGES[:-1], EDGES[1:]):
        out.append((lo, hi - 1))
    out.append((EDGES[-1], (1 << 31) - 1))
    return out


def apply(table: dict) -> None:
    for e in table.get("buckets", []):
        nb_tile_override(int(e["n_lo"]), int(e["n_hi"]), int(e["nsplit"]))


def clear(table: dict) -> None:
    for e in table.get("buckets", []):
        nb_tile_override(int(e["n_lo"]), int(e["n_hi"]), 0)


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


def _time_forces(ic, mode: str, repeats: int) -> float:
    """Mean time of one whole force evaluation (gather, force kernel and combine), from events
    on the system's stream."""
    import torch

    from .system import System

    s = System.from_ic(ic, mode=mode)
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


def tune(mode: str = "kahan", q: float = 0.5, repeats: int = 4, max_n: int = 262144,
         log=print) -> dict:
    import torch

    import synth

    table = {"arch": torch.cuda.get_device_properties(0).gcnArchName.split(":")[0],
             "library_version": nb_version(), "mode": mode, "q": q, "buckets": []}
    for lo, hi in buckets():
        n = int(64 * round(math.sqrt(max(lo, EDGES[0] // 2) * min(hi, max_n)) / 64))
        if lo > max_n:
            break
        ic = synth.make_binary(n, q, seed=7)
        timings, seen = {}, set()
        for ns in CANDIDATES:
            nb_tile_override(n, n, ns)
            try:
                cfg = nb_tile_config(n, ic.n1, MODES[mode])
                # requests that give the same work split as an earlier one are skipped
                split = (cfg["nsplit"], cfg["jchunk"])
                if split in seen or cfg["nsplit"] > ns:
                    continue
                seen.add(split)
                timings[ns] = _time_forces(ic, mode, repeats)
            finally:
                nb_tile_override(n, n, 0)
        best = min(timings, key=timings.get)
        log("bucket [%d, %d] tuned at n=%d: nsplit %d (%.3f ms); %s" % (
            lo, hi, n, best, timings[best],
            " ".join("%d:%.3f" % (k, v) for k, v in sorted(timings.items()))))
        table["buckets"].append({"n_lo": lo, "n_hi": hi, "n_tuned": n, "nsplit": best,
                                 "ms": round(timings[best], 4),
                                 "candidates_ms": {str(k): round(v, 4) for k, v in timings.items()}})
    return table


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--mode", default="kahan", choices=["kahan", "plain", "fp64"])
    ap.add_argument("--repeats", type=int, default=4)
    ap.add_argument("--max-n", type=int, default=262144)
    args = ap.parse_args()
    table = tune(args.mode, repeats=args.repeats, max_n=args.max_n,
                 log=lambda *a: print(*a, file=sys.stderr, flush=True))
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
        f.write("\n")
    print(json.dumps({"written": args.out, "buckets": len(table["buckets"])}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
