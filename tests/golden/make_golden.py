"""Writes tests/golden/ic_checksums.json: frozen SHA-256 digests of generator outputs.

Run from the repository root: ``python tests/golden/make_golden.py``. It calls only the input
generator; the digests freeze the particular samples so that a change of draw order is noticed.
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

CASES = [(2048, 0.5, 0), (65536, 0.5, 0), (262144, 0.3, 0), (131072, 0.8, 0), (4096, 0.1, 1)]


def main():
    out = {"generator": "synth.make_binary (PCG64)", "checksums": {}}
    for n, q, seed in CASES:
        out["checksums"]["%d:%r:%d" % (n, q, seed)] = synth.make_binary(n, q, seed).checksum()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ic_checksums.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
