"""The library driven from plain C with hipMalloc'd buffers (tests/c_abi_gpu.c, built by
__graft_entry__.build()) gives bitwise the same state as the same run through the Python binding.
"""

import os
import struct
import subprocess

import numpy as np
import pytest

import synth
from gpu_common import print_case, require_gpu

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c_abi_gpu")


def test_c_program_matches_python_binding(tmp_path):
    nb = require_gpu()
    if not os.path.exists(EXE):
        pytest.skip("tests/c_abi_gpu is not built (run __graft_entry__.build())")
    ic = synth.make_binary(3000, 0.4, seed=42)
    steps = 20
    p, v = ic.f32()
    prm = [ic.G, ic.m, 1e-4, ic.D1, ic.D2, ic.q, ic.a, ic.R2, 1e-4]
    src = tmp_path / "in.bin"
    with open(src, "wb") as f:
        f.write(struct.pack("<2q", ic.n, ic.n1))
        f.write(struct.pack("<9d", *prm))
        for col in (p[:, 0], p[:, 1], p[:, 2], v[:, 0], v[:, 1], v[:, 2]):
            f.write(np.ascontiguousarray(col, dtype=np.float32).tobytes())
    out = tmp_path / "out.bin"
    # the binding installs the tuned split table when it loads; the C program asks for the same
    from paper_2303_12166_amd import autotune

    table = autotune.load_table(autotune.TABLE_PATH) or {}
    if table.get("library_version") != nb.nb_version():
        table = {}
    buckets = table.get("tables", {}).get("kahan", {}).get("buckets", [])
    b = next((b for b in buckets if b["n_lo"] <= ic.n <= b["n_hi"]), {"nsplit": 0, "rows": 1})
    req, rows = b["nsplit"], b.get("rows", 1)
    assert nb.nb_tile_config(ic.n, ic.n1, nb.NB_FP32_KAHAN)["rows"] == rows
    print_case("C program", ic.n, steps, "split request", req, "rows", rows)
    r = subprocess.run([EXE, str(src), str(out), str(steps), str(req), str(rows)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = np.fromfile(out, dtype=np.float32, count=6 * ic.n)
    tail = np.fromfile(out, dtype=np.float64, offset=6 * ic.n * 4)
    xc = raw[: 3 * ic.n].reshape(3, ic.n).T
    vc = raw[3 * ic.n:].reshape(3, ic.n).T

    s = nb.System(p, v, ic.n1, G=ic.G, m=ic.m, dt=1e-4, D1=ic.D1, D2=ic.D2, q=ic.q, a=ic.a,
                  R2_0=ic.R2, growth_rate=1e-4, mode="kahan")
    s.step(steps)
    d = s.diagnostics(with_pe=True)
    assert np.array_equal(s.positions(), xc)
    assert np.array_equal(s.velocities(), vc)
    s.close()
    ke, pe, d2, step = tail
    assert step == steps and d2 == d["D2"]
    assert ke == d["KE"] and pe == d["PE"]
