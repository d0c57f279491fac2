"""CPU-side checks of libnbody: it loads, exports every entry point include/nbody.h declares,
and validates arguments without touching a GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


@pytest.fixture(scope="module")
def nb():
    import paper_2303_12166_amd as nb
    from paper_2303_12166_amd import build

    if not os.path.exists(nb.lib_path()):
        build.build()
    nb.load()
    return nb


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(nb_\w+)\s*\(", text, re.M)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ("nb_scratch_bytes", "nb_create", "nb_forces", "nb_step", "nb_diagnostics",
                 "nb_destroy", "nb_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol(nb):
    lib = ctypes.CDLL(nb.lib_path())
    missing = [name for name in declared_functions() if not hasattr(lib, name)]
    assert not missing


def test_binding_covers_every_declared_symbol(nb):
    for name in declared_functions():
        assert callable(getattr(nb, name)), name


def test_abi_struct_sizes_match_header(nb):
    # nb_params: 2 int64 + 9 double + 4 int32 + 3 double; nb_diag: 14 double + 1 int64 + 6 int32
    assert ctypes.sizeof(nb.NbParams) == 8 * 11 + 16 + 24
    assert ctypes.sizeof(nb.NbBuffers) == 8 * 12
    assert ctypes.sizeof(nb.NbDiag) == 8 * 14 + 8 + 4 * 6


def _params(nb, **kw):
    base = dict(n=2048, n1=1366, G=1.0, m=1.5 / 2048, dt=1e-4, D1=0.0489, D2=0.0411, q=0.5,
                a=1.0, R2_0=0.2, growth_rate=1e-4, growth_on=1, mode=nb.NB_FP32_KAHAN)
    base.update(kw)
    return nb.NbParams(**base)


def test_scratch_bytes_and_tile_config(nb):
    small = nb.nb_scratch_bytes(_params(nb))
    big = nb.nb_scratch_bytes(_params(nb, n=262144, n1=201650))
    assert 0 < small < big
    cfg = nb.nb_tile_config(262144, 201650, nb.NB_FP32_KAHAN)
    assert cfg["iblock"] == 256 * cfg["ki"]
    assert cfg["jchunk"] % 256 == 0
    assert cfg["nsplit"] * cfg["jchunk"] >= 262144
    assert nb.nb_tile_config(262144, 201650, nb.NB_FP32_PLAIN)["nsplit"] == 1


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("n,n1", [(1, 1), (2, 1), (300, 200), (2048, 1366), (65536, 43691),
                                  (262144, 201650)])
def test_tile_config_covers_every_slot(nb, mode, n, n1):
    cfg = nb.nb_tile_config(n, n1, mode)
    npad = -(-n1 // 256) * 256 + -(-(n - n1) // 256) * 256
    assert cfg["nsplit"] >= 1 and cfg["jchunk"] % 256 == 0
    assert cfg["nsplit"] * cfg["jchunk"] >= npad
    assert cfg["iblock"] == 256 * cfg["ki"]


def test_tile_override(nb):
    K, F = nb.NB_FP32_KAHAN, nb.NB_FP64
    before = nb.nb_tile_config(100000, 60000, K)  # the installed table's choice, if any
    before64 = nb.nb_tile_config(100000, 60000, F)
    nb.nb_tile_override(99000, 101000, K, 3, 2)
    cfg = nb.nb_tile_config(100000, 60000, K)
    assert cfg["nsplit"] == 3 and cfg["rows"] == 2
    # overrides are per mode: the FP64 split is untouched
    assert nb.nb_tile_config(100000, 60000, F) == before64
    nb.nb_tile_override(99000, 101000, F, 5, 1)
    assert nb.nb_tile_config(100000, 60000, F)["nsplit"] == 5
    assert nb.nb_tile_config(100000, 60000, K)["nsplit"] == 3
    # and per element law: the eqs. (4)-(6) split of the same size is untouched
    P = nb.NB_LAW_PAPER
    before_p = nb.nb_tile_config(100000, 60000, K, P)
    nb.nb_tile_override(99000, 101000, K, 7, 1, law=P)
    assert nb.nb_tile_config(100000, 60000, K, P)["nsplit"] == 7
    assert nb.nb_tile_config(100000, 60000, K)["nsplit"] == 3
    nb.nb_tile_override(99000, 101000, K, 0, 1)
    nb.nb_tile_override(99000, 101000, F, 0, 1)
    nb.nb_tile_override(99000, 101000, K, 0, 1, law=P)
    assert nb.nb_tile_config(100000, 60000, K) == before
    assert nb.nb_tile_config(100000, 60000, F) == before64
    assert nb.nb_tile_config(100000, 60000, K, P) == before_p


def test_library_shares_the_hip_runtime_of_pytorch():
    """Loaded before PyTorch is imported, libnbody.so still binds to PyTorch's HIP runtime: the
    process maps one libamdhip64, not a second copy from the ROCm installation (whose runtime
    would find no device next to PyTorch's)."""
    import subprocess
    import sys

    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_2303_12166_amd as nb\n"
            "nb.load()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "1"


def test_built_in_split_above_the_tuned_range(nb):
    """Above the tuned table's sizes the built-in rule applies: bands of four tile rows under the
    contact law and of two under eqs. (4)-(6) in the FP32 Kahan mode (from 256 tiles on), one row
    in the FP64 mode."""
    import json

    from paper_2303_12166_amd.autotune import TABLE_PATH

    with open(TABLE_PATH) as f:
        tables = json.load(f)["tables"]
    n, n1 = 1048576, 582542
    assert all(b["n_hi"] < n for t in tables.values() for b in t["buckets"])
    K, F, P = nb.NB_FP32_KAHAN, nb.NB_FP64, nb.NB_LAW_PAPER
    assert nb.nb_tile_config(n, n1, K)["rows"] == 4
    assert nb.nb_tile_config(n, n1, K, P)["rows"] == 2
    assert nb.nb_tile_config(n, n1, F)["rows"] == 1
    assert nb.nb_tile_config(n, n1, F, P)["rows"] == 1


def test_workspace_budget_coarsens_the_split(nb):
    """Over the budget, taller bands come first (FP32 Kahan), then fewer chunks; without a
    budget the split is the requested one again."""
    K, F = nb.NB_FP32_KAHAN, nb.NB_FP64
    n, n1 = 262144, 201650
    p = _params(nb, n=n, n1=n1)
    p64 = _params(nb, n=n, n1=n1, mode=F)
    nb.nb_tile_override(n, n, K, 114, 1)
    nb.nb_tile_override(n, n, F, 114, 1)
    try:
        full, full64 = nb.nb_scratch_bytes(p), nb.nb_scratch_bytes(p64)
        nb.nb_set_workspace_budget(1_000_000_000)
        try:
            cfg = nb.nb_tile_config(n, n1, K)
            cfg64 = nb.nb_tile_config(n, n1, F)
            small, small64 = nb.nb_scratch_bytes(p), nb.nb_scratch_bytes(p64)
        finally:
            nb.nb_set_workspace_budget(0)
        assert small <= 1_000_000_000 < full
        assert cfg["rows"] == 4 and cfg["nsplit"] == 114
        # the FP64 kernel has one row per band: only its chunk count can shrink, and its
        # reactions alone (doubles) exceed the budget, so it ends at one chunk
        assert cfg64["rows"] == 1 and cfg64["nsplit"] == 1 and small64 < full64
        assert nb.nb_scratch_bytes(p) == full
        assert nb.nb_tile_config(n, n1, K)["rows"] == 1
    finally:
        nb.nb_tile_override(n, n, K, 0, 1)
        nb.nb_tile_override(n, n, F, 0, 1)


# (n_lo, n_hi, mode, law, nsplit, rows)
@pytest.mark.parametrize("args", [(0, 10, 1, 0, 3, 3), (0, 10, 2, 0, 3, 2), (0, 10, 0, 0, 3, 4),
                                  (0, 10, 7, 0, 3, 1), (10, 0, 1, 0, 3, 1), (0, 10, 1, 0, -1, 1),
                                  (0, 10, 1, 2, 3, 1)])
def test_tile_override_rejects_bad_arguments(nb, args):
    assert nb.load().nb_tile_override(*args) == nb.NB_E_INVAL


@pytest.mark.parametrize("bad", [dict(n=-1), dict(n1=3000), dict(mode=7), dict(D1=0.0),
                                 dict(m=float("nan")), dict(q=-0.5), dict(growth_rate=-1.0),
                                 dict(n=1 << 31, n1=0), dict(n=1 << 30, n1=0), dict(law=5),
                                 dict(law=1, mode=0), dict(law=1, beta=1.5),
                                 dict(law=1, gamma=-1.0), dict(law=1, eps=-0.1),
                                 dict(law=1, G=0.0)])
def test_invalid_params_rejected(nb, bad):
    with pytest.raises(nb.NbError) as e:
        nb.nb_scratch_bytes(_params(nb, **bad))
    assert e.value.status == nb.NB_E_INVAL


def test_create_rejects_null_buffers_without_gpu_calls(nb):
    with pytest.raises(nb.NbError) as e:
        nb.nb_create(_params(nb), nb.NbBuffers())
    assert e.value.status == nb.NB_E_INVAL


def test_create_rejects_small_scratch(nb):
    b = nb.NbBuffers(*([256] * 11), 16)  # aligned fake addresses, never dereferenced
    with pytest.raises(nb.NbError) as e:
        nb.nb_create(_params(nb), b)
    assert e.value.status == nb.NB_E_NOMEM


def test_create_refuses_pointers_it_cannot_verify(nb):
    # aligned fake addresses and enough scratch: the pointer check (HIP's pointer attributes)
    # refuses them before any copy or launch; without a GPU the device query fails first
    p = _params(nb)
    b = nb.NbBuffers(*([256] * 11), nb.nb_scratch_bytes(p))
    with pytest.raises(nb.NbError) as e:
        nb.nb_create(p, b)
    assert e.value.status in (nb.NB_E_HIP, nb.NB_E_INVAL)


def test_step_rejects_bad_arguments(nb):
    lib = nb.load()
    assert lib.nb_step(None, 1, 1, None) == nb.NB_E_INVAL
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.nb_step(arr, 1, 1, None) == nb.NB_E_INVAL
    assert lib.nb_step(arr, 0, 1, None) == nb.NB_E_INVAL


def test_step_static_rejects_bad_arguments(nb):
    lib = nb.load()
    assert lib.nb_step_static(None, 1, 1, None) == nb.NB_E_INVAL
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.nb_step_static(arr, 1, 1, None) == nb.NB_E_INVAL
    assert lib.nb_step_static(arr, 0, 1, None) == nb.NB_E_INVAL
    assert lib.nb_step_static(arr, 1, -1, None) == nb.NB_E_INVAL
    # more systems than the fixed table holds: refused before any entry is looked at
    many = (ctypes.c_void_p * (nb.NB_STATIC_MAX_SYS + 1))()
    assert lib.nb_step_static(many, nb.NB_STATIC_MAX_SYS + 1, 1, None) == nb.NB_E_LIMIT
    assert "static segment table" in nb.nb_strerror(nb.NB_E_LIMIT)


def test_sorted_order_rejects_bad_arguments(nb):
    lib = nb.load()
    n = ctypes.c_int64(0)
    assert lib.nb_sorted_order(None, None, 0, ctypes.byref(n), None) == nb.NB_E_INVAL
    assert lib.nb_resort(None, None) == nb.NB_E_INVAL


def test_strerror_and_version(nb):
    assert nb.nb_strerror(nb.NB_E_NOMEM).startswith("workspace")
    assert nb.nb_strerror(12345) == "unknown status"
    assert nb.nb_version() >= 1


def test_timing_without_launches(nb):
    nb.nb_timing_reset()
    assert nb.nb_timing_read() == (0.0, 0)


def test_retention_rejects_null_arguments(nb):
    import ctypes as C

    lib = nb.load()
    v = C.c_int32(0)
    assert lib.nb_retention(None, C.byref(v), C.byref(v), None) == nb.NB_E_INVAL


def test_scratch_bytes_grow_by_sorted_velocities_under_the_paper_law(nb):
    """NB_LAW_PAPER adds three sorted velocity arrays (nalloc slots each, 256-byte aligned) to a
    system of the same work split."""
    big = dict(n=200000, n1=150000)
    # the same work split for both laws (a tuned table may give them different ones)
    splits = [(m, w) for m in (nb.NB_FP32_KAHAN, nb.NB_FP64)
              for w in (nb.NB_LAW_CONTACT, nb.NB_LAW_PAPER)]
    for m, w in splits:
        nb.nb_tile_override(big["n"], big["n"], m, 40, 1, law=w)
    try:
        base = _params(nb, **big)
        paper = _params(nb, law=nb.NB_LAW_PAPER, eps=0.001, gamma=1.0, beta=0.5, **big)
        extra = nb.nb_scratch_bytes(paper) - nb.nb_scratch_bytes(base)
        b64 = _params(nb, mode=nb.NB_FP64, **big)
        p64 = _params(nb, mode=nb.NB_FP64, law=nb.NB_LAW_PAPER, eps=0.001, gamma=1.0, beta=0.5,
                      **big)
        extra64 = nb.nb_scratch_bytes(p64) - nb.nb_scratch_bytes(b64)
    finally:
        for m, w in splits:
            nb.nb_tile_override(big["n"], big["n"], m, 0, 1, law=w)
    # each star padded to whole 256-slot tiles (a multiple of the i-block, so nalloc = slots)
    slots = -(-(base.n1) // 256) * 256 + -(-(base.n - base.n1) // 256) * 256
    per = -(-slots * 4 // 256) * 256
    assert extra == 3 * per
    # FP64: eight bytes per slot
    assert extra64 == 3 * (-(-slots * 8 // 256) * 256)


def test_huge_systems_report_nomem_instead_of_overflowing(nb):
    """Near the 2^30 element limit the symmetric and FP64 work splits would need more than 2^31
    units; the library reports NB_E_NOMEM rather than wrapping the count."""
    big = dict(n=(1 << 30) - 1, n1=1 << 29)
    assert nb.nb_scratch_bytes(_params(nb, mode=nb.NB_FP32_PLAIN, **big)) > 0
    for mode in (nb.NB_FP32_KAHAN, nb.NB_FP64):
        with pytest.raises(nb.NbError) as e:
            nb.nb_scratch_bytes(_params(nb, mode=mode, **big))
        assert e.value.status == nb.NB_E_NOMEM
