"""MI355X (gfx950) implementation of the all-pairs binary-star element model.

Python binding of libnbody (include/nbody.h): the functions below carry the C entry points' names
and only marshal arguments; every step of the computation runs in the HIP kernels of the library.
If the library has not been built, loading raises instead of falling back to anything else.

``System`` is a convenience wrapper that keeps one system's state in PyTorch device tensors.
"""

from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

from . import _abi
from ._abi import (  # noqa: F401
    LAWS,
    MODES,
    NB_LAW_CONTACT,
    NB_LAW_PAPER,
    NB_E_HIP,
    NB_E_INVAL,
    NB_E_LIMIT,
    NB_E_MISMATCH,
    NB_E_NOMEM,
    NB_E_NONFINITE,
    NB_FP32_KAHAN,
    NB_FP32_PLAIN,
    NB_FP64,
    NB_L1_LOG_CAP,
    NB_OK,
    NB_STATIC_MAX_SYS,
    NbBuffers,
    NbDiag,
    NbParams,
)

_lock = threading.Lock()
_lib = None


class NbError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (where, _strerror(status), status))


class LibraryMissing(ImportError):
    pass


def lib_path() -> str:
    return _abi.LIB_PATH


def load() -> ctypes.CDLL:
    """Loads libnbody.so (built in-tree by ``python -m paper_2303_12166_amd.build``).

    PyTorch is imported first. Its bundled HIP runtime and the ROCm one that libnbody.so was
    linked against carry the same soname (libamdhip64.so.7), so with PyTorch's already in the
    process the library binds to it and shares its device, memory and streams. Loaded the other
    way round, the process would hold two HIP runtimes, and the library's would find no device
    once PyTorch's had taken it."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_abi.LIB_PATH):
                raise LibraryMissing(
                    "libnbody.so is not built (%s); run python -m paper_2303_12166_amd.build"
                    % _abi.LIB_PATH)
            import torch  # noqa: F401  (its HIP runtime must be the process's one)

            _lib = _abi.declare(ctypes.CDLL(_abi.LIB_PATH))
    # measured j-split table for this GPU (see autotune.py); the built-in rule otherwise
    from .autotune import apply_saved

    apply_saved()
    return _lib


def _strerror(status: int) -> str:
    try:
        return load().nb_strerror(int(status)).decode()
    except Exception:  # pragma: no cover - only when the library itself is missing
        return "status %d" % status


def _check(rc: int, where: str) -> None:
    if rc != NB_OK:
        raise NbError(rc, where)


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        return ctypes.c_void_p(None)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- C entry points


def nb_version() -> int:
    return int(load().nb_version())


def nb_strerror(status: int) -> str:
    return _strerror(status)


def nb_scratch_bytes(params: NbParams) -> int:
    out = ctypes.c_size_t(0)
    _check(load().nb_scratch_bytes(ctypes.byref(params), ctypes.byref(out)), "nb_scratch_bytes")
    return int(out.value)


def nb_create(params: NbParams, buffers: NbBuffers, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p(None)
    _check(load().nb_create(ctypes.byref(params), ctypes.byref(buffers), _stream(stream),
                            ctypes.byref(h)), "nb_create")
    return h


def nb_forces(handle: ctypes.c_void_p, stream=None) -> None:
    _check(load().nb_forces(handle, _stream(stream)), "nb_forces")


def nb_step(handles, n_steps: int, stream=None) -> None:
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                             for h in handles])
    _check(load().nb_step(arr, len(handles), int(n_steps), _stream(stream)), "nb_step")


def nb_step_static(handles, n_steps: int, stream=None) -> None:
    """nb_step with the segment table in the library's fixed per-GPU array (no allocation);
    at most NB_STATIC_MAX_SYS systems, and calls on one GPU must be ordered on one stream."""
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                             for h in handles])
    _check(load().nb_step_static(arr, len(handles), int(n_steps), _stream(stream)),
           "nb_step_static")


def nb_diagnostics(handle: ctypes.c_void_p, with_pe: bool = False, stream=None) -> dict:
    d = NbDiag()
    rc = load().nb_diagnostics(handle, int(bool(with_pe)), ctypes.byref(d), _stream(stream))
    if rc not in (NB_OK, NB_E_NONFINITE):
        raise NbError(rc, "nb_diagnostics")
    return {
        "com": np.array(d.com[:]),
        "P": np.array(d.P[:]),
        "L": np.array(d.L[:]),
        "KE": d.KE,
        "PE": d.PE,
        "E": d.E,
        "D2": d.D2,
        "R2": d.R2,
        "step": int(d.step),
        "n_past_L1": int(d.n_past_L1),
        "cross_fwd": int(d.cross_fwd),
        "cross_bwd": int(d.cross_bwd),
        "growth_stopped": bool(d.growth_stopped),
        "nonfinite": int(d.nonfinite),
        "status": int(rc),
    }


def nb_nonfinite_async(handles, out_host, stream=None) -> None:
    """Queues copies of each system's non-finite count into ``out_host`` (an int32 tensor or
    array with at least len(handles) entries, pinned for asynchrony); valid once ``stream`` has
    passed the call."""
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                             for h in handles])
    if hasattr(out_host, "data_ptr"):
        if out_host.numel() < len(handles) or out_host.device.type != "cpu":
            raise ValueError("out_host must be a host int32 tensor with one entry per system")
        ptr = ctypes.cast(ctypes.c_void_p(out_host.data_ptr()), ctypes.POINTER(ctypes.c_int32))
    else:
        if out_host.dtype != np.int32 or out_host.size < len(handles):
            raise ValueError("out_host must be an int32 array with one entry per system")
        ptr = out_host.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    _check(load().nb_nonfinite_async(arr, len(handles), ptr, _stream(stream)),
           "nb_nonfinite_async")


def nb_retention(handle: ctypes.c_void_p, stream=None) -> tuple:
    """(n_past, n_bound): donor elements past L1 and those of them bound to the accretor."""
    past, bound = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(load().nb_retention(handle, ctypes.byref(past), ctypes.byref(bound), _stream(stream)),
           "nb_retention")
    return int(past.value), int(bound.value)


def nb_resort(handle: ctypes.c_void_p, stream=None) -> None:
    """Rebuilds the sorted order from the current positions (synchronises the stream)."""
    _check(load().nb_resort(handle, _stream(stream)), "nb_resort")


def nb_sorted_order(handle: ctypes.c_void_p, stream=None) -> np.ndarray:
    """The force kernels' sorted slot order: element index per slot, -1 for padding."""
    lib = load()
    total = ctypes.c_int64(0)
    _check(lib.nb_sorted_order(handle, None, 0, ctypes.byref(total), _stream(stream)),
           "nb_sorted_order")
    out = np.zeros(max(int(total.value), 1), dtype=np.int32)
    _check(lib.nb_sorted_order(handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               int(total.value), ctypes.byref(total), _stream(stream)),
           "nb_sorted_order")
    return out[: int(total.value)]


def nb_l1_log(handle: ctypes.c_void_p, max_steps: int = NB_L1_LOG_CAP, stream=None) -> np.ndarray:
    out = np.zeros((max(int(max_steps), 1), 4), dtype=np.int32)
    n = ctypes.c_int32(0)
    _check(load().nb_l1_log(handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            int(max_steps), ctypes.byref(n), _stream(stream)), "nb_l1_log")
    return out[: n.value].copy()


def nb_timing_enable(on: bool) -> None:
    _check(load().nb_timing_enable(int(bool(on))), "nb_timing_enable")


def nb_timing_read() -> tuple[float, int]:
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(load().nb_timing_read(ctypes.byref(ms), ctypes.byref(cnt)), "nb_timing_read")
    return float(ms.value), int(cnt.value)


def nb_timing_reset() -> None:
    _check(load().nb_timing_reset(), "nb_timing_reset")


def nb_tile_config(n: int, n1: int, mode: int, law: int = NB_LAW_CONTACT) -> dict:
    v = [ctypes.c_int32(0) for _ in range(5)]
    _check(load().nb_tile_config(int(n), int(n1), int(mode), int(law),
                                 *[ctypes.byref(x) for x in v]), "nb_tile_config")
    return dict(zip(("ki", "nsplit", "iblock", "jchunk", "rows"), (int(x.value) for x in v)))


def nb_tile_override(n_lo: int, n_hi: int, mode: int, nsplit: int, rows: int = 1,
                     law: int = NB_LAW_CONTACT) -> None:
    _check(load().nb_tile_override(int(n_lo), int(n_hi), int(mode), int(law), int(nsplit),
                                   int(rows)), "nb_tile_override")


def nb_graph_create(handles, n_steps: int, stream=None) -> ctypes.c_void_p:
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                             for h in handles])
    g = ctypes.c_void_p(None)
    _check(load().nb_graph_create(arr, len(handles), int(n_steps), _stream(stream),
                                  ctypes.byref(g)), "nb_graph_create")
    return g


def nb_graph_launch(graph: ctypes.c_void_p, stream=None) -> None:
    _check(load().nb_graph_launch(graph, _stream(stream)), "nb_graph_launch")


def nb_graph_destroy(graph: ctypes.c_void_p) -> None:
    load().nb_graph_destroy(graph)


def nb_set_workspace_budget(nbytes: int) -> None:
    """Workspace budget for systems created afterwards (0: none); see include/nbody.h."""
    _check(load().nb_set_workspace_budget(int(nbytes)), "nb_set_workspace_budget")


def nb_set_force_grid(blocks: int) -> None:
    _check(load().nb_set_force_grid(int(blocks)), "nb_set_force_grid")


def nb_valu_probe(op: int, blocks: int, iters: int, sink, stream=None) -> tuple:
    """(kernel ms, lane-instructions executed, shader-clock cycles per constant-rate counter
    tick) of one vector-ALU issue-rate probe launch; ``sink`` is a device tensor of at least 32
    bytes."""
    ms = ctypes.c_double(0.0)
    ops = ctypes.c_int64(0)
    ratio = ctypes.c_double(0.0)
    _check(load().nb_valu_probe(int(op), int(blocks), int(iters),
                                ctypes.c_void_p(sink.data_ptr()), _stream(stream),
                                ctypes.byref(ms), ctypes.byref(ops), ctypes.byref(ratio)),
           "nb_valu_probe")
    return float(ms.value), int(ops.value), float(ratio.value)


def nb_destroy(handle: ctypes.c_void_p) -> None:
    load().nb_destroy(handle)


from .system import System, step_many  # noqa: E402,F401
