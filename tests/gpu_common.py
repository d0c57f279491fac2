"""Helpers shared by the GPU tests (inputs and error metrics only; no arithmetic of the method)."""

from __future__ import annotations

import numpy as np


def require_gpu():
    import torch

    import paper_2303_12166_amd as nb

    nb.load()  # raises if the HIP library is missing: GPU tests never run without it
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return nb


def force_error(a_gpu: np.ndarray, a_ref: np.ndarray) -> float:
    """max_i |a_gpu,i - a_ref,i| / max_k |a_ref,k| (per-element relative to the largest force)."""
    scale = np.linalg.norm(a_ref, axis=1).max()
    if scale == 0.0:
        return float(np.abs(a_gpu).max())
    return float(np.linalg.norm(a_gpu - a_ref, axis=1).max() / scale)


def sample_rows(n: int, n1: int, k: int, seed: int = 0) -> np.ndarray:
    """Rows spanning both stars, both ends, the star boundary and block edges, plus random ones."""
    rng = np.random.default_rng(seed)
    fixed = [0, 1, 255, 256, 511, 512, n1 - 1, n1, n1 + 1, n - 2, n - 1]
    rows = set(r for r in fixed if 0 <= r < n)
    rows.update(int(r) for r in rng.integers(0, n, size=max(k - len(rows), 0)))
    return np.array(sorted(rows), dtype=np.int64)


def print_case(*parts):
    print("[case]", *parts, flush=True)
