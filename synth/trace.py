"""Synthetic request trace for the serving workload.

Each request asks for one two-star run: Poisson arrivals at a mean rate, N log-uniform in a range
and rounded to a multiple of 64, q uniform, the particle seed equal to the request id. The draws
come from their own PCG64 stream so that the trace is fixed by (count, rate, seed).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    t_arrive: float
    n: int
    q: float
    steps: int
    seed: int


def make_trace(
    count: int = 256,
    rate: float = 20.0,
    n_min: int = 4096,
    n_max: int = 131072,
    q_min: float = 0.1,
    q_max: float = 1.0,
    steps: int = 500,
    seed: int = 2303_12166,
) -> list[Request]:
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]  # first request arrives at t = 0
    logn = rng.uniform(math.log(n_min), math.log(n_max), size=count)
    qs = rng.uniform(q_min, q_max, size=count)
    out = []
    for k in range(count):
        n = int(64 * round(math.exp(logn[k]) / 64.0))
        n = min(max(n, n_min), n_max)
        out.append(Request(rid=k, t_arrive=float(t[k]), n=n, q=float(qs[k]), steps=steps, seed=k))
    return out
