"""Host-side pieces of the server that need no GPU: footprints and summary statistics."""

import math

import pytest


@pytest.fixture(scope="module")
def serve():
    import paper_2303_12166_amd as nb
    from paper_2303_12166_amd import build

    import os

    if not os.path.exists(nb.lib_path()):
        build.build()
    from paper_2303_12166_amd import serve as s

    return s


def test_footprint_grows_with_n(serve):
    a = serve.footprint_bytes(4096, 0.5)
    b = serve.footprint_bytes(131072, 0.5)
    assert 0 < a < b
    # at least the nine FP32 state arrays
    assert b >= 9 * 4 * 131072
    # FP64 doubles the state, the partials and the reactions of the same work split (at 4096 the
    # FP32 Kahan split has four times the partials of small-system units, so compare at 131072)
    assert serve.footprint_bytes(131072, 0.5, "fp64") > b


def test_summary_statistics(serve):
    R = serve.Record
    recs = [R(0, 100, 0.5, 10, 0.0, 0.0, 1.0, status="done"),
            R(1, 200, 0.5, 10, 0.5, 0.5, 2.5, status="done"),
            R(2, 300, 0.5, 10, 1.0, 1.0, 4.0, status="done"),
            R(3, 300, 0.5, 10, 1.0, status="rejected")]
    s = serve.summarize(recs)
    assert s["completed"] == 3 and s["rejected"] == 1
    assert s["span_s"] == pytest.approx(4.0)
    assert s["sims_per_s"] == pytest.approx(0.75)
    assert s["latency_p50_s"] == pytest.approx(2.0)
    assert s["latency_max_s"] == pytest.approx(3.0)
    assert s["interactions_per_s"] == pytest.approx((100**2 + 200**2 + 300**2) * 10 / 4.0)
    assert serve.summarize([R(0, 1, 0.5, 1, 0.0)])["completed"] == 0
    assert not math.isnan(s["latency_p99_s"])
