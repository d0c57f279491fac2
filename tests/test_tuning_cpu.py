"""CPU-side checks of the saved work-split table (paper_2303_12166_amd/tuning/gfx950.json): its
buckets tile the size range the tuner covers, every choice is one the kernels build, and loading
the library installs each choice (no GPU calls)."""

import json
import os

import pytest

from paper_2303_12166_amd import autotune

pytestmark = pytest.mark.skipif(not os.path.exists(autotune.TABLE_PATH),
                                reason="no saved table")


@pytest.fixture(scope="module")
def nb():
    import paper_2303_12166_amd as nb
    from paper_2303_12166_amd import build

    if not os.path.exists(nb.lib_path()):
        build.build()
    nb.load()
    return nb


@pytest.fixture(scope="module")
def table():
    with open(autotune.TABLE_PATH) as f:
        return json.load(f)


def test_table_header(nb, table):
    assert table["arch"] == "gfx950"
    assert table["library_version"] == nb.nb_version()
    assert sorted(table["tables"]) == sorted(autotune.KEYS)


@pytest.mark.parametrize("key", autotune.KEYS)
def test_buckets_tile_the_tuned_range(table, key):
    got = [(b["n_lo"], b["n_hi"]) for b in table["tables"][key]["buckets"]]
    want = autotune.buckets()[:len(got)]
    assert got == want
    # every bucket up to the one holding the largest tuned size (262,144)
    assert got[-1][0] <= 262144 <= got[-1][1]


@pytest.mark.parametrize("key", autotune.KEYS)
def test_choices_are_buildable(table, key):
    mode, _ = autotune.split_key(key)
    for b in table["tables"][key]["buckets"]:
        assert b["rows"] in autotune.ROWS[mode], b
        assert b["nsplit"] in autotune.CHUNKS, b
        assert b["n_lo"] <= b["n_tuned"] <= b["n_hi"], b
        assert b["ms"] > 0, b
        assert "%d:%d" % (b["rows"], b["nsplit"]) in b["candidates_ms"], b


@pytest.mark.parametrize("key", autotune.KEYS)
def test_loading_installs_every_choice(nb, table, key):
    mode, law = autotune.split_key(key)
    q = table["tables"][key]["q"]
    for b in table["tables"][key]["buckets"]:
        for n in sorted({b["n_lo"], b["n_tuned"], min(b["n_hi"], 1 << 20)}):
            n1 = n - int(n * q / (1 + q))
            cfg = nb.nb_tile_config(n, n1, nb.MODES[mode], nb.LAWS[law])
            assert cfg["rows"] == b["rows"], (key, n, b, cfg)
            # the runtime may merge chunks (a chunk holds whole tiles), never split them further
            assert 1 <= cfg["nsplit"] <= b["nsplit"], (key, n, b, cfg)
