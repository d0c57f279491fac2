"""The C ABI from C: tests/c_abi_check.c is compiled with gcc against include/nbody.h, linked
against the built libnbody.so and run (host-only entry points, no GPU)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def c_output(tmp_path_factory):
    import paper_2303_12166_amd as nb
    from paper_2303_12166_amd import build

    if not os.path.exists(nb.lib_path()):
        build.build()
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("cabi") / "c_abi_check")
    libdir = os.path.dirname(nb.lib_path())
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_abi_check.c"), nb.lib_path(),
                    "-Wl,-rpath," + libdir, "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120, check=True).stdout
    return dict(line.split(" ", 1) for line in out.strip().splitlines())


def test_scratch_bytes_from_c(c_output):
    rc, nbytes = c_output["scratch"].split()
    assert rc == "0" and int(nbytes) > 0
    rc_p, nbytes_p = c_output["paper"].split()
    # at N = 2048 the contact law splits its units by j group (four times the chunk partials)
    # and the paper law does not, so the two sizes are not ordered; both must be valid
    assert rc_p == "0" and int(nbytes_p) > 0 and int(nbytes_p) != int(nbytes)


def test_errors_from_c(c_output):
    assert c_output["plain-paper"].startswith("-1 ")  # NB_E_INVAL: no plain kernel for eqs. 4-6
    assert c_output["create-null"] == "-1 null"


def test_tile_config_and_version_from_c(c_output):
    rc, ki, ns, ib, jc, rows = (int(x) for x in c_output["tile"].split())
    assert rc == 0 and ki == 1 and ib == 256 and ns >= 1 and jc % 256 == 0
    assert rows in (1, 2, 4)
    assert int(c_output["version"]) >= 4
