"""Host logic of the cube-graph hierarchy (no GPU): a small C++ checker, built here with g++
against the library's host sources, verifies on several meshes that every colour class is an
independent set covering its level and that the packed 16-bit rows are present exactly on
levels whose couplings share one value, decoding to the same columns."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from bcm_inputs import CHANNEL_BC, OPEN_BC, configs, uniform_mesh
from test_oracle_operators import _tiny_multilevel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1808_04099_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("graph_check") / "graph_check")
    cmd = [gxx, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "host", "graph_check.cpp"),
           os.path.join(CSRC, "mesh.cpp"), os.path.join(CSRC, "coarse.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    return out


def _dump(mesh, d):
    with open(os.path.join(d, "meta.txt"), "w") as fh:
        fh.write(f"{mesh.n_cubes} {mesh.n} {mesh.root_edge!r}\n")
    np.ascontiguousarray(mesh.origin, np.float64).tofile(os.path.join(d, "origin.bin"))
    np.ascontiguousarray(mesh.level, np.int8).tofile(os.path.join(d, "level.bin"))
    np.ascontiguousarray(mesh.nbr, np.int32).tofile(os.path.join(d, "nbr.bin"))
    np.ascontiguousarray(mesh.face_bc, np.int8).tofile(os.path.join(d, "fbc.bin"))


MESHES = {
    "channel_16x8x8": lambda: uniform_mesh((16, 8, 8), 0.125, 4, CHANNEL_BC),
    "open_3x3x3": lambda: uniform_mesh((3, 3, 3), 1.0 / 3, 4, OPEN_BC),
    "tiny_3level": _tiny_multilevel,
    "multilevel_small": lambda: configs.multilevel_small()["mesh"],
}


@pytest.mark.parametrize("name", sorted(MESHES))
def test_graph_colouring_and_packed_rows(checker, tmp_path, name):
    _dump(MESHES[name](), str(tmp_path))
    r = subprocess.run([checker, str(tmp_path)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
    if name.startswith("channel") or name.startswith("open"):
        # lattices: red-black colouring on every level, packed rows on every level of width 6
        levels = [line for line in r.stdout.splitlines() if line.startswith("level")]
        assert levels and all("2 colours" in line for line in levels), r.stdout
        assert all(line.endswith("packed 1") for line in levels if "W 6," in line), r.stdout
        assert any("W 6," in line for line in levels), r.stdout


# ---------------------------------------------------------------------------------------------
# The same host sources built with AddressSanitizer and UndefinedBehaviorSanitizer (g++, CPU
# only): mesh validation, metadata, launch order and the cube-graph hierarchy on valid meshes,
# and the rejection paths on invalid ones, must run without a sanitizer report.
# ---------------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def checker_asan(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("graph_check_asan") / "graph_check")
    cmd = [gxx, "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "host", "graph_check.cpp"),
           os.path.join(CSRC, "mesh.cpp"), os.path.join(CSRC, "coarse.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if r.returncode != 0 and "sanitizer" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return out


def _broken(which):
    m = uniform_mesh((3, 2, 2), 0.25, 4, CHANNEL_BC)
    if which == "unlinked_interior_face":       # boundary kind on a face with a cube across
        m.nbr[0, 1] = -1
        m.face_bc[0, 1] = 1
        o = int(np.argwhere(m.nbr[:, 0, 0] == 0)[0][0])
        m.nbr[o, 0] = -1
        m.face_bc[o, 0] = 1
    elif which == "bad_index":
        m.nbr[2, 3, 0] = m.n_cubes + 5
    elif which == "off_lattice":
        m.origin[4, 1] += 0.01
    return m


@pytest.mark.parametrize("name", sorted(MESHES) + ["unlinked_interior_face", "bad_index",
                                                   "off_lattice"])
def test_host_sources_under_sanitizers(checker_asan, tmp_path, name):
    mesh = MESHES[name]() if name in MESHES else _broken(name)
    _dump(mesh, str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([checker_asan, str(tmp_path)], capture_output=True, text=True,
                       timeout=300, env=env)
    report = r.stdout + r.stderr
    assert "Sanitizer" not in report and "runtime error" not in report, report[-3000:]
    if name in MESHES:
        assert r.returncode == 0 and r.stdout.strip().endswith("ok"), report
    else:
        assert r.returncode == 1 and "mesh rejected" in r.stdout, report
