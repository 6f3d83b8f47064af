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
