"""Every direct global-to-LDS load of the pipelined split-bf16 GEMMs stays inside its operand, at
the shapes the library launches them with (projection, nonlocal product, Gram product, rotation)
for the workload cells and serving cells, and at ragged shapes.  The test compiles a host program
that runs the kernels' own address arithmetic (pipe_addr.hpp) over every load of the first and
last K tile of every workgroup tile.  CPU only."""
import os
import shutil
import subprocess

import pytest

from paper_2406_10765_amd import pw, synth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("pipe") / "pipe_bounds")
    subprocess.run([cxx, "-O2", "-std=c++17", os.path.join(HERE, "pipe_bounds.cpp"), "-o", exe], check=True)
    return exe


def run(exe, *args):
    r = subprocess.run([exe] + [str(a) for a in args], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def shapes(cell):
    info = pw.plan(cell, pw.PW_MIXED, flags=pw.PW_FLAG_BF16_ALL)
    npw, nproj, nb, nbb = int(info.npw), int(info.nproj), int(info.nbands), int(info.filter_block)
    ldw = (npw + 15) // 16 * 16
    out = [("nn", npw, nbb, nproj, ldw, nproj),   # nonlocal product: beta planes x D P planes
           ("nn", npw, nb, nb, ldw, nb),          # rotation: block planes x coefficient planes
           ("cn", nproj, nbb, npw, ldw, ldw, 29),  # projection
           ("cn", nb, 2 * nb, npw, ldw, ldw, 25)]  # Gram / projected matrix
    return out


CELLS = [synth.make_cell("si8"), synth.make_cell("si64"), synth.make_cell("si512"),
         synth.silicon_cell((3, 3, 3), 20.0), synth.silicon_cell((1, 1, 2), 15.0)]


@pytest.mark.parametrize("cell", CELLS, ids=["si8", "si64", "si512", "si216_e20", "si16_e15"])
def test_pipeline_loads_in_bounds_at_product_shapes(harness, cell):
    for s in shapes(cell):
        if s[0] == "nn" and s[3] % 16:
            continue  # the launcher keeps the previous kernel when K is not a multiple of 16
        run(harness, *s)


@pytest.mark.parametrize("args", [("nn", 5000, 300, 512, 5008, 512), ("cn", 600, 300, 10000, 10016, 10016, 4),
                                  ("nn", 1, 1, 16, 4, 16), ("cn", 1, 1, 1, 16, 16, 1),
                                  ("nn", 257, 129, 32, 260, 32), ("cn", 255, 127, 17, 32, 32, 2)])
def test_pipeline_loads_in_bounds_at_ragged_shapes(harness, args):
    run(harness, *args)
