"""CPU enumeration of the step kernel's load and store offsets (no GPU).

tests/step_index_check.cpp compiles the step's own index functions
(lbm_index.hpp) for the host and walks the blocks of a launch: every offset
must stay inside the block's window of the state (the buffer resource the
kernel loads through) and address the population and cell the pull and
wall rules name, by the documented layout formula.  Small ragged boxes are
checked on every cell; the 512^3 and 1024^3 boxes (state offsets beyond
4 GiB) on every block's first and last row and on all face cells."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
VB = {"fp64": 8, "fp32": 4, "fp16": 2}


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("idx") / "step_index_check")
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"
    subprocess.run([hipcc, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                    os.path.join(HERE, "step_index_check.cpp"), "-o", exe], check=True,
                   stderr=subprocess.DEVNULL)
    return exe


def _valid(nx, ny, nz, qt, prec):
    """Whether the library accepts the box (the window limit of lbm_create)."""
    from paper_1710_04751_amd import capi
    from paper_1710_04751_amd import solver as S
    p = S.make_params(nx, 1e4, nx=nx, ny=ny, nz=nz, precision=prec, thermal_q=qt)
    return capi.lib().lbm_workspace_bytes(p) != 0


def _run(checker, nx, ny, nz, qt, prec, by, spec, mode):
    r = subprocess.run([checker, *map(str, (nx, ny, nz, qt, VB[prec], by, spec, mode))],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
    return int(r.stdout.split()[1])


SMALL = [(37, 23, 19), (4, 4, 4), (5, 4, 6), (6, 5, 4), (64, 7, 5), (17, 33, 9)]


@pytest.mark.parametrize("shape", SMALL)
@pytest.mark.parametrize("qt,spec", [(7, 0), (15, 0), (15, 1)])
@pytest.mark.parametrize("prec", ["fp32", "fp16", "fp64"])
def test_every_cell_of_small_boxes(checker, shape, qt, spec, prec):
    nx, ny, nz = shape
    n = 0
    for by in (1, 2, 4):
        n += _run(checker, nx, ny, nz, qt, prec, by, spec, 0)
    assert n > 0


@pytest.mark.parametrize("n,qt,prec,by,spec", [
    (512, 7, "fp32", 1, 0), (512, 7, "fp32", 2, 0), (512, 7, "fp16", 1, 0),
    (512, 7, "fp64", 1, 0), (512, 15, "fp32", 1, 1), (1024, 7, "fp32", 1, 0),
    (1024, 7, "fp16", 2, 0)])
def test_blocks_of_the_largest_boxes(checker, n, qt, prec, by, spec):
    if not _valid(n, n, n, qt, prec):
        pytest.skip(f"{n}^3 {prec} q{qt} is refused by the library")
    assert _run(checker, n, n, n, qt, prec, by, spec, 1) > 0
