"""The stored state layout that lbm_state_info documents (include/lbm.h):
groups of Rg = pop_stride / nx consecutive x-rows, one run per population
per group.  Populations written through lbm_set_populations, with values
exact in every storage type, are read back from the raw state at the
documented positions, and Rg follows the stated rule (the largest power of
two with one run within 32 KB and no more rows than the grid has)."""
import numpy as np
import pytest

from gpu_helpers import log, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FLOW_W = np.array([2 / 9] + [1 / 9] * 6 + [1 / 72] * 8)


@pytest.fixture(scope="module")
def solver():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_04751_amd import solver as S
    return S


@pytest.mark.parametrize("shape,qt,prec", [((17, 9, 5), 15, "fp64"), ((16, 16, 16), 7, "fp64"),
                                           ((40, 6, 4), 7, "fp32"), ((33, 7, 9), 15, "fp16"),
                                           ((512, 4, 4), 7, "fp32")])
def test_state_layout_matches_the_documented_formula(solver, shape, qt, prec):
    from paper_1710_04751_amd import capi
    nx, ny, nz = shape
    log(f"case: layout {shape} q{qt} {prec}")
    cav = solver.Cavity(solver.make_params(nx=nx, ny=ny, nz=nz, Ra=1e3, precision=prec,
                                           thermal_q=qt))
    n = cav.ncell
    rng = np.random.default_rng(5)
    # deviations k/1024 with |k| < 64: exact in FP16, FP32 and FP64
    dF = rng.integers(-64, 64, size=(15, n)) / 1024.0
    G = rng.integers(-64, 64, size=(qt, n)) / 1024.0
    cav.set_populations(FLOW_W[:, None] + dF, G)
    F0, G0, stride, vb = cav.state_info()
    rq, nrows = 15 + qt, ny * nz
    rg = stride // nx
    expect_rg = 1
    while 2 * expect_rg * nx * vb <= 32768 and 2 * expect_rg <= nrows:
        expect_rg *= 2
    assert stride == rg * nx and rg == expect_rg
    assert G0 - F0 == 15 * stride * vb
    nvals = -(-nrows // rg) * rq * stride
    dtype = {8: torch.float64, 4: torch.float32, 2: torch.float16}[vb]
    raw = torch.zeros(nvals + 16, dtype=dtype, device="cuda")
    # the state is 256-byte aligned and sized, so a copy rounded up to 16 bytes stays inside it
    capi.lbm_copy_probe(raw.data_ptr(), F0, (nvals * vb + 15) // 16 * 16)
    torch.cuda.synchronize()
    raw = to_np(raw)[:nvals].astype(np.float64)
    c = np.arange(n)
    r, x = c // nx, c % nx
    hit = np.zeros(nvals, dtype=np.int32)
    for a in range(rq):
        idx = ((r // rg) * rq + a) * stride + (r % rg) * nx + x
        want = dF[a] if a < 15 else G[a - 15]
        assert np.max(np.abs(raw[idx] - want)) <= 1e-15, a
        hit[idx] += 1
    # one position per (cell, population); the rest is the last group's padding
    assert hit.max() == 1 and hit.sum() == n * rq
    log(shape, prec, "rows per group", rg)
    cav.close()
