"""lbm_nusselt_noalloc (static device scratch, no allocation) against
lbm_nusselt (workspace scratch): the same results bit for bit, on two calls
in a row, the second on a smaller cavity, and the size limit reported as an
argument error before any launch."""
import numpy as np
import pytest

from gpu_helpers import log, to_np

FIELDS = ("nu_hot_wall", "nu_cold_wall", "nu_hot_mid", "nu_cold_mid", "nu_max", "z_max",
          "nu_min", "z_min")


@pytest.mark.gpu
def test_nusselt_noalloc_matches_the_workspace_call():
    import torch
    from paper_1710_04751_amd import capi
    from paper_1710_04751_amd import solver as S

    cases = [  # the second call has fewer wall cells than the first
        dict(nx=40, ny=36, nz=28, Ra=2e4, precision="fp64", thermal_q=15, steps=300),
        dict(nx=12, ny=12, nz=12, Ra=1e3, precision="fp32", thermal_q=7, steps=200),
    ]
    for c in cases:
        log(f"noalloc nusselt: {c}")
        p = S.make_params(c["nx"], c["Ra"], nx=c["nx"], ny=c["ny"], nz=c["nz"],
                          precision=c["precision"], thermal_q=c["thermal_q"])
        cav = S.Cavity(p)
        cav.step(c["steps"])
        shape = (p.nz, p.ny)
        lh0 = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
        lc0 = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
        lh1 = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
        lc1 = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        ref = capi.lbm_nusselt(cav.h, lh0.data_ptr(), lc0.data_ptr())
        got = capi.lbm_nusselt_noalloc(cav.h, lh1.data_ptr(), lc1.data_ptr())
        torch.cuda.synchronize()
        for f in FIELDS:
            assert getattr(got, f) == getattr(ref, f), (f, getattr(got, f), getattr(ref, f))
        assert np.array_equal(to_np(lh1), to_np(lh0)) and np.array_equal(to_np(lc1), to_np(lc0))
        assert np.all(np.isfinite(to_np(lh1))) and abs(ref.nu_hot_wall - ref.nu_cold_wall) < 1.0
        # without profile outputs as well
        bare = capi.lbm_nusselt_noalloc(cav.h)
        for f in FIELDS:
            assert getattr(bare, f) == getattr(ref, f)
        cav.close()


@pytest.mark.gpu
def test_nusselt_noalloc_refuses_walls_beyond_its_scratch():
    import torch
    from paper_1710_04751_amd import capi
    from paper_1710_04751_amd import solver as S

    # ny * nz = 1025 * 1024 > 2^20 wall cells; FP16 storage keeps it small
    p = S.make_params(4, 1e3, nx=4, ny=1025, nz=1024, precision="fp16")
    cav = S.Cavity(p)
    torch.cuda.synchronize()
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_nusselt_noalloc(cav.h)
    assert ei.value.status == capi.LBM_ERR_ARG
    assert "scratch" in capi.lbm_last_error()
    # the workspace call still serves it
    r = capi.lbm_nusselt(cav.h)
    assert np.isfinite(r.nu_hot_wall)
    cav.close()
