"""512^3 cavity at Ra 1e6 against the 128^3 FP64 oracle (tests/golden/), in
the precision forms of the benchmark: 10,000 steps from rest with FP32 and
with FP16 storage (FP32 arithmetic), against the oracle's 2,500 steps (the
same t u0 / L), compared as 4x4x4 block means on the oracle's mid-planes
y = 64 and z = 64 (bench.precision_study).

FP32 against the oracle is a comparison of two grids (512^3 and 128^3), not
of arithmetic: the Ra 1e6 boundary layers are 4 cells thick on 128^3, so
the bars are set at about twice the measured differences (T max 5.9e-3, rms
4.8e-4; velocity, over the peak speed component, max 0.10, rms 4.7e-3).

FP16 storage rounds every stored population to nearest (11 significant
bits).  The scalar populations are stored as they are (|g| up to 1/8), so
each store can drop an update below half an ulp (3e-5 - 6e-5), and in the
slowly changing bulk the same rounding repeats step after step instead of
averaging out.  Measured after 10,000 steps: T differs from FP32 by 3.3% of
max |T| in rms (14.8% max), the velocity by 4.3% in rms.  The bars (twice
those) guard that finding; the FP32 bars above show the scheme itself is
accurate.

FP16 storage with stochastic rounding removes the bias: every store errs by
less than one ulp (<= 2^-13 for |g| <= 1/8) with mean zero, so T (7
populations) takes a random walk of at most sqrt(7) 2^-13 per step, i.e.
1.6e-2 of T's scale after 10,000 steps even without any damping; the bar
is that bound (T rms 3.2e-2 of max |T| = 0.5).  Measured: T rms 5.0e-5, max
8.4e-4 (diffusion averages the walk out), 650 times below round-to-nearest."""
import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def study():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    log("case: 512^3 Ra 1e6 FP32 and FP16 storage, 10,000 steps, vs 128^3 oracle")
    out = bench.precision_study(log=log)
    assert out is not None, "tests/golden/cavity128_ra1e6_d3q7_2500.npz is missing"
    log(out)
    return out


def _u(e, suffix=""):
    return max(e["ux" + suffix], e["uy" + suffix], e["uz" + suffix])


def test_fp32_512_matches_the_128_oracle(study):
    e = study["fp32"]["vs_oracle128"]
    assert e["T"] < 1.2e-2 and e["T_rms"] < 1e-3
    assert _u(e) < 0.2 and _u(e, "_rms") < 1e-2


def test_fp16_storage_error_stays_within_its_measured_bound(study):
    d = study["fp16_vs_fp32"]
    assert d["T_rms"] < 0.066 and d["T"] < 0.3
    assert _u(d, "_rms") < 0.09
    e32, e16 = study["fp32"]["vs_oracle128"], study["fp16"]["vs_oracle128"]
    # the FP16 difference is the storage's, not the grid's: FP32 is the closer one
    assert e32["T_rms"] < e16["T_rms"]


def test_fp16_stochastic_rounding_is_unbiased(study):
    d, d_rne = study["fp16_sr_vs_fp32"], study["fp16_vs_fp32"]
    assert d["T_rms"] < 3.2e-2 and d["T"] < 3.2e-2
    assert _u(d, "_rms") < 3.2e-2
    assert d["T_rms"] < 0.01 * d_rne["T_rms"]
