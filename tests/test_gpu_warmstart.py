"""The learned warm start end to end at a small size: steady 32^3 cavities
from the batched solver (FP64, the steady rule of the benchmark) train the
network on the GPU; held-out Rayleigh numbers started from its prediction
reach the steady rule in fewer steps than from rest, at the same steady
Nusselt number (within 0.5%).

FP64, not the benchmark's FP32: in FP32 a 32^3 cavity never reaches the
rule's residual tolerance (1e-8) and its run ends when the residual stops
falling at the rounding floor, which happens at a step that varies by tens
of thousands between neighbouring Rayleigh numbers (22,000 and 41,000 steps
from rest at log10 Ra 3.071 and 3.069).  Step ratios there measure that
floor as much as the start; in FP64 every run ends by the tolerance.

Range: Ra in [1e3, 8e3].  On the 32^3 grid the symmetric steady state stops
being an attractor from Ra ~ 1e4 (the staggered and antisymmetric modes of
the discrete model grow), and warm starts there can leave it.  Even a start
from the exact steady (u, T) takes 60-70% of the steps from rest here: its
populations lack the non-equilibrium part and the density field, and the
transient that follows has to fall below the tolerance too.  With targets
brought to one RMS per channel the median per-cavity ratio was 0.67 (every
cavity 0.60-0.76); with one velocity scale for u, v and w it was 1.0, since
the small spanwise component went unlearnt.  The bar is a median below 0.8
over 24 held-out cavities; the 64^3 study of the benchmark is the full-size
measurement."""
import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def result():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_04751_amd import warmstart
    log("case: warm start study 32^3")
    r = warmstart.study(grid=32, n_train=48, n_test=24, ra_range=(1e3, 8e3), epochs=500, batch=8,
                        lr=2e-3, max_steps=300_000, precision="fp64", log=log)
    for row in r["rows"]:
        log(row)
    log({k: v for k, v in r.items() if k != "rows"})
    return r


def test_every_cavity_reaches_the_steady_rule(result):
    assert result["train_converged"] == 48 and result["test_converged"] == 24
    assert result["fallbacks"] == 0


def test_warm_start_cuts_steps(result):
    assert result["steps_ratio_median"] < 0.8


def test_nusselt_number_is_unchanged(result):
    assert result["nu_rel_diff_max"] < 5e-3
