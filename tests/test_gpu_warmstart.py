"""The learned warm start end to end at a small size: steady 32^3 cavities
from the batched solver train the network on the GPU; held-out Rayleigh
numbers started from its prediction reach the steady rule in fewer steps
than from rest, at the same steady Nusselt number (within 0.5%)."""
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
    r = warmstart.study(grid=32, n_train=24, n_test=6, ra_range=(1e3, 2e4), epochs=300, batch=8,
                        lr=2e-3, max_steps=300_000, log=log)
    for row in r["rows"]:
        log(row)
    log({k: v for k, v in r.items() if k != "rows"})
    return r


def test_every_cavity_reaches_the_steady_rule(result):
    assert result["train_converged"] == 24 and result["test_converged"] == 6
    assert result["fallbacks"] == 0


def test_warm_start_cuts_steps(result):
    assert result["warm_steps_mean"] < result["cold_steps_mean"]
    assert result["steps_ratio_median"] < 1.0


def test_nusselt_number_is_unchanged(result):
    assert result["nu_rel_diff_max"] < 5e-3
