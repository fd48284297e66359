"""Host logic of the warm-start pipeline (no GPU): the per-channel scaling of
the training targets."""
import pytest

torch = pytest.importorskip("torch")


def test_channel_scale_brings_each_channel_to_the_target_rms():
    from paper_1710_04751_amd import warmstart as WS
    g = torch.Generator().manual_seed(3)
    t = torch.randn(5, 4, 3, 3, 3, generator=g, dtype=torch.float64)
    t[:, 1] *= 1e-3  # a channel 1000 times smaller, as the spanwise velocity is
    t[:, 3] += 0.25  # and one with a mean
    sc = WS.channel_scale(t.float(), rms=0.5)
    assert len(sc) == 4
    for c in range(4):
        rms = float((t[:, c] * sc[c]).pow(2).mean().sqrt())
        assert abs(rms - 0.5) < 1e-5, (c, rms)
    # the small channel gets the large factor
    assert sc[1] > 500 * sc[0]


def test_channel_scale_refuses_an_all_zero_channel():
    from paper_1710_04751_amd import warmstart as WS
    t = torch.ones(2, 4, 2, 2, 2)
    t[:, 2] = 0.0
    with pytest.raises(ValueError):
        WS.channel_scale(t)
