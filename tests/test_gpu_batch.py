"""Batched form: many cavities in one persistent launch per step.

Each member must evolve exactly as the same cavity run alone (the batched
and single-cavity kernels share the per-cell update), whatever the launch
shape, graph replay or retirement of other members; a member also matches
the oracle directly."""
import math

import numpy as np
import pytest

from gpu_helpers import field_errors, log, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def solver():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_04751_amd import solver as S
    return S


def _members(solver, prec, qt, sizes, ras, **extra):
    ps = []
    for (nx, ny, nz), ra in zip(sizes, ras):
        ps.append(solver.make_params(nx=nx, ny=ny, nz=nz, Ra=ra, precision=prec, thermal_q=qt,
                                     u0=0.1, omega_bulk=1.0, fourth_maxwell=1, **extra))
    return ps


SIZES = [(32, 32, 32), (48, 40, 36), (20, 28, 16), (64, 16, 24), (96, 12, 10)]
RAS = [1e4, 3e4, 2e3, 5e4, 1e5]


@pytest.mark.parametrize("prec,qt,spec,sr", [("fp32", 7, 0, 0), ("fp64", 15, 0, 0),
                                              ("fp16", 7, 0, 0), ("fp32", 15, 1, 0),
                                              ("fp16", 7, 0, 1), ("fp16", 15, 1, 1)])
def test_batch_equals_single_runs(solver, prec, qt, spec, sr):
    """130 steps: one graph replay of 100 steps and 30 single launches; with
    stochastic rounding each member draws the random bits of its own single
    run (the step keys advance on the device across replays)."""
    log(f"case: batch vs single {prec} q{qt} specular {spec} stochastic rounding {sr}")
    params = _members(solver, prec, qt, SIZES, RAS, scalar_specular=spec, round_stochastic=sr)
    batch = solver.Batch(params)
    batch.step(130)  # graph replay (100) + single launches
    info = batch.launch_info()
    assert info["steps"] == 130 and info["graph_steps"] == 100
    for i, p in enumerate(params):
        cav = solver.Cavity(p)
        cav.step(130)
        Fs, Gs = cav.populations()
        Fb, Gb = batch.members[i].populations()
        assert torch.equal(Fs, Fb) and torch.equal(Gs, Gb), i
        cav.close()
    batch.close()


def test_retired_member_freezes_and_rejoins(solver):
    log("case: batch retirement")
    params = _members(solver, "fp32", 7, SIZES[:3], RAS[:3])
    batch = solver.Batch(params)
    batch.step(40)
    batch.set_active([1, 0, 1])
    batch.step(60)
    batch.set_active([1, 1, 1])  # rejoins at an even step: its state is in step
    batch.step(20)
    expect = [120, 60, 120]
    for i, p in enumerate(params):
        assert batch.members[i].steps_done() == expect[i]
        cav = solver.Cavity(p)
        cav.step(expect[i])
        assert torch.equal(cav.populations()[0], batch.members[i].populations()[0]), i
        cav.close()
    batch.close()


def test_stochastic_rounding_keys_follow_each_member(solver):
    """FP16 storage with stochastic rounding: a member that sat out steps and
    one re-initialised mid-run keep drawing the random bits of their own
    single runs (keys = each member's step count), through graph replays."""
    log("case: batch stochastic rounding with retirement and restart")
    params = _members(solver, "fp16", 7, SIZES[:3], RAS[:3], round_stochastic=1)
    batch = solver.Batch(params)
    batch.step(40)
    batch.set_active([1, 0, 1])
    batch.step(60)
    batch.members[2].init_rest()  # batch step 100 (even): restarts at step 0
    batch.set_active([1, 1, 1])
    batch.step(120)  # one graph replay and 20 single launches
    expect = [220, 160, 120]
    for i, p in enumerate(params):
        assert batch.members[i].steps_done() == expect[i]
        cav = solver.Cavity(p)
        cav.step(expect[i])
        Fs, Gs = cav.populations()
        Fb, Gb = batch.members[i].populations()
        assert torch.equal(Fs, Fb) and torch.equal(Gs, Gb), i
        cav.close()
    batch.close()


@pytest.mark.parametrize("bpc", [0, 3])
def test_launch_shapes_with_graphs_and_retirement(solver, bpc):
    """One block per tile of the whole batch (bpc = 0; blocks past the active
    tiles return at once) or a persistent grid of 3 blocks per compute unit,
    replayed from graphs of 20 steps while two members retire and rejoin:
    every member bit-identical to the same cavity run alone."""
    log(f"case: batch launch bpc={bpc}, graphs of 20 steps, retirement")
    params = _members(solver, "fp32", 7, SIZES, RAS)
    batch = solver.Batch(params)
    batch.set_launch(256, bpc, 20)
    info = batch.launch_info()
    assert info["threads"] == 256 and info["graph_steps"] == 20
    if bpc == 0:
        # tiles of 256 // nx whole x-rows of one plane
        tiles = sum(nz * -(-ny // max(1, 256 // nx)) for nx, ny, nz in SIZES)
        assert info["grid_blocks"] == tiles == info["active_tiles"]
    batch.step(40)
    batch.set_active([1, 0, 1, 1, 0])
    batch.step(60)
    batch.set_active([1, 1, 1, 1, 1])
    batch.step(20)
    expect = [120, 60, 120, 120, 60]
    for i, p in enumerate(params):
        assert batch.members[i].steps_done() == expect[i]
        cav = solver.Cavity(p)
        cav.step(expect[i])
        Fs, Gs = cav.populations()
        Fb, Gb = batch.members[i].populations()
        assert torch.equal(Fs, Fb) and torch.equal(Gs, Gb), i
        cav.close()
    batch.close()


def test_autotuned_shape_gives_identical_results(solver):
    params = _members(solver, "fp32", 7, SIZES, RAS)
    batch = solver.Batch(params)
    threads, bpc = batch.autotune(steps_per_trial=4)
    log("case: batch autotune ->", threads, bpc)
    assert threads % 64 == 0 and threads >= 96 and 0 <= bpc <= 32
    done = batch.launch_info()["steps"]
    assert done % 2 == 0
    batch.step(100)
    for i, p in enumerate(params):
        cav = solver.Cavity(p)
        cav.step(done + 100)
        assert torch.equal(cav.populations()[1], batch.members[i].populations()[1]), i
        cav.close()
    batch.close()


def test_batch_member_matches_oracle(solver, oracle):
    log("case: batch member vs oracle fp64")
    params = _members(solver, "fp64", 7, [(14, 12, 10), (16, 16, 16)], [2e3, 1e3])
    batch = solver.Batch(params)
    batch.step(300)
    for i, (nx, ny, nz) in enumerate([(14, 12, 10), (16, 16, 16)]):
        p = oracle.cavity_params(nx, [2e3, 1e3][i], u0=0.1, ny=ny, nz=nz, omega_bulk=1.0,
                                 fourth_maxwell=1)
        F, G = oracle.rest_state(p)
        _, _, mac = oracle.run(p, 300, F, G)
        m = {k: to_np(v) for k, v in batch.members[i].macros(fp64=True).items()}
        err = field_errors(m, mac)
        log(i, err)
        assert err["rho"] < 1e-12 and err["u"] < 1e-12 and err["T"] < 1e-12
    batch.close()


def test_run_to_steady_and_residuals(solver):
    log("case: batch run to steady")
    params = _members(solver, "fp64", 7, [(12, 12, 12), (16, 12, 14), (10, 10, 10)],
                      [1e3, 2e3, 5e2])
    batch = solver.Batch(params)
    steps, status, res = batch.run_to_steady(tol=1e-9, check_every=500, max_steps=60000)
    log("steps", steps, "status", status, "res", res)
    assert all(s == 0 for s in status)
    assert all(r < 1e-9 for r in res)
    assert all(s > 0 and s % 500 == 0 for s in steps)
    # each member stopped where it converged and stays there
    for i in range(3):
        assert batch.members[i].steps_done() == steps[i]
    assert batch.launch_info()["active_tiles"] == 0
    # smaller Ra (faster diffusion relative to the box) converges first
    assert steps[2] <= steps[0]
    batch.close()


def test_member_misuse_is_refused(solver):
    from paper_1710_04751_amd import capi
    params = _members(solver, "fp32", 7, SIZES[:2], RAS[:2])
    batch = solver.Batch(params)
    h = batch.members[0].h
    with pytest.raises(capi.LbmError) as e:
        capi.lbm_step(h, 1)
    assert e.value.status == capi.LBM_ERR_STATE
    batch.step(1)
    with pytest.raises(capi.LbmError) as e:
        capi.lbm_init_rest(h)
    assert e.value.status == capi.LBM_ERR_STATE
    batch.close()


def test_largest_batch(solver):
    """255 members (the limit) of small uneven boxes in one launch; a sample
    of members equals its single-cavity run bit for bit."""
    import numpy as np
    log("case: batch of 255 members")
    rng = np.random.default_rng(255)
    sizes = [tuple(int(v) for v in rng.integers(4, 12, 3)) for _ in range(255)]
    ras = [float(10 ** rng.uniform(3, 4)) for _ in range(255)]
    params = _members(solver, "fp32", 7, sizes, ras)
    batch = solver.Batch(params)
    batch.step(60)
    for i in (0, 17, 128, 254):
        cav = solver.Cavity(params[i])
        cav.step(60)
        assert torch.equal(cav.populations()[0], batch.members[i].populations()[0]), i
        cav.close()
    batch.close()
