"""GPU observables against the oracle: the FP64 Nusselt reduction, the
steady-state residual, NaN detection and the macroscopic-field output."""
import math

import numpy as np
import pytest

from gpu_helpers import log, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def solver():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_04751_amd import solver as S
    return S


def _summary(nh, nc):
    """Face means, mid-line (y = L/2) means and hot-line extremes."""
    nz, ny = nh.shape
    y0, y1 = (ny // 2, ny // 2) if ny % 2 else (ny // 2 - 1, ny // 2)
    lh = 0.5 * (nh[:, y0] + nh[:, y1])
    lc = 0.5 * (nc[:, y0] + nc[:, y1])
    return {"nu_hot_wall": nh.mean(), "nu_cold_wall": nc.mean(), "nu_hot_mid": lh.mean(),
            "nu_cold_mid": lc.mean(), "nu_max": lh.max(), "z_max": (np.argmax(lh) + 0.5) / nz,
            "nu_min": lh.min(), "z_min": (np.argmin(lh) + 0.5) / nz}


@pytest.mark.parametrize("qt,n", [(7, 16), (15, 13)])
def test_nusselt_matches_oracle(solver, oracle, qt, n):
    log(f"case: nusselt {n}^3 q{qt} fp64")
    p = oracle.cavity_params(n, 1e3, qt=qt)
    F, G = oracle.rest_state(p)
    F, G, _ = oracle.run(p, 600, F, G)
    nh, nc = oracle.nusselt(p, G)
    ref = _summary(nh, nc)
    cav = solver.Cavity(solver.make_params(n, 1e3, precision="fp64", thermal_q=qt))
    cav.step(600)
    r, lh, lc = cav.nusselt(local=True)
    lh, lc = to_np(lh), to_np(lc)
    assert np.max(np.abs(lh - nh)) < 1e-11 * np.max(np.abs(nh))
    assert np.max(np.abs(lc - nc)) < 1e-11 * np.max(np.abs(nc))
    for k, v in ref.items():
        assert abs(getattr(r, k) - v) <= 1e-11 * max(1.0, abs(v)), (k, getattr(r, k), v)
    log("nusselt", {k: getattr(r, k) for k in ref})
    cav.close()


def test_residual_matches_oracle(solver, oracle):
    log("case: residual 16^3 fp64")
    p = oracle.cavity_params(16, 1e3)
    F, G = oracle.rest_state(p)
    F, G, m1 = oracle.run(p, 500, F, G)
    F, G, m2 = oracle.run(p, 300, F, G)
    ref = np.max(np.abs(m2[4] - m1[4]))
    cav = solver.Cavity(solver.make_params(16, 1e3, precision="fp64"))
    cav.step(500)
    s, v = cav.residual()
    assert s == 0 and math.isinf(v)
    cav.step(300)
    s, v = cav.residual()
    assert s == 0
    assert abs(v - ref) <= 1e-12 * max(ref, 1e-30) + 1e-15, (v, ref)
    cav.close()


def test_nan_is_reported_unstable(solver):
    """A NaN forced into the initial temperature (from the host) surfaces as
    LBM_ERR_UNSTABLE at the next residual; the kernels just carry the NaN."""
    from paper_1710_04751_amd import capi
    log("case: NaN detection")
    cav = solver.Cavity(solver.make_params(16, 1e3, precision="fp32"))
    T = torch.zeros(cav.shape)
    T[5, 6, 7] = float("nan")
    cav.init_macros(T=T)
    cav.step(2)
    s, v = cav.residual()
    assert s == capi.LBM_ERR_UNSTABLE and math.isnan(v)
    cav.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_macros_single_and_double(solver, oracle, prec):
    """lbm_macros in both output types agree with the oracle's pre-collision
    moments of the same step."""
    p = oracle.cavity_params(12, 2e3, u0=0.1, qt=15, ny=10, nz=14)
    assert p.omega_nu < 1.77  # inside the linear stability range
    F, G = oracle.rest_state(p)
    F, G, mac = oracle.run(p, 300, F, G)
    cav = solver.Cavity(solver.make_params(nx=12, ny=10, nz=14, Ra=2e3, u0=0.1, precision=prec,
                                           thermal_q=15))
    cav.step(300)
    tol = 1e-12 if prec == "fp64" else 1e-5
    for fp64 in (True, False):
        m = cav.macros(fp64=fp64)
        for i, k in enumerate(("rho", "ux", "uy", "uz", "T")):
            sc = np.max(np.abs(mac[1:4])) if k.startswith("u") else np.max(np.abs(mac[i]))
            err = np.max(np.abs(to_np(m[k]).astype(np.float64) - mac[i])) / sc
            lim = tol if fp64 else max(tol, 1e-6)
            assert err <= lim, (k, fp64, err)
    cav.close()


@pytest.mark.parametrize("shape", [(14, 12, 10), (13, 11, 9)])
def test_centerlines_match_oracle(solver, oracle, shape):
    """Velocity profiles on the symmetry plane and their Table 1 peaks agree
    with the oracle's definitions (FP64)."""
    from oracle.oracle import centerline_profiles, table1_peaks
    nx, ny, nz = shape
    log(f"case: centerlines {shape} fp64")
    p = oracle.cavity_params(nx, 2e3, u0=0.1, ny=ny, nz=nz, omega_bulk=1.0, fourth_maxwell=1)
    F, G = oracle.rest_state(p)
    _, _, mac = oracle.run(p, 400, F, G)
    ul_ref, wl_ref = centerline_profiles(mac, 0.1)
    pk_ref = table1_peaks(mac, 0.1)
    cav = solver.Cavity(solver.make_params(nx=nx, ny=ny, nz=nz, Ra=2e3, u0=0.1,
                                           precision="fp64", omega_bulk=1.0, fourth_maxwell=1))
    cav.step(400)
    pk, ul, wl = cav.centerlines(profiles=True)
    sc = max(np.max(np.abs(ul_ref)), np.max(np.abs(wl_ref)))
    assert np.max(np.abs(to_np(ul) - ul_ref)) < 1e-12 * sc
    assert np.max(np.abs(to_np(wl) - wl_ref)) < 1e-12 * sc
    for k, v in pk_ref.items():
        assert abs(getattr(pk, k) - v) < 1e-10 * max(1.0, abs(v)), (k, getattr(pk, k), v)
    log("peaks", pk_ref)
    cav.close()


def test_run_to_steady_rules(solver):
    """Tolerance, plateau, stall and step-limit endings of lbm_run_to_steady."""
    from paper_1710_04751_amd import capi
    log("case: run_to_steady single cavity")
    mk = lambda prec: solver.Cavity(solver.make_params(12, 1e3, u0=0.1, precision=prec))
    cav = mk("fp64")
    steps, how, res = cav.run_to_steady(tol=1e-10, check_every=500, max_steps=200000)
    log("fp64 tol:", steps, how, res)
    assert how == capi.LBM_STEADY_TOL and res < 1e-10 and steps == cav.steps_done()
    assert steps % 500 == 0 and steps > 0
    # FP32 cannot reach 1e-15 (T is stored with 24-bit significands): the
    # residual stalls at the precision's floor and the plateau rule stops it
    c32 = mk("fp32")
    steps, how, res = c32.run_to_steady(tol=1e-15, check_every=500, max_steps=400000,
                                        plateau_checks=8, plateau_floor=1e-6)
    log("fp32 plateau:", steps, how, res)
    assert how in (capi.LBM_STEADY_PLATEAU, capi.LBM_STEADY_TOL)
    if how == capi.LBM_STEADY_PLATEAU:
        assert 0 < steps <= c32.steps_done() - 8 * 500 and res < 1e-6
    # with the floor below what FP32 reaches, the stall does not end the run
    c4 = mk("fp32")
    steps, how, res = c4.run_to_steady(tol=1e-15, check_every=500, max_steps=30000,
                                       plateau_checks=8, plateau_floor=1e-12)
    log("fp32 floor 1e-12:", steps, how, res)
    assert how in (capi.LBM_STEADY_MAX_STEPS, capi.LBM_STEADY_TOL)
    if how == capi.LBM_STEADY_MAX_STEPS:
        assert steps == -1 and c4.steps_done() == 30000
    c4.close()
    # the same floor with the stall rule: a residual that reaches no new
    # minimum for 8 checks above the floor ends the run as stalled (and only
    # once it wanders: the run first goes past the steps the FP32 plateau
    # needed above)
    c5 = mk("fp32")
    steps, how, res = c5.run_to_steady(tol=1e-15, check_every=500, max_steps=400000,
                                       plateau_checks=8, plateau_floor=1e-12, stall_checks=8)
    log("fp32 stall:", steps, how, res, c5.steps_done())
    assert how in (capi.LBM_STEADY_STALLED, capi.LBM_STEADY_TOL)
    if how == capi.LBM_STEADY_STALLED:
        assert steps == -1 and c5.steps_done() < 400000 and res > 1e-15
    c5.close()
    # a step limit below the convergence time
    c3 = mk("fp64")
    steps, how, res = c3.run_to_steady(tol=1e-12, check_every=100, max_steps=1000)
    assert how == capi.LBM_STEADY_MAX_STEPS and steps == -1 and c3.steps_done() == 1000
    for c in (cav, c32, c3):
        c.close()


@pytest.mark.parametrize("shape", [(12, 10, 8), (11, 9, 7)])
def test_symmetrize_matches_oracle(solver, oracle, shape):
    """In-place projection onto the cavity's symmetries (float32 fields)."""
    from paper_1710_04751_amd import workloads as W
    nx, ny, nz = shape
    f = [W.smooth_field((nz, ny, nx), s, a).astype(np.float32) for s, a in
         ((21, 0.02), (22, 0.02), (23, 0.02), (24, 0.5))]
    ref = oracle.cavity_symmetrize(*[a.astype(np.float64) for a in f])
    cav = solver.Cavity(solver.make_params(nx=nx, ny=ny, nz=nz, Ra=1e3))
    t = [torch.tensor(a).cuda() for a in f]
    cav.symmetrize(*t)
    for a, b in zip(t, ref):
        assert np.max(np.abs(to_np(a).astype(np.float64) - b)) <= 1e-7 * np.max(np.abs(b))
    cav.close()
