"""Steady differentially heated cavity, 64^3, Ra = 1e4, Pr = 0.71, u0 = 0.05:
D3Q7 and D3Q15 scalar lattices in FP64 and FP32, each run from rest until
max |T_n - T_(n-1000)| < 1e-8 (FP32: or the residual's plateau at its
precision floor).

Checks: energy balance (hot-wall and cold-wall Nu agree at steady state),
FP32 against FP64 on the same lattice, and the symmetry-plane quantities
against Table 1 of the paper (Sec. 3: 91^3 cascaded LBM with the D3Q15
scalar lattice, and the Navier-Stokes reference solution), within what the
coarser 64^3 grid allows."""
import json
import os

import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def solver():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_04751_amd import solver as S
    return S


@pytest.fixture(scope="module")
def table1():
    t = json.load(open(os.path.join(HERE, "golden", "table1_cavity.json")))
    i = t["Ra"].index(1e4)
    return {col: {k: v[i] for k, v in t[col].items() if isinstance(v, list) and k != "grid"}
            for col in ("lbm", "reference")}


@pytest.fixture(scope="module")
def steady(solver):
    """The four steady solutions: (qt, precision) -> observables."""
    from paper_1710_04751_amd import capi
    from paper_1710_04751_amd import workloads as W
    out = {}
    for qt in (7, 15):
        for prec in ("fp64", "fp32"):
            cav = solver.Cavity(solver.make_params(64, 1e4, precision=prec, thermal_q=qt))
            steps, how, res = cav.run_to_steady(max_steps=2_000_000, **W.STEADY_RULE)
            nu = cav.nusselt()
            pk = cav.centerlines()
            r = {"steps": steps, "how": how, "residual": res,
                 **{k: getattr(nu, k) for k in ("nu_hot_wall", "nu_cold_wall", "nu_hot_mid",
                                               "nu_cold_mid", "nu_max", "z_max", "nu_min",
                                               "z_min")},
                 **{k: getattr(pk, k) for k in ("u_max", "u_pos", "w_max", "w_pos")}}
            log(f"steady 64^3 Ra=1e4 q{qt} {prec}:", json.dumps(r))
            assert how in (capi.LBM_STEADY_TOL, capi.LBM_STEADY_PLATEAU), r
            if prec == "fp64":
                assert how == capi.LBM_STEADY_TOL, r
            out[(qt, prec)] = r
            cav.close()
    return out


@pytest.mark.parametrize("qt", [7, 15])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_energy_balance_at_steady_state(steady, qt, prec):
    r = steady[(qt, prec)]
    assert abs(r["nu_hot_wall"] - r["nu_cold_wall"]) < 1e-4 * r["nu_hot_wall"]
    assert abs(r["nu_hot_mid"] - r["nu_cold_mid"]) < 1e-3 * r["nu_hot_mid"]


@pytest.mark.parametrize("qt", [7, 15])
def test_fp32_matches_fp64_at_steady_state(steady, qt):
    """FP32 stops at its floor: the residual stalls near 3e-7 (a few units
    in the last place of T = 0.5) instead of reaching 1e-8, and the steady
    fields carry noise of that size.  Velocities (~0.01 in lattice units)
    therefore agree to ~3e-5 relative and the wall-averaged Nu to ~1e-5;
    the bars are 1e-4 and 2e-5."""
    a, b = steady[(qt, "fp32")], steady[(qt, "fp64")]
    assert a["residual"] < 1e-6
    for k, tol in (("nu_hot_wall", 2e-5), ("nu_hot_mid", 2e-5), ("u_max", 1e-4),
                   ("w_max", 1e-4)):
        assert abs(a[k] - b[k]) < tol * abs(b[k]), (k, a[k], b[k])
    for k in ("u_pos", "w_pos"):
        assert abs(a[k] - b[k]) < 1e-4, (k, a[k], b[k])


@pytest.mark.parametrize("qt", [7, 15])
def test_symmetry_plane_quantities_against_table1(steady, table1, qt):
    """Table 1 at Ra = 1e4: Nu_mean 2.2647 (LBM) / 2.302 (reference), u_max
    0.1965 / 0.2013, w_max 0.2232 / 0.2252 (units of u0).  The 64^3 grid
    (boundary layer of ~6 cells) is held to 3% outside the span of the two
    columns and positions to two cells.  The local extremes on the hot wall
    sit at or near the corners, where 64 against 91 cells matters most: 8%.
    With the D3Q15 scalar lattice the first and last layers along z carry
    diagonal links that also cross the adiabatic faces, so the link-flux
    local Nu of the corner cells is not the wall gradient the paper
    tabulates; its extremes are checked on D3Q7 only."""
    r = steady[(qt, "fp64")]
    checks = [("nu_hot_mid", "Nu_mean", 0.03), ("u_max", "u_max", 0.03),
              ("w_max", "w_max", 0.03)]
    if qt == 7:
        checks += [("nu_max", "Nu_max", 0.08), ("nu_min", "Nu_min", 0.08)]
    for ours, key, tol in checks:
        lo = min(table1["lbm"][key], table1["reference"][key]) * (1 - tol)
        hi = max(table1["lbm"][key], table1["reference"][key]) * (1 + tol)
        assert lo <= r[ours] <= hi, (ours, r[ours], lo, hi)
    pos = [("u_pos", "u_max_pos"), ("w_pos", "w_max_pos")]
    if qt == 7:
        pos.append(("z_max", "Nu_max_pos"))
        assert r["z_min"] > 0.95  # the minimum sits at the top corner
    for ours, key in pos:
        ref = 0.5 * (table1["lbm"][key] + table1["reference"][key])
        assert abs(r[ours] - ref) < 2.0 / 64 + 0.01, (ours, r[ours], ref)
