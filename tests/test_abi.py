"""The C-ABI library loads, exports every symbol include/lbm.h declares, and
validates parameters on the host (no device work, runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("lbm.h", "lbm_nn.h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def capi():
    from paper_1710_04751_amd import capi as C
    if not os.path.exists(C.LIB_PATH):
        pytest.fail("liblbm.so is not built (run __graft_entry__.build())")
    C.lib()
    return C


def test_every_declared_function_is_exported(capi):
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(capi.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding covers them under the same names
    assert sorted(capi.exported_names()) == names


def test_params_defaults_and_lattice_mapping(capi):
    p = capi.lbm_params_init(16, 1e3)
    assert (p.nx, p.ny, p.nz, p.thermal_q, p.precision) == (16, 16, 16, 7, capi.LBM_FP32)
    L = capi.lbm_params_lattice(p)
    # Ra = g beta dT L^3/(nu alpha), Pr = nu/alpha, u0^2 = g beta dT L
    Lx, dT = 16.0, 1.0
    assert abs(L.gbeta * dT * Lx ** 3 / (L.nu * L.alpha) - 1e3) < 1e-9
    assert abs(L.nu / L.alpha - 0.71) < 1e-14
    assert abs(L.gbeta * dT * Lx - 0.05 ** 2) < 1e-15
    assert abs((1 / L.omega_nu - 0.5) / 3 - L.nu) < 1e-15
    assert abs((1 / L.omega_T - 0.5) / 3 - L.alpha) < 1e-15
    assert L.omega_bulk == L.omega_nu and L.T_ref == 0.0


@pytest.mark.parametrize("field,value,msg", [
    ("nx", 3, ">= 4"), ("thermal_q", 9, "7 or 15"), ("R", float("inf"), "source"),
    ("u0", 0.2, "0.3"), ("omega_hi", 2.0, "(0, 2)"), ("precision", 7, "precision"),
    ("block_x", 48, "multiple of 64"), ("Pr", -1.0, "positive"),
    ("round_stochastic", 1, "round_stochastic"), ("scalar_specular", 2, "scalar_specular"),
])
def test_invalid_parameters_are_rejected(capi, field, value, msg):
    p = capi.lbm_params_init(16, 1e3)
    setattr(p, field, value)
    if field == "block_x":
        p.block_y = 1
    assert capi.lib().lbm_workspace_bytes(ctypes.byref(p)) == 0
    assert msg in capi.lbm_last_error()
    with pytest.raises(capi.LbmError) as e:
        capi.lbm_create(p, 0x1000, 1 << 30)
    assert e.value.status == capi.LBM_ERR_ARG


def test_grid_size_limits(capi):
    # 32-bit cell indices: 1291^3 > 2^31 cells is refused
    p = capi.lbm_params_init(1291, 1e6)
    assert capi.lib().lbm_workspace_bytes(ctypes.byref(p)) == 0
    assert "too large" in capi.lbm_last_error()
    # the step kernel's window of 3 ny + 2 rows must fit 32-bit byte offsets
    p = capi.lbm_params_init(16, 1e3)
    p.nx, p.ny, p.nz = 8192, 8192, 4
    p.precision = capi.LBM_FP64
    assert capi.lib().lbm_workspace_bytes(ctypes.byref(p)) == 0
    assert "too large" in capi.lbm_last_error()
    # 1024^3 in FP32 (two states of 22 populations: 189 GB) fits one MI355X
    p = capi.lbm_params_init(1024, 1e6)
    n = capi.lbm_workspace_bytes(p)
    assert n >= 2 * 22 * 4 * 1024 ** 3


def test_workspace_checks_before_any_device_work(capi):
    p = capi.lbm_params_init(16, 1e3)
    nbytes = capi.lbm_workspace_bytes(p)
    # two states of (15 + 7) populations, FP32, padded rows
    assert nbytes >= 2 * 22 * 16 ** 3 * 4
    with pytest.raises(capi.LbmError) as e:
        capi.lbm_create(p, None, nbytes)
    assert e.value.status == capi.LBM_ERR_ARG
    with pytest.raises(capi.LbmError):
        capi.lbm_create(p, 0x1000, nbytes - 1)
    with pytest.raises(capi.LbmError):
        capi.lbm_create(p, 0x1001, nbytes)  # misaligned
    with pytest.raises(capi.LbmError):
        capi.lbm_copy_probe(0x1000, 0x2000, 17)


def test_batch_validation_on_host(capi):
    a = capi.lbm_params_init(32, 1e4)
    b = capi.lbm_params_init(48, 1e5)
    n2 = capi.lbm_batch_workspace_bytes([a, b])
    assert n2 >= capi.lbm_workspace_bytes(a) + capi.lbm_workspace_bytes(b)
    b.precision = capi.LBM_FP64
    with pytest.raises(capi.LbmError, match="share precision"):
        capi.lbm_batch_workspace_bytes([a, b])
    b.precision = a.precision
    b.nx = 3
    with pytest.raises(capi.LbmError, match="member 1"):
        capi.lbm_batch_workspace_bytes([a, b])
    with pytest.raises(capi.LbmError, match="1 to 255"):
        capi.lbm_batch_workspace_bytes([a] * 256)


def test_network_parameter_count_and_config_checks(capi):
    from oracle import nn_oracle
    assert capi.lbm_nn_param_count() == nn_oracle.param_count()
    c = capi.nn_config(64, 8)
    assert capi.lbm_nn_workspace_bytes(c) > 4 * 4 * nn_oracle.param_count()
    for bad in (capi.nn_config(48, 8), capi.nn_config(64, 0), capi.nn_config(64, 65),
                capi.nn_config(4, 1), capi.nn_config(64, 8, lr=-1.0)):
        with pytest.raises(capi.LbmError):
            capi.lbm_nn_workspace_bytes(bad)
    with pytest.raises(capi.LbmError):
        capi.lbm_nn_create(c, 0x1000, 16)


def test_batch_members_must_share_the_kernel_variant(capi):
    """A batch is one kernel: members differing in precision, scalar lattice,
    rounding mode or collision path are refused on the host."""
    def member(**kw):
        p = capi.lbm_params_init(16, 1e3)
        for k, v in kw.items():
            setattr(p, k, v)
        return p
    base = dict(precision=capi.LBM_FP32_S16, round_stochastic=1)
    assert capi.lbm_batch_workspace_bytes([member(**base), member(**base)]) > 0
    for other, msg in ((dict(precision=capi.LBM_FP32_S16), "rounding"),
                       (dict(base, thermal_q=15), "thermal_q"),
                       (dict(base, omega_hi=1.2), "collision path")):
        arr = (capi.lbm_params * 2)(member(**base), member(**other))
        assert capi.lib().lbm_batch_workspace_bytes(arr, 2) == 0
        assert msg in capi.lbm_last_error()
