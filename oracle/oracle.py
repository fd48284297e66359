"""ctypes wrapper of the plain CPU oracle (lbm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py.  The GPU library never imports this module.

All arrays are float64 numpy arrays.  State layout: F[15][nz][ny][nx] and
G[qt][nz][ny][nx] (post-collision populations), as in the oracle's C code.
"""
import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_LIBS = {}


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("qt", ctypes.c_int32), ("periodic", ctypes.c_int32), ("specular", ctypes.c_int32),
        ("omega_nu", ctypes.c_double), ("omega_bulk", ctypes.c_double),
        ("omega_hi", ctypes.c_double),
        ("omega_T", ctypes.c_double), ("omega_hiT", ctypes.c_double),
        ("cs2T", ctypes.c_double), ("gbeta", ctypes.c_double),
        ("T_hot", ctypes.c_double), ("T_cold", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("fourth_maxwell", ctypes.c_int32), ("pad2_", ctypes.c_int32),
        ("R", ctypes.c_double),
    ]


@dataclass
class Params:
    """Lattice-unit description of one oracle run."""
    nx: int
    ny: int
    nz: int
    qt: int = 7
    omega_nu: float = 1.0
    omega_bulk: float = 0.0  # <= 0: same as omega_nu
    omega_hi: float = 1.0
    omega_T: float = 1.0
    omega_hiT: float = 1.0
    cs2T: float = 1.0 / 3.0
    gbeta: float = 0.0
    T_hot: float = 0.5
    T_cold: float = -0.5
    T_ref: float = 0.0
    periodic: int = 0  # bit 0/1/2: periodic in x/y/z instead of walls
    fourth_maxwell: int = 0  # 4th-order flow equilibrium: 0 kxx~kyy~/rho, 1 rho/9
    R: float = 0.0  # uniform scalar source per cell and step
    specular: int = 0  # scalar on the adiabatic faces: 0 bounce-back, 1 specular reflection
    alpha: float = float("nan")  # thermal diffusivity, for the Nusselt number
    nu: float = float("nan")

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    def c_struct(self) -> _Params:
        return _Params(self.nx, self.ny, self.nz, self.qt, self.periodic, self.specular,
                       self.omega_nu, self.omega_bulk, self.omega_hi, self.omega_T,
                       self.omega_hiT, self.cs2T, self.gbeta, self.T_hot, self.T_cold,
                       self.T_ref, self.fourth_maxwell, 0, self.R)


def cavity_params(n, Ra, Pr=0.71, u0=0.05, qt=7, cs2T=1.0 / 3.0, ny=None, nz=None,
                  T_hot=0.5, T_cold=-0.5, omega_hi=1.0, omega_hiT=1.0, omega_bulk=0.0,
                  fourth_maxwell=0, R=0.0, specular=0) -> Params:
    """Map (Ra, Pr, u0, L = n) to lattice parameters.

    Reading (the paper gives Ra = g beta dT L^3 / (alpha nu) and Pr = nu/alpha,
    Sec. 3, but no lattice mapping): the velocity scale sqrt(g beta dT L) is
    fixed at u0, so g beta = u0^2 / (dT L), nu = u0 L sqrt(Pr / Ra),
    alpha = nu / Pr.  Relaxation rates: nu = c_s^2 (1/omega - 1/2) with
    c_s^2 = 1/3 (Appendix A) and alpha = c_sphi^2 (1/omega_T - 1/2) (eq. 23).
    T0 = (T_hot + T_cold)/2 (Sec. 3).
    """
    L = float(n)
    dT = T_hot - T_cold
    gbeta = u0 * u0 / (dT * L)
    nu = u0 * L * math.sqrt(Pr / Ra)
    alpha = nu / Pr
    return Params(nx=n, ny=ny or n, nz=nz or n, qt=qt,
                  omega_nu=1.0 / (3.0 * nu + 0.5), omega_bulk=omega_bulk, omega_hi=omega_hi,
                  fourth_maxwell=fourth_maxwell,
                  omega_T=1.0 / (alpha / cs2T + 0.5), omega_hiT=omega_hiT,
                  cs2T=cs2T, gbeta=gbeta, T_hot=T_hot, T_cold=T_cold,
                  T_ref=0.5 * (T_hot + T_cold), R=R, alpha=alpha, nu=nu, specular=specular)


def _lib(long_double=False):
    key = bool(long_double)
    if key in _LIBS:
        return _LIBS[key]
    path = _build.LIB_LD if long_double else _build.LIB
    if not os.path.exists(path):
        _build.build(force=False)
    lib = ctypes.CDLL(path)
    pre = "oracle_ld_" if long_double else "oracle_"
    dp = ctypes.POINTER(ctypes.c_double)
    fns = {}
    def f(name, res, args):
        fn = getattr(lib, pre + name)
        fn.restype = res
        fn.argtypes = args
        fns[name] = fn
    P = ctypes.POINTER(_Params)
    f("set_threads", ctypes.c_int, [ctypes.c_int])
    f("real_bytes", ctypes.c_int, [])
    f("collide_flow", None, [dp, dp, dp, ctypes.c_int, dp, dp])
    f("collide_thermal", None, [ctypes.c_int, dp, dp, ctypes.c_double, dp, ctypes.c_double, dp])
    f("scalar_source", None, [ctypes.c_int, ctypes.c_double, dp, dp])
    f("equilibrium", None, [ctypes.c_int, ctypes.c_double, dp, ctypes.c_double,
                            ctypes.c_double, dp, dp])
    f("run", ctypes.c_int, [P, ctypes.c_int64, dp, dp, dp])
    f("step_cells", None, [P, ctypes.c_int64, dp, ctypes.POINTER(ctypes.c_int32), dp, dp, dp])
    f("init_equilibrium", None, [P, dp, dp, dp, dp, dp, dp, dp])
    f("nusselt", None, [P, dp, ctypes.c_double, dp, dp])
    _LIBS[key] = fns
    return fns


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(n=0, long_double=False) -> int:
    """Set (n > 0) or query the OpenMP thread count; returns the count used."""
    return _lib(long_double)["set_threads"](int(n))


def collide_flow(fbar, F, omega, fourth_maxwell=0, long_double=False):
    """Flow collision of one cell: returns (post-collision f, rho, u)."""
    fb = np.ascontiguousarray(fbar, dtype=np.float64)
    Fr = np.ascontiguousarray(F, dtype=np.float64)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    out = np.empty(15)
    ru = np.empty(4)
    _lib(long_double)["collide_flow"](_ptr(fb), _ptr(Fr), _ptr(om), int(fourth_maxwell),
                                      _ptr(out), _ptr(ru))
    return out, ru[0], ru[1:].copy()


def collide_thermal(qt, gbar, u, cs2, omega, R=0.0, long_double=False):
    """Thermal collision of one cell with a local source R (gbar is the
    transformed distribution g - S/2 of eq. (13))."""
    g = np.ascontiguousarray(gbar, dtype=np.float64)
    ur = np.ascontiguousarray(u, dtype=np.float64)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    out = np.empty(qt)
    _lib(long_double)["collide_thermal"](qt, _ptr(g), _ptr(ur), float(cs2), _ptr(om), float(R),
                                         _ptr(out))
    return out


def scalar_source(qt, R, u):
    """Source populations S^phi of a cell with source R and velocity u."""
    ur = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty(qt)
    _lib()["scalar_source"](qt, float(R), _ptr(ur), _ptr(out))
    return out


def equilibrium(qt, rho, u, phi, cs2=1.0 / 3.0):
    """(feq[15], geq[qt]) at (rho, u) and (phi, u)."""
    ur = np.ascontiguousarray(u, dtype=np.float64)
    feq = np.empty(15)
    geq = np.empty(qt)
    _lib()["equilibrium"](qt, float(rho), _ptr(ur), float(phi), float(cs2), _ptr(feq), _ptr(geq))
    return feq, geq


def rest_state(p: Params):
    """Fluid at rest with rho = 1 and T = 0 (F = w, G = 0)."""
    return init_equilibrium(p, T=np.zeros((p.nz, p.ny, p.nx)))


def init_equilibrium(p: Params, rho=None, ux=None, uy=None, uz=None, T=None):
    """Equilibrium populations from macroscopic fields ([nz][ny][nx])."""
    def arr(a):
        return None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    F = np.empty((15, p.nz, p.ny, p.nx))
    G = np.empty((p.qt, p.nz, p.ny, p.nx))
    cp = p.c_struct()
    _lib()["init_equilibrium"](ctypes.byref(cp), _ptr(arr(rho)), _ptr(arr(ux)), _ptr(arr(uy)),
                               _ptr(arr(uz)), _ptr(arr(T)), _ptr(F), _ptr(G))
    return F, G


def run(p: Params, nsteps, F, G, long_double=False):
    """Advance nsteps from the post-collision state (F, G).

    Returns (F, G, mac) where mac[5][nz][ny][nx] = rho, ux, uy, uz, T of the
    last step (pre-collision moments)."""
    F = np.array(F, dtype=np.float64, order="C", copy=True)
    G = np.array(G, dtype=np.float64, order="C", copy=True)
    assert F.shape == (15, p.nz, p.ny, p.nx) and G.shape == (p.qt, p.nz, p.ny, p.nx)
    mac = np.full((5, p.nz, p.ny, p.nx), np.nan)
    cp = p.c_struct()
    rc = _lib(long_double)["run"](ctypes.byref(cp), int(nsteps), _ptr(F), _ptr(G), _ptr(mac))
    if rc != 0:
        raise RuntimeError(f"oracle run failed ({rc})")
    return F, G, mac


def step_cells(p: Params, nb, pos, long_double=False):
    """One update of selected cells from their 3x3x3 neighbourhoods.

    nb: [n][27][15+qt] previous post-collision populations, index
    (dz+1)*9+(dy+1)*3+(dx+1); pos: [n][3] int (x, y, z).
    Returns (fout [n][15], gout [n][qt], mac [n][5])."""
    nb = np.ascontiguousarray(nb, dtype=np.float64)
    pos = np.ascontiguousarray(pos, dtype=np.int32)
    n = pos.shape[0]
    assert nb.shape == (n, 27, 15 + p.qt)
    fout = np.empty((n, 15))
    gout = np.empty((n, p.qt))
    mac = np.empty((n, 5))
    cp = p.c_struct()
    _lib(long_double)["step_cells"](ctypes.byref(cp), n, _ptr(nb),
                                    pos.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    _ptr(fout), _ptr(gout), _ptr(mac))
    return fout, gout, mac


def nusselt(p: Params, G, alpha=None):
    """Local Nusselt numbers (hot, cold) [nz][ny] from the stored state G."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    a = p.alpha if alpha is None else alpha
    nh = np.empty((p.nz, p.ny))
    nc = np.empty((p.nz, p.ny))
    cp = p.c_struct()
    _lib()["nusselt"](ctypes.byref(cp), _ptr(G), float(a), _ptr(nh), _ptr(nc))
    return nh, nc


def midline_profile(local_nu):
    """Local Nu along z on the mid-plane y = L/2 (mean of the two middle rows
    for even ny)."""
    ny = local_nu.shape[1]
    if ny % 2:
        return local_nu[:, ny // 2].copy()
    return 0.5 * (local_nu[:, ny // 2 - 1] + local_nu[:, ny // 2])


def _middle(n):
    """Indices of the cells across the centre of n cells: one for odd n, the
    two middle ones for even n."""
    return list(range((n - 1) // 2, n // 2 + 1))


def centerline_profiles(mac, u0):
    """Velocity profiles on the symmetry plane y = L/2 (Table 1 quantities),
    in units of u0, from the macroscopic fields mac[5][nz][ny][nx]:
    u_line[z] = -u_x on the vertical centreline x = L/2 (the velocity along
    the heated axis pointing from the cold to the hot wall), and
    w_line[x] = u_z on the horizontal centreline z = L/2."""
    _, nz, ny, nx = mac.shape
    ys, xs, zs = _middle(ny), _middle(nx), _middle(nz)
    u_line = np.array([-np.mean([mac[1, z, y, x] for y in ys for x in xs]) for z in range(nz)])
    w_line = np.array([np.mean([mac[3, z, y, x] for z in zs for y in ys]) for x in range(nx)])
    return u_line / u0, w_line / u0


def parabola_peak(v):
    """Maximum of samples v[i] taken at (i + 1/2)/n, refined by the parabola
    through the largest sample and its two neighbours; (value, position)."""
    n = len(v)
    k = int(np.argmax(v))
    if 0 < k < n - 1:
        a, b, c = v[k - 1], v[k], v[k + 1]
        curv = a - 2 * b + c
        if curv < 0:
            off = 0.5 * (a - c) / curv
            return b - 0.25 * (a - c) * off, (k + 0.5 + off) / n
    return float(v[k]), (k + 0.5) / n


def table1_peaks(mac, u0):
    """u_max with its height z/L, and w_max with its distance from the cold
    wall over L (the paper's heated axis runs from the cold to the hot wall),
    each from centerline_profiles."""
    u_line, w_line = centerline_profiles(mac, u0)
    u_max, u_pos = parabola_peak(u_line)
    w_max, w_pos = parabola_peak(w_line[::-1])
    return {"u_max": u_max, "u_pos": u_pos, "w_max": w_max, "w_pos": w_pos}


def staggered_momentum(F):
    """Staggered momentum sums (sum (-1)^x j_x, sum (-1)^y j_y,
    sum (-1)^z j_z) of a stored state F[15][nz][ny][nx], with j the raw
    first moment of the populations."""
    _, nz, ny, nx = F.shape
    ex = np.array([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1])
    ey = np.array([0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1])
    ez = np.array([0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1])
    jx = np.tensordot(ex, F, axes=1)
    jy = np.tensordot(ey, F, axes=1)
    jz = np.tensordot(ez, F, axes=1)
    sx = (-1.0) ** np.arange(nx)
    sy = (-1.0) ** np.arange(ny)
    sz = (-1.0) ** np.arange(nz)
    return (float(np.sum(jx * sx[None, None, :])), float(np.sum(jy * sy[None, :, None])),
            float(np.sum(jz * sz[:, None, None])))


def staggered_free(ux, uy, uz, T=None, gbeta=0.0, T_ref=0.0):
    """Velocity fields [nz][ny][nx] with the staggered momentum of a start
    from rest: sum (-1)^x u_x = sum (-1)^y u_y = 0 and sum (-1)^z u_z =
    S/2 with S = g beta sum (-1)^z (T - T_ref), reached by adding uniform
    (-1)^x, (-1)^y, (-1)^z patterns (with rho = 1 the momentum is the
    velocity)."""
    out = []
    for a, axis in ((ux, 2), (uy, 1), (uz, 0)):
        a = np.asarray(a, dtype=np.float64)
        shape = [1, 1, 1]
        shape[axis] = a.shape[axis]
        s = ((-1.0) ** np.arange(a.shape[axis])).reshape(shape)
        target = 0.0
        if axis == 0 and T is not None:
            target = 0.5 * gbeta * np.sum((np.asarray(T, dtype=np.float64) - T_ref) * s)
        out.append(a - s * (np.sum(a * s) - target) / a.size)
    return out


def cavity_symmetrize(ux, uy, uz, T, T0=0.0):
    """Signed mean of fields [nz][ny][nx] over the cavity's symmetry group:
    identity, the mirror y -> ny-1-y (uy changes sign), the half turn
    (x, z) -> (nx-1-x, nz-1-z) (ux, uz, T - T0 change sign) and their
    product."""
    mir = lambda a: a[:, ::-1, :]
    rot = lambda a: a[::-1, :, ::-1]
    f = lambda a, sm, sr: 0.25 * (a + sm * mir(a) + sr * rot(a) + sm * sr * mir(rot(a)))
    t = np.asarray(T, dtype=np.float64) - T0
    return (f(np.asarray(ux, dtype=np.float64), 1, -1), f(np.asarray(uy, dtype=np.float64), -1, 1),
            f(np.asarray(uz, dtype=np.float64), 1, -1), T0 + f(t, 1, -1))
