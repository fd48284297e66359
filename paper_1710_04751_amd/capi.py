"""ctypes binding of liblbm.so: the C ABI of include/lbm.h under the same
names.  Argument marshalling only; every step of the method runs in the
library's HIP kernels.  Device pointers are passed as Python ints (for
example torch_tensor.data_ptr()); NULL is 0 or None.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_ERR_ARG, LBM_ERR_HIP, LBM_ERR_UNSTABLE, LBM_ERR_STATE = 0, -1, -2, -3, -4
LBM_FP64, LBM_FP32, LBM_FP32_S16 = 0, 1, 2


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("thermal_q", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("fourth_maxwell", ctypes.c_int32),
        ("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("u0", ctypes.c_double),
        ("T_hot", ctypes.c_double), ("T_cold", ctypes.c_double), ("cs2_T", ctypes.c_double),
        ("omega_bulk", ctypes.c_double), ("omega_hi", ctypes.c_double),
        ("omega_hi_T", ctypes.c_double), ("R", ctypes.c_double),
        ("lattice_units", ctypes.c_int32), ("block_x", ctypes.c_int32),
        ("block_y", ctypes.c_int32), ("round_stochastic", ctypes.c_int32),
        ("scalar_specular", ctypes.c_int32),
        ("nu", ctypes.c_double), ("alpha", ctypes.c_double), ("gbeta", ctypes.c_double),
    ]


class lbm_lattice(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("nu", "alpha", "gbeta", "omega_nu", "omega_bulk", "omega_T", "T_ref")]


class lbm_nu(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("nu_hot_wall", "nu_cold_wall", "nu_hot_mid", "nu_cold_mid",
                 "nu_max", "z_max", "nu_min", "z_min")]


class lbm_peaks(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("u_max", "u_pos", "w_max", "w_pos")]


LBM_STEADY_TOL, LBM_STEADY_PLATEAU, LBM_STEADY_MAX_STEPS, LBM_STEADY_UNSTABLE = 0, 1, 2, 3
LBM_STEADY_STALLED = 4


class lbm_nn_config(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("target_scale", ctypes.c_float * 4)]


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lbm status {status}: {msg}")
        self.status = status


_lib = None
vp = ctypes.c_void_p
H = ctypes.c_void_p  # lbm_handle*

# name -> (restype, argtypes); mirrors include/lbm.h
_SIGS = {
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_params_init": (ctypes.c_int, [ctypes.POINTER(lbm_params), ctypes.c_int32, ctypes.c_double]),
    "lbm_params_lattice": (ctypes.c_int, [ctypes.POINTER(lbm_params), ctypes.POINTER(lbm_lattice)]),
    "lbm_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(lbm_params)]),
    "lbm_create": (ctypes.c_int, [ctypes.POINTER(lbm_params), vp, ctypes.c_size_t, vp,
                                  ctypes.POINTER(H)]),
    "lbm_destroy": (ctypes.c_int, [H]),
    "lbm_get_lattice": (ctypes.c_int, [H, ctypes.POINTER(lbm_lattice)]),
    "lbm_steps_done": (ctypes.c_int64, [H]),
    "lbm_init_rest": (ctypes.c_int, [H]),
    "lbm_init_macros": (ctypes.c_int, [H, vp, vp, vp, vp]),
    "lbm_step": (ctypes.c_int, [H, ctypes.c_int64]),
    "lbm_macros": (ctypes.c_int, [H, vp, vp, vp, vp, vp, ctypes.c_int]),
    "lbm_nusselt": (ctypes.c_int, [H, ctypes.POINTER(lbm_nu), vp, vp]),
    "lbm_nusselt_noalloc": (ctypes.c_int, [H, ctypes.POINTER(lbm_nu), vp, vp]),
    "lbm_residual": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_double)]),
    "lbm_centerlines": (ctypes.c_int, [H, vp, vp, ctypes.POINTER(lbm_peaks)]),
    "lbm_symmetrize": (ctypes.c_int, [H, vp, vp, vp, vp]),
    "lbm_run_to_steady": (ctypes.c_int, [H, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_double)]),
    "lbm_get_populations": (ctypes.c_int, [H, vp, vp]),
    "lbm_set_populations": (ctypes.c_int, [H, vp, vp]),
    "lbm_gather_cells": (ctypes.c_int, [H, vp, ctypes.c_int64, vp, vp, ctypes.c_int]),
    "lbm_state_info": (ctypes.c_int, [H, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int32)]),
    "lbm_step_kernel_name": (ctypes.c_char_p, [H]),
    "lbm_set_block": (ctypes.c_int, [H, ctypes.c_int32, ctypes.c_int32]),
    "lbm_autotune": (ctypes.c_int, [H, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]),
    "lbm_copy_probe": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp]),
    "lbm_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(lbm_params), ctypes.c_int32]),
    "lbm_batch_create": (ctypes.c_int, [ctypes.POINTER(lbm_params), ctypes.c_int32, vp,
                                        ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
    "lbm_batch_destroy": (ctypes.c_int, [vp]),
    "lbm_batch_member": (vp, [vp, ctypes.c_int32]),
    "lbm_batch_step": (ctypes.c_int, [vp, ctypes.c_int64]),
    "lbm_batch_residuals": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int32)]),
    "lbm_batch_set_active": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int32)]),
    "lbm_batch_run_to_steady": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_int64,
                                               ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                               ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(ctypes.c_int32),
                                               ctypes.POINTER(ctypes.c_double)]),
    "lbm_batch_set_launch": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "lbm_batch_autotune": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32)]),
    "lbm_batch_launch_info": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_int64)]),
    # include/lbm_nn.h
    "lbm_nn_param_count": (ctypes.c_int64, []),
    "lbm_nn_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(lbm_nn_config)]),
    "lbm_nn_create": (ctypes.c_int, [ctypes.POINTER(lbm_nn_config), vp, ctypes.c_size_t, vp,
                                     ctypes.POINTER(vp)]),
    "lbm_nn_destroy": (ctypes.c_int, [vp]),
    "lbm_nn_set_params": (ctypes.c_int, [vp, vp]),
    "lbm_nn_get_params": (ctypes.c_int, [vp, vp]),
    "lbm_nn_forward": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_float), vp,
                                      ctypes.POINTER(ctypes.c_float)]),
    "lbm_nn_gradient": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_float), vp,
                                       ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.c_int64, vp, ctypes.POINTER(ctypes.c_double)]),
    "lbm_nn_train_step": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_float), vp,
                                         ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    "lbm_nn_set_lr": (ctypes.c_int, [vp, ctypes.c_float]),
    "lbm_nn_activation": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32, vp]),
    "lbm_nn_flops": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]),
}


def lib():
    """The loaded liblbm.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return list(_SIGS)


def check(status):
    if status != LBM_OK:
        raise LbmError(status, lbm_last_error())
    return status


def lbm_last_error():
    return lib().lbm_last_error().decode()


def lbm_params_init(n, Ra):
    p = lbm_params()
    check(lib().lbm_params_init(ctypes.byref(p), int(n), float(Ra)))
    return p


def lbm_params_lattice(p):
    L = lbm_lattice()
    check(lib().lbm_params_lattice(ctypes.byref(p), ctypes.byref(L)))
    return L


def lbm_workspace_bytes(p):
    n = lib().lbm_workspace_bytes(ctypes.byref(p))
    if n == 0:
        raise LbmError(LBM_ERR_ARG, lbm_last_error())
    return n


def lbm_create(p, workspace_ptr, workspace_bytes, stream_ptr=None):
    h = H()
    check(lib().lbm_create(ctypes.byref(p), workspace_ptr, workspace_bytes, stream_ptr or None,
                           ctypes.byref(h)))
    return h


def lbm_destroy(h):
    return check(lib().lbm_destroy(h))


def lbm_get_lattice(h):
    L = lbm_lattice()
    check(lib().lbm_get_lattice(h, ctypes.byref(L)))
    return L


def lbm_steps_done(h):
    return lib().lbm_steps_done(h)


def lbm_init_rest(h):
    return check(lib().lbm_init_rest(h))


def lbm_init_macros(h, ux=None, uy=None, uz=None, T=None):
    return check(lib().lbm_init_macros(h, ux, uy, uz, T))


def lbm_step(h, nsteps):
    return check(lib().lbm_step(h, int(nsteps)))


def lbm_macros(h, rho=None, ux=None, uy=None, uz=None, T=None, fp64=False):
    return check(lib().lbm_macros(h, rho, ux, uy, uz, T, 1 if fp64 else 0))


def lbm_nusselt(h, local_hot=None, local_cold=None):
    out = lbm_nu()
    check(lib().lbm_nusselt(h, ctypes.byref(out), local_hot, local_cold))
    return out


def lbm_nusselt_noalloc(h, local_hot=None, local_cold=None):
    out = lbm_nu()
    check(lib().lbm_nusselt_noalloc(h, ctypes.byref(out), local_hot, local_cold))
    return out


def lbm_residual(h):
    """Returns (status, max_dT); status LBM_ERR_UNSTABLE is returned, not raised."""
    v = ctypes.c_double()
    s = lib().lbm_residual(h, ctypes.byref(v))
    if s not in (LBM_OK, LBM_ERR_UNSTABLE):
        check(s)
    return s, v.value


def lbm_centerlines(h, u_line=None, w_line=None, peaks=True):
    """Returns an lbm_peaks (synchronising) when peaks is true, else None."""
    pk = lbm_peaks() if peaks else None
    check(lib().lbm_centerlines(h, u_line, w_line, ctypes.byref(pk) if peaks else None))
    return pk


def lbm_symmetrize(h, ux=None, uy=None, uz=None, T=None):
    return check(lib().lbm_symmetrize(h, ux, uy, uz, T))


def lbm_run_to_steady(h, tol, check_every, max_steps, plateau_checks=0, plateau_floor=0.0,
                      stall_checks=0):
    """Returns (steps, how, last residual); how is an LBM_STEADY_* value.  An
    unstable run raises LbmError(LBM_ERR_UNSTABLE)."""
    steps, how, res = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_double()
    check(lib().lbm_run_to_steady(h, float(tol), int(check_every), int(max_steps),
                                  int(plateau_checks), float(plateau_floor), int(stall_checks),
                                  ctypes.byref(steps),
                                  ctypes.byref(how),
                                  ctypes.byref(res)))
    return steps.value, how.value, res.value


def lbm_get_populations(h, F=None, G=None):
    return check(lib().lbm_get_populations(h, F, G))


def lbm_set_populations(h, F, G):
    return check(lib().lbm_set_populations(h, F, G))


def lbm_gather_cells(h, cells, n, F=None, G=None, check_range=True):
    return check(lib().lbm_gather_cells(h, cells, int(n), F, G, 1 if check_range else 0))


def lbm_state_info(h):
    F, G, ps, vb = vp(), vp(), ctypes.c_int64(), ctypes.c_int32()
    check(lib().lbm_state_info(h, ctypes.byref(F), ctypes.byref(G), ctypes.byref(ps),
                               ctypes.byref(vb)))
    return F.value, G.value, ps.value, vb.value


def lbm_step_kernel_name(h):
    return lib().lbm_step_kernel_name(h).decode()


def lbm_set_block(h, bx, by):
    return check(lib().lbm_set_block(h, int(bx), int(by)))


def lbm_autotune(h, steps_per_trial):
    bx, by = ctypes.c_int32(), ctypes.c_int32()
    check(lib().lbm_autotune(h, int(steps_per_trial), ctypes.byref(bx), ctypes.byref(by)))
    return bx.value, by.value


def lbm_copy_probe(dst, src, nbytes, stream_ptr=None):
    return check(lib().lbm_copy_probe(dst, src, int(nbytes), stream_ptr or None))


# -- batched form ----------------------------------------------------------

def _params_array(params):
    arr = (lbm_params * len(params))(*params)
    return arr


def lbm_batch_workspace_bytes(params):
    n = lib().lbm_batch_workspace_bytes(_params_array(params), len(params))
    if n == 0:
        raise LbmError(LBM_ERR_ARG, lbm_last_error())
    return n


def lbm_batch_create(params, workspace_ptr, workspace_bytes, stream_ptr=None):
    b = vp()
    check(lib().lbm_batch_create(_params_array(params), len(params), workspace_ptr,
                                 workspace_bytes, stream_ptr or None, ctypes.byref(b)))
    return b


def lbm_batch_destroy(b):
    return check(lib().lbm_batch_destroy(b))


def lbm_batch_member(b, i):
    h = lib().lbm_batch_member(b, int(i))
    if not h:
        raise LbmError(LBM_ERR_ARG, "member index out of range")
    return vp(h)


def lbm_batch_step(b, nsteps):
    return check(lib().lbm_batch_step(b, int(nsteps)))


def lbm_batch_residuals(b, n):
    r = (ctypes.c_double * n)()
    st = (ctypes.c_int32 * n)()
    check(lib().lbm_batch_residuals(b, r, st))
    return list(r), list(st)


def lbm_batch_set_active(b, active):
    a = (ctypes.c_int32 * len(active))(*[1 if v else 0 for v in active])
    return check(lib().lbm_batch_set_active(b, a))


def lbm_batch_run_to_steady(b, n, tol, check_every, max_steps, plateau_checks=0,
                            plateau_floor=0.0, stall_checks=0):
    """Returns (steps, how, last residual) per member; how is an LBM_STEADY_* value."""
    steps = (ctypes.c_int64 * n)()
    st = (ctypes.c_int32 * n)()
    res = (ctypes.c_double * n)()
    check(lib().lbm_batch_run_to_steady(b, float(tol), int(check_every), int(max_steps),
                                        int(plateau_checks), float(plateau_floor),
                                        int(stall_checks), steps, st,
                                        res))
    return list(steps), list(st), list(res)


def lbm_batch_set_launch(b, threads, blocks_per_cu, graph_steps):
    return check(lib().lbm_batch_set_launch(b, int(threads), int(blocks_per_cu),
                                            int(graph_steps)))


def lbm_batch_autotune(b, steps_per_trial):
    t, bp = ctypes.c_int32(), ctypes.c_int32()
    check(lib().lbm_batch_autotune(b, int(steps_per_trial), ctypes.byref(t), ctypes.byref(bp)))
    return t.value, bp.value


def lbm_batch_launch_info(b):
    t, g, at, gs = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    st = ctypes.c_int64()
    check(lib().lbm_batch_launch_info(b, ctypes.byref(t), ctypes.byref(g), ctypes.byref(at),
                                      ctypes.byref(gs), ctypes.byref(st)))
    return {"threads": t.value, "grid_blocks": g.value, "active_tiles": at.value,
            "graph_steps": gs.value, "steps": st.value}


# ---------------------------------------------------------------------------
# include/lbm_nn.h
# ---------------------------------------------------------------------------

def lbm_nn_param_count():
    return int(lib().lbm_nn_param_count())


def nn_config(grid, batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, target_scale=(1, 1, 1, 1)):
    c = lbm_nn_config()
    c.grid, c.batch, c.lr, c.beta1, c.beta2, c.eps = grid, batch, lr, beta1, beta2, eps
    for i in range(4):
        c.target_scale[i] = float(target_scale[i])
    return c


def lbm_nn_workspace_bytes(cfg):
    n = lib().lbm_nn_workspace_bytes(ctypes.byref(cfg))
    if n == 0:
        raise LbmError(LBM_ERR_ARG, lbm_last_error())
    return n


def lbm_nn_create(cfg, workspace_ptr, workspace_bytes, stream_ptr=None):
    h = vp()
    check(lib().lbm_nn_create(ctypes.byref(cfg), workspace_ptr, workspace_bytes, stream_ptr,
                              ctypes.byref(h)))
    return h.value


def lbm_nn_destroy(h):
    return check(lib().lbm_nn_destroy(h))


def lbm_nn_set_params(h, params_ptr):
    return check(lib().lbm_nn_set_params(h, params_ptr))


def lbm_nn_get_params(h, params_ptr):
    return check(lib().lbm_nn_get_params(h, params_ptr))


def _floats(vals):
    return (ctypes.c_float * len(vals))(*[float(v) for v in vals])


def _ints(vals):
    return (ctypes.c_int32 * len(vals))(*[int(v) for v in vals])


def lbm_nn_forward(h, log10_ra, out_ptr, out_scale=None):
    sc = _floats(out_scale) if out_scale is not None else None
    return check(lib().lbm_nn_forward(h, len(log10_ra), _floats(log10_ra), out_ptr, sc))


def lbm_nn_gradient(h, log10_ra, targets_ptr, target_count, target_index, target_stride,
                    grad_ptr=None):
    loss = ctypes.c_double()
    check(lib().lbm_nn_gradient(h, len(log10_ra), _floats(log10_ra), targets_ptr,
                                int(target_count), _ints(target_index), int(target_stride),
                                grad_ptr, ctypes.byref(loss)))
    return loss.value


def lbm_nn_train_step(h, log10_ra, targets_ptr, target_count, target_index, target_stride,
                      want_loss=True):
    loss = ctypes.c_double()
    check(lib().lbm_nn_train_step(h, len(log10_ra), _floats(log10_ra), targets_ptr,
                                  int(target_count), _ints(target_index), int(target_stride),
                                  ctypes.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def lbm_nn_set_lr(h, lr):
    return check(lib().lbm_nn_set_lr(h, float(lr)))


def lbm_nn_activation(h, layer, n, out_ptr):
    return check(lib().lbm_nn_activation(h, int(layer), int(n), out_ptr))


def lbm_nn_flops(h, n):
    f, t = ctypes.c_double(), ctypes.c_double()
    check(lib().lbm_nn_flops(h, int(n), ctypes.byref(f), ctypes.byref(t)))
    return f.value, t.value
