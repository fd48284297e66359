"""Torch-facing wrapper of the C ABI: device memory and streams come from
PyTorch; every computation is a call into liblbm.so."""
import torch

from . import capi

_PREC = {"fp64": capi.LBM_FP64, "fp32": capi.LBM_FP32, "fp16": capi.LBM_FP32_S16,
         "fp32_s16": capi.LBM_FP32_S16}


def make_params(n=None, Ra=1e3, *, nx=None, ny=None, nz=None, precision="fp32", thermal_q=7,
                **fields):
    """lbm_params with the library defaults (lbm_params_init), then overrides."""
    p = capi.lbm_params_init(n or nx, Ra)
    p.nx = nx or n
    p.ny = ny or n or nx
    p.nz = nz or n or nx
    p.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
    p.thermal_q = thermal_q
    for k, v in fields.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


class Cavity:
    """One differentially heated cavity on one GPU."""

    def __init__(self, params, device="cuda", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.p = params
        self.device = torch.device(device)
        self.nbytes = capi.lbm_workspace_bytes(params)
        self._raw = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._raw.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream
        sp = stream.cuda_stream if stream is not None else None
        self.h = capi.lbm_create(params, self._ws_ptr, self.nbytes, sp)
        self.lattice = capi.lbm_get_lattice(self.h)

    # -- shape helpers --------------------------------------------------
    @property
    def shape(self):
        return (self.p.nz, self.p.ny, self.p.nx)

    @property
    def ncell(self):
        return self.p.nx * self.p.ny * self.p.nz

    def _empty(self, *lead, dtype=torch.float64):
        return torch.empty(*lead, *self.shape, dtype=dtype, device=self.device)

    # -- C ABI calls ----------------------------------------------------
    def step(self, nsteps):
        capi.lbm_step(self.h, nsteps)

    def init_rest(self):
        capi.lbm_init_rest(self.h)

    def init_macros(self, ux=None, uy=None, uz=None, T=None):
        keep = [None if t is None else t.to(self.device, torch.float32).contiguous()
                for t in (ux, uy, uz, T)]
        for t in keep:
            if t is not None and t.numel() != self.ncell:
                raise ValueError(f"field has {t.numel()} values, the grid has {self.ncell}")
        self._inputs_ready()
        capi.lbm_init_macros(self.h, *[None if t is None else t.data_ptr() for t in keep])
        self._sync_if_needed()

    def symmetrize(self, ux=None, uy=None, uz=None, T=None):
        """Project float32 device fields onto the cavity's symmetries, in
        place (lbm_symmetrize)."""
        fs = [ux, uy, uz, T]
        for t in fs:
            if t is not None and (t.dtype != torch.float32 or not t.is_contiguous() or
                                  t.numel() != self.ncell or not t.is_cuda):
                raise ValueError("fields must be contiguous float32 device tensors of the grid")
        self._inputs_ready()
        capi.lbm_symmetrize(self.h, *[None if t is None else t.data_ptr() for t in fs])
        self._sync_if_needed()

    def macros(self, fp64=True):
        dt = torch.float64 if fp64 else torch.float32
        out = self._empty(5, dtype=dt)
        self._inputs_ready()
        capi.lbm_macros(self.h, *[out[i].data_ptr() for i in range(5)], fp64=fp64)
        self._sync_if_needed()
        return {"rho": out[0], "ux": out[1], "uy": out[2], "uz": out[3], "T": out[4]}

    def nusselt(self, local=False):
        if local:
            lh = torch.empty(self.p.nz, self.p.ny, dtype=torch.float64, device=self.device)
            lc = torch.empty_like(lh)
            self._inputs_ready()
            r = capi.lbm_nusselt(self.h, lh.data_ptr(), lc.data_ptr())
            self._sync_if_needed()
            return r, lh, lc
        return capi.lbm_nusselt(self.h)

    def residual(self):
        return capi.lbm_residual(self.h)

    def centerlines(self, profiles=False):
        """Peak velocities of Table 1 (lbm_peaks, units of u0); with
        profiles=True also the two centreline profiles (float64 tensors)."""
        if not profiles:
            return capi.lbm_centerlines(self.h)
        ul = torch.empty(self.p.nz, dtype=torch.float64, device=self.device)
        wl = torch.empty(self.p.nx, dtype=torch.float64, device=self.device)
        self._inputs_ready()
        pk = capi.lbm_centerlines(self.h, ul.data_ptr(), wl.data_ptr())
        return pk, ul, wl

    def run_to_steady(self, tol=1e-8, check_every=1000, max_steps=10 ** 7, plateau_checks=0,
                      plateau_floor=0.0, stall_checks=0):
        """(steps, how, last residual) of lbm_run_to_steady."""
        return capi.lbm_run_to_steady(self.h, tol, check_every, max_steps, plateau_checks,
                                      plateau_floor, stall_checks)

    def populations(self):
        F = self._empty(15)
        G = self._empty(self.p.thermal_q)
        self._inputs_ready()
        capi.lbm_get_populations(self.h, F.data_ptr(), G.data_ptr())
        self._sync_if_needed()
        return F, G

    def set_populations(self, F, G):
        F = torch.as_tensor(F, dtype=torch.float64).to(self.device).contiguous()
        G = torch.as_tensor(G, dtype=torch.float64).to(self.device).contiguous()
        if F.numel() != 15 * self.ncell or G.numel() != self.p.thermal_q * self.ncell:
            raise ValueError("populations must be [15][ncell] and [q][ncell]")
        self._inputs_ready()
        capi.lbm_set_populations(self.h, F.data_ptr(), G.data_ptr())
        self._sync_if_needed()

    def gather_cells(self, cells):
        c = torch.as_tensor(cells, dtype=torch.int64).to(self.device).contiguous()
        n = c.numel()
        F = torch.empty(n, 15, dtype=torch.float64, device=self.device)
        G = torch.empty(n, self.p.thermal_q, dtype=torch.float64, device=self.device)
        self._inputs_ready()
        capi.lbm_gather_cells(self.h, c.data_ptr(), n, F.data_ptr(), G.data_ptr())
        self._sync_if_needed()
        return F, G

    def state_info(self):
        return capi.lbm_state_info(self.h)

    def kernel_name(self):
        return capi.lbm_step_kernel_name(self.h)

    def steps_done(self):
        return capi.lbm_steps_done(self.h)

    def autotune(self, steps_per_trial=5):
        return capi.lbm_autotune(self.h, steps_per_trial)

    def set_block(self, bx, by):
        capi.lbm_set_block(self.h, bx, by)

    def _inputs_ready(self):
        # inputs were produced, and output buffers allocated, on torch's
        # current stream: the library's stream must not run ahead of them
        if self.stream is not None:
            self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _sync_if_needed(self):
        # outputs are consumed on torch's current stream; order them after the
        # library's stream when the two differ
        if self.stream is not None:
            torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def close(self):
        if getattr(self, "h", None):
            capi.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Member(Cavity):
    """A batch member viewed as a cavity (observables only)."""

    def __init__(self, batch, i, params):
        self.p = params
        self.device = batch.device
        self.stream = batch.stream
        self.h = capi.lbm_batch_member(batch.b, i)
        self.lattice = capi.lbm_get_lattice(self.h)
        self._batch = batch

    def close(self):  # released with the batch
        self.h = None


class Batch:
    """Many cavities advanced together (persistent launch, hipGraph)."""

    def __init__(self, params_list, device="cuda", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.params = list(params_list)
        self.n = len(self.params)
        self.device = torch.device(device)
        # graphs need a stream of their own
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.nbytes = capi.lbm_batch_workspace_bytes(self.params)
        self._raw = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._raw.data_ptr() + 255) // 256 * 256
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self.b = capi.lbm_batch_create(self.params, ptr, self.nbytes, self.stream.cuda_stream)
        self.members = [_Member(self, i, self.params[i]) for i in range(self.n)]

    @property
    def cells(self):
        return sum(p.nx * p.ny * p.nz for p in self.params)

    def step(self, nsteps):
        capi.lbm_batch_step(self.b, nsteps)

    def residuals(self):
        return capi.lbm_batch_residuals(self.b, self.n)

    def set_active(self, active):
        capi.lbm_batch_set_active(self.b, active)

    def run_to_steady(self, tol, check_every=1000, max_steps=10 ** 6, plateau_checks=0,
                      plateau_floor=0.0, stall_checks=0):
        return capi.lbm_batch_run_to_steady(self.b, self.n, tol, check_every, max_steps,
                                            plateau_checks, plateau_floor, stall_checks)

    def set_launch(self, threads, blocks_per_cu, graph_steps):
        capi.lbm_batch_set_launch(self.b, threads, blocks_per_cu, graph_steps)

    def autotune(self, steps_per_trial=10):
        return capi.lbm_batch_autotune(self.b, steps_per_trial)

    def launch_info(self):
        return capi.lbm_batch_launch_info(self.b)

    def close(self):
        if getattr(self, "b", None):
            for m in self.members:
                m.close()
            capi.lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
