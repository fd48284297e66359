"""The learned warm start: the encoder-decoder of include/lbm_nn.h on PyTorch
device memory.  Argument marshalling only; every layer, the loss, the
backward pass and Adam run in the library's HIP kernels."""
import math

import numpy as np
import torch

from . import capi


# (level, channels) of each layer's output, in the order of include/lbm_nn.h;
# level l is the grid G / 2^l.
LAYER_NAMES = ["enc1a", "enc1b", "enc2a", "enc2b", "enc3a", "enc3b", "bota", "botb", "botc",
               "dec3a", "dec3b", "dec2a", "dec2b", "dec1a", "dec1b", "head"]
LAYER_OUTPUTS = [(0, 16), (0, 16), (1, 32), (1, 32), (2, 64), (2, 64), (3, 128), (3, 128),
                 (3, 128), (2, 64), (2, 64), (1, 32), (1, 32), (0, 16), (0, 16), (0, 4)]


# (input channels, output channels, kernel edge) of each layer
LAYER_SHAPES = [(4, 16, 3), (16, 16, 3), (16, 32, 3), (32, 32, 3), (32, 64, 3), (64, 64, 3),
                (64, 128, 3), (128, 128, 3), (128, 128, 3), (192, 64, 3), (64, 64, 3),
                (96, 32, 3), (32, 32, 3), (48, 16, 3), (16, 16, 3), (16, 4, 1)]


def init_params(seed):
    """Seeded starting parameters: normal weights with variance 2 / fan-in
    (He initialisation, suited to ReLU), zero biases; flat FP32 vector in
    the library's parameter layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co, k in LAYER_SHAPES:
        fan_in = ci * k ** 3
        parts.append((rng.standard_normal(co * fan_in) * math.sqrt(2.0 / fan_in)).astype(np.float32))
        parts.append(np.zeros(co, dtype=np.float32))
    return np.concatenate(parts)


class WarmStartNet:
    """Network over a G^3 grid with room for `batch` samples per call."""

    def __init__(self, grid, batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 target_scale=(1.0, 1.0, 1.0, 1.0), device="cuda", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.grid, self.batch = grid, batch
        self.device = torch.device(device)
        self.cfg = capi.nn_config(grid, batch, lr, beta1, beta2, eps, target_scale)
        self.nbytes = capi.lbm_nn_workspace_bytes(self.cfg)
        self._raw = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._raw.data_ptr() + 255) // 256 * 256
        self.stream = stream
        self.h = capi.lbm_nn_create(self.cfg, ptr, self.nbytes,
                                    stream.cuda_stream if stream is not None else None)
        self.P = capi.lbm_nn_param_count()

    def _ready(self):
        if self.stream is not None:
            self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _done(self):
        if self.stream is not None:
            torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def set_params(self, theta):
        t = torch.as_tensor(theta, dtype=torch.float32).to(self.device).contiguous()
        if t.numel() != self.P:
            raise ValueError(f"{t.numel()} parameters given, the network has {self.P}")
        self._keep = t
        self._ready()
        capi.lbm_nn_set_params(self.h, t.data_ptr())
        self._done()

    def get_params(self):
        t = torch.empty(self.P, dtype=torch.float32, device=self.device)
        self._ready()
        capi.lbm_nn_get_params(self.h, t.data_ptr())
        self._done()
        return t

    def forward(self, log10_ra, out_scale=None):
        """[n][4][G][G][G] FP32 prediction (times out_scale per channel)."""
        n = len(log10_ra)
        out = torch.empty(n, 4, self.grid, self.grid, self.grid, dtype=torch.float32,
                          device=self.device)
        self._ready()
        capi.lbm_nn_forward(self.h, list(log10_ra), out.data_ptr(), out_scale)
        self._done()
        return out

    def _targets(self, targets):
        g = self.grid
        on_device = targets.is_cuda and (self.device.index is None or
                                         targets.device.index == self.device.index)
        if (targets.dtype != torch.float32 or not targets.is_contiguous() or targets.dim() != 5
                or tuple(targets.shape[1:]) != (4, g, g, g) or not on_device):
            raise ValueError(f"targets must be a contiguous float32 device tensor [N][4][{g}]"
                             f"[{g}][{g}]")
        return targets.data_ptr(), targets.shape[0], 4 * g ** 3

    def gradient(self, log10_ra, targets, index):
        """(loss, gradient [P]) for samples targets[index[i]] (no update)."""
        ptr, count, stride = self._targets(targets)
        g = torch.empty(self.P, dtype=torch.float32, device=self.device)
        self._ready()
        loss = capi.lbm_nn_gradient(self.h, list(log10_ra), ptr, count, list(index), stride,
                                    g.data_ptr())
        self._done()
        return loss, g

    def train_step(self, log10_ra, targets, index, want_loss=True):
        ptr, count, stride = self._targets(targets)
        self._ready()
        loss = capi.lbm_nn_train_step(self.h, list(log10_ra), ptr, count, list(index), stride,
                                      want_loss)
        self._done()
        return loss

    def activation(self, layer, n):
        """Output of a layer of the last forward pass (n samples), FP32
        channels-last [n][g][g][g][c] on the layer's grid (the head's from
        its input of that pass with the current parameters)."""
        level, c = LAYER_OUTPUTS[layer]
        g = self.grid >> level
        out = torch.empty(n, g, g, g, c, dtype=torch.float32, device=self.device)
        self._ready()
        capi.lbm_nn_activation(self.h, layer, n, out.data_ptr())
        self._done()
        return out

    def set_lr(self, lr):
        capi.lbm_nn_set_lr(self.h, lr)

    def flops(self, n):
        return capi.lbm_nn_flops(self.h, n)

    def close(self):
        if getattr(self, "h", None):
            capi.lbm_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
