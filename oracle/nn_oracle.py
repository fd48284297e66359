"""Plain FP64 NumPy reference of the learned warm-start network.

TEST INFRASTRUCTURE ONLY: imported by tests/ (and nothing in the GPU
library).  Every function is the textbook definition written out, slow and
obviously correct, so that the GPU's BF16 kernels can be checked against it.

The network maps the Rayleigh number of a differentially heated cube and
the cell-centre coordinates to the four steady fields (u, v, w, T): a 3D
convolutional encoder-decoder with four resolution levels of 16, 32, 64 and
128 channels, skip connections by channel concatenation, average pooling
down and nearest-neighbour upsampling up, ReLU after every 3x3x3
convolution and a 1x1x1 linear head.

Layouts: activations are channels-last, x[n][z][y][x][c].  A convolution's
weight is w[co][kz][ky][kx][ci] (cross-correlation, zero padding that keeps
the grid size), its bias b[co].  The flattened parameter vector holds, layer
after layer in LAYERS order, the weight (that index order) then the bias.
"""
import math

import numpy as np

BASE = 16
LEVELS = 4
IN_CH = 4   # normalised log10 Ra, x, y, z
OUT_CH = 4  # u, v, w (over u0), T

# (name, input channels, output channels, kernel size, relu).  Decoder
# layers 'a' read the concatenation [skip, upsampled] of their level.
LAYERS = [
    ("enc1a", IN_CH, 16, 3, True), ("enc1b", 16, 16, 3, True),
    ("enc2a", 16, 32, 3, True), ("enc2b", 32, 32, 3, True),
    ("enc3a", 32, 64, 3, True), ("enc3b", 64, 64, 3, True),
    ("bota", 64, 128, 3, True), ("botb", 128, 128, 3, True), ("botc", 128, 128, 3, True),
    ("dec3a", 64 + 128, 64, 3, True), ("dec3b", 64, 64, 3, True),
    ("dec2a", 32 + 64, 32, 3, True), ("dec2b", 32, 32, 3, True),
    ("dec1a", 16 + 32, 16, 3, True), ("dec1b", 16, 16, 3, True),
    ("head", 16, OUT_CH, 1, False),
]


def param_count():
    return sum(co * k ** 3 * ci + co for _, ci, co, k, _ in LAYERS)


def unflatten(theta):
    """Flat parameter vector -> {name: (w, b)} (views)."""
    out, o = {}, 0
    for name, ci, co, k, _ in LAYERS:
        nw = co * k ** 3 * ci
        w = theta[o:o + nw].reshape(co, k, k, k, ci)
        b = theta[o + nw:o + nw + co]
        out[name] = (w, b)
        o += nw + co
    assert o == theta.size
    return out


def init_params(seed):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co, k, _ in LAYERS:
        parts.append(rng.standard_normal(co * k ** 3 * ci) * math.sqrt(2.0 / (ci * k ** 3)))
        parts.append(np.zeros(co))
    return np.concatenate(parts)


# --------------------------------------------------------------------------
# Operations
# --------------------------------------------------------------------------

def conv3d(x, w, b):
    """out[n,z,y,x,o] = b[o] + sum over taps and c of
    x[n, z+kz-p, y+ky-p, x+kx-p, c] w[o,kz,ky,kx,c], p = k // 2, with x = 0
    outside the grid."""
    n, d, h, wd, _ = x.shape
    k = w.shape[1]
    p = k // 2
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (p, p), (0, 0)))
    out = np.zeros((n, d, h, wd, w.shape[0]))
    for kz in range(k):
        for ky in range(k):
            for kx in range(k):
                out += xp[:, kz:kz + d, ky:ky + h, kx:kx + wd, :] @ w[:, kz, ky, kx, :].T
    return out + b


def conv3d_at(x, w, b, pos):
    """conv3d at listed output voxels only: out[i, o] = b[o] + sum over taps
    and c of x[n, z+kz-p, y+ky-p, x+kx-p, c] w[o,kz,ky,kx,c] for pos[i] =
    (n, z, y, x), x = 0 outside the grid; also the sum of the absolute
    values of the terms (for rounding bounds).  Direct summation per voxel,
    for grids too large to convolve whole."""
    pos = np.asarray(pos)
    n, d, h, wd, _ = x.shape
    k = w.shape[1]
    p = k // 2
    out = np.tile(np.asarray(b, dtype=np.float64), (len(pos), 1))
    mag = np.tile(np.abs(np.asarray(b, dtype=np.float64)), (len(pos), 1))
    for kz in range(k):
        for ky in range(k):
            for kx in range(k):
                zz = pos[:, 1] + kz - p
                yy = pos[:, 2] + ky - p
                xx = pos[:, 3] + kx - p
                ok = (zz >= 0) & (zz < d) & (yy >= 0) & (yy < h) & (xx >= 0) & (xx < wd)
                v = np.zeros((len(pos), x.shape[-1]))
                v[ok] = x[pos[ok, 0], zz[ok], yy[ok], xx[ok], :]
                wt = w[:, kz, ky, kx, :]
                out += v @ wt.T
                mag += np.abs(v) @ np.abs(wt).T
    return out, mag


def conv3d_backward(x, w, dout):
    """Gradients of sum(dout * conv3d(x, w, b)) with respect to x, w, b."""
    n, d, h, wd, _ = x.shape
    k = w.shape[1]
    p = k // 2
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (p, p), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for kz in range(k):
        for ky in range(k):
            for kx in range(k):
                win = (slice(None), slice(kz, kz + d), slice(ky, ky + h), slice(kx, kx + wd))
                dxp[win] += dout @ w[:, kz, ky, kx, :]
                dw[:, kz, ky, kx, :] = np.einsum("ndhwo,ndhwc->oc", dout, xp[win])
    dx = dxp[:, p:p + d, p:p + h, p:p + wd, :]
    db = dout.sum(axis=(0, 1, 2, 3))
    return dx, dw, db


def relu(x):
    return np.maximum(x, 0.0)


def avgpool2(x):
    """Mean over non-overlapping 2x2x2 blocks."""
    n, d, h, w, c = x.shape
    return x.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4, 6))


def avgpool2_backward(dy):
    """Adjoint of avgpool2: each child receives 1/8 of its parent's gradient."""
    return upsample2(dy) / 8.0


def upsample2(x):
    """Nearest-neighbour upsampling by 2 along z, y, x."""
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def upsample2_backward(dy):
    """Adjoint of upsample2: sum over each 2x2x2 block."""
    n, d, h, w, c = dy.shape
    return dy.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4, 6))


def inputs(log10_ra, grid):
    """Input channels [n][G][G][G][4]: s = (log10 Ra - 4) / 2 everywhere, and
    the cell-centre coordinates 2 (i + 1/2) / G - 1 along x, y, z."""
    c = 2.0 * (np.arange(grid) + 0.5) / grid - 1.0
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    out = np.empty((len(log10_ra), grid, grid, grid, IN_CH))
    for i, lr in enumerate(log10_ra):
        out[i, ..., 0] = (lr - 4.0) / 2.0
        out[i, ..., 1] = x
        out[i, ..., 2] = y
        out[i, ..., 3] = z
    return out


# --------------------------------------------------------------------------
# Network
# --------------------------------------------------------------------------

def forward(theta, x):
    """Returns (output [n][G][G][G][4], cache of every activation)."""
    P = unflatten(theta)
    a = {"in": x}

    def conv(name, inp):
        w, b = P[name]
        y = conv3d(inp, w, b)
        return relu(y)

    a["enc1a"] = conv("enc1a", x)
    a["enc1b"] = conv("enc1b", a["enc1a"])
    a["pool1"] = avgpool2(a["enc1b"])
    a["enc2a"] = conv("enc2a", a["pool1"])
    a["enc2b"] = conv("enc2b", a["enc2a"])
    a["pool2"] = avgpool2(a["enc2b"])
    a["enc3a"] = conv("enc3a", a["pool2"])
    a["enc3b"] = conv("enc3b", a["enc3a"])
    a["pool3"] = avgpool2(a["enc3b"])
    a["bota"] = conv("bota", a["pool3"])
    a["botb"] = conv("botb", a["bota"])
    a["botc"] = conv("botc", a["botb"])
    a["cat3"] = np.concatenate([a["enc3b"], upsample2(a["botc"])], axis=-1)
    a["dec3a"] = conv("dec3a", a["cat3"])
    a["dec3b"] = conv("dec3b", a["dec3a"])
    a["cat2"] = np.concatenate([a["enc2b"], upsample2(a["dec3b"])], axis=-1)
    a["dec2a"] = conv("dec2a", a["cat2"])
    a["dec2b"] = conv("dec2b", a["dec2a"])
    a["cat1"] = np.concatenate([a["enc1b"], upsample2(a["dec2b"])], axis=-1)
    a["dec1a"] = conv("dec1a", a["cat1"])
    a["dec1b"] = conv("dec1b", a["dec1a"])
    w, b = P["head"]
    out = conv3d(a["dec1b"], w, b)
    return out, a


def mse(out, target):
    """Mean of squared differences over every element."""
    return float(np.mean((out - target) ** 2))


def backward(theta, a, dout, keep=None):
    """Gradient of sum(dout * forward(theta, x)) with respect to theta (flat,
    same layout), by the chain rule through every layer.  keep (a dict), when
    given, receives each layer's (input, gradient of its pre-activation)."""
    P = unflatten(theta)
    grads = {}

    def conv_back(name, inp, out_act, dy):
        w, _ = P[name]
        dpre = dy * (out_act > 0)  # relu
        if keep is not None:
            keep[name] = (inp, dpre)
        dx, dw, db = conv3d_backward(inp, w, dpre)
        grads[name] = (dw, db)
        return dx

    w, _ = P["head"]
    if keep is not None:
        keep["head"] = (a["dec1b"], dout)
    dx, dw, db = conv3d_backward(a["dec1b"], w, dout)
    grads["head"] = (dw, db)
    d = conv_back("dec1b", a["dec1a"], a["dec1b"], dx)
    dcat = conv_back("dec1a", a["cat1"], a["dec1a"], d)
    d_enc1b = dcat[..., :16].copy()
    d = upsample2_backward(dcat[..., 16:])
    d = conv_back("dec2b", a["dec2a"], a["dec2b"], d)
    dcat = conv_back("dec2a", a["cat2"], a["dec2a"], d)
    d_enc2b = dcat[..., :32].copy()
    d = upsample2_backward(dcat[..., 32:])
    d = conv_back("dec3b", a["dec3a"], a["dec3b"], d)
    dcat = conv_back("dec3a", a["cat3"], a["dec3a"], d)
    d_enc3b = dcat[..., :64].copy()
    d = upsample2_backward(dcat[..., 64:])
    d = conv_back("botc", a["botb"], a["botc"], d)
    d = conv_back("botb", a["bota"], a["botb"], d)
    d = conv_back("bota", a["pool3"], a["bota"], d)
    d_enc3b += avgpool2_backward(d)
    d = conv_back("enc3b", a["enc3a"], a["enc3b"], d_enc3b)
    d = conv_back("enc3a", a["pool2"], a["enc3a"], d)
    d_enc2b += avgpool2_backward(d)
    d = conv_back("enc2b", a["enc2a"], a["enc2b"], d_enc2b)
    d = conv_back("enc2a", a["pool1"], a["enc2a"], d)
    d_enc1b += avgpool2_backward(d)
    d = conv_back("enc1b", a["enc1a"], a["enc1b"], d_enc1b)
    conv_back("enc1a", a["in"], a["enc1a"], d)
    flat = []
    for name, *_ in LAYERS:
        dw, db = grads[name]
        flat += [dw.ravel(), db]
    return np.concatenate(flat)


def loss_and_gradient(theta, x, target):
    """MSE loss of the network on (x, target) and its gradient."""
    out, a = forward(theta, x)
    dout = 2.0 * (out - target) / out.size
    return mse(out, target), backward(theta, a, dout)


def adam_step(theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One step of Adam (Kingma & Ba, 2015) with bias correction; t counts
    from 1.  Returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
