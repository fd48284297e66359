"""Pins of the network oracle (oracle/nn_oracle.py) against definitions that
do not come from the oracle itself: brute-force loops, a library
correlation, central finite differences, exact adjoint identities and the
closed form of Adam's first step."""
import math

import numpy as np
import pytest

from oracle import nn_oracle as N


def test_conv3d_equals_brute_force_loops():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 4, 5, 2))
    w = rng.standard_normal((3, 3, 3, 3, 2))
    b = rng.standard_normal(3)
    out = N.conv3d(x, w, b)
    n_, d, h, wd, ci = x.shape
    for n in range(2):
        for z in range(d):
            for y in range(h):
                for xx in range(wd):
                    for o in range(3):
                        s = b[o]
                        for kz in range(3):
                            for ky in range(3):
                                for kx in range(3):
                                    zz, yy, x2 = z + kz - 1, y + ky - 1, xx + kx - 1
                                    if 0 <= zz < d and 0 <= yy < h and 0 <= x2 < wd:
                                        for c in range(ci):
                                            s += x[n, zz, yy, x2, c] * w[o, kz, ky, kx, c]
                        assert abs(out[n, z, y, xx, o] - s) < 1e-12


def test_conv3d_equals_library_correlation():
    ndimage = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 6, 5, 7, 3))
    w = rng.standard_normal((4, 3, 3, 3, 3))
    b = rng.standard_normal(4)
    out = N.conv3d(x, w, b)
    for o in range(4):
        ref = b[o] + sum(ndimage.correlate(x[0, ..., c], w[o, ..., c], mode="constant", cval=0.0)
                         for c in range(3))
        assert np.max(np.abs(out[0, ..., o] - ref)) < 1e-12
    # 1x1x1 kernel: a per-voxel matrix product
    w1 = rng.standard_normal((2, 1, 1, 1, 3))
    assert np.allclose(N.conv3d(x, w1, np.zeros(2)), x @ w1[:, 0, 0, 0, :].T, atol=1e-14)


def test_conv3d_at_equals_brute_force_loops():
    """The per-voxel form (for grids too large to convolve whole) against
    the loops written out, at every voxel of a ragged grid, with its sum of
    absolute terms; and the 1x1x1 case."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 4, 5, 2))
    w = rng.standard_normal((3, 3, 3, 3, 2))
    b = rng.standard_normal(3)
    pos = np.array([(n, z, y, xx) for n in range(2) for z in range(3) for y in range(4)
                    for xx in range(5)])
    out, mag = N.conv3d_at(x, w, b, pos)
    for i, (n, z, y, xx) in enumerate(pos):
        for o in range(3):
            s, m = b[o], abs(b[o])
            for kz in range(3):
                for ky in range(3):
                    for kx in range(3):
                        zz, yy, x2 = z + kz - 1, y + ky - 1, xx + kx - 1
                        if 0 <= zz < 3 and 0 <= yy < 4 and 0 <= x2 < 5:
                            for c in range(2):
                                t = x[n, zz, yy, x2, c] * w[o, kz, ky, kx, c]
                                s += t
                                m += abs(t)
            assert abs(out[i, o] - s) < 1e-12 and abs(mag[i, o] - m) < 1e-12
    w1 = rng.standard_normal((4, 1, 1, 1, 2))
    out1, _ = N.conv3d_at(x, w1, np.zeros(4), pos)
    assert np.allclose(out1, x[pos[:, 0], pos[:, 1], pos[:, 2], pos[:, 3]] @ w1[:, 0, 0, 0, :].T,
                       atol=1e-14)


def test_conv3d_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 4, 3, 5, 2))
    w = rng.standard_normal((3, 3, 3, 3, 2))
    b = rng.standard_normal(3)
    r = rng.standard_normal((1, 4, 3, 5, 3))
    f = lambda x_, w_, b_: float(np.sum(r * N.conv3d(x_, w_, b_)))
    dx, dw, db = N.conv3d_backward(x, w, r)
    h = 1e-6
    for idx in [(0, 0, 0, 0, 0), (0, 3, 2, 4, 1), (0, 1, 1, 2, 0), (0, 2, 0, 3, 1)]:
        e = np.zeros_like(x)
        e[idx] = h
        assert abs((f(x + e, w, b) - f(x - e, w, b)) / (2 * h) - dx[idx]) < 1e-7
    for idx in [(0, 0, 0, 0, 0), (2, 1, 2, 0, 1), (1, 2, 2, 2, 0)]:
        e = np.zeros_like(w)
        e[idx] = h
        assert abs((f(x, w + e, b) - f(x, w - e, b)) / (2 * h) - dw[idx]) < 1e-7
    for o in range(3):
        e = np.zeros(3)
        e[o] = h
        assert abs((f(x, w, b + e) - f(x, w, b - e)) / (2 * h) - db[o]) < 1e-7


def test_pool_and_upsample_values_and_adjoints():
    x = np.arange(2 * 4 * 4 * 4 * 3, dtype=np.float64).reshape(2, 4, 4, 4, 3)
    p = N.avgpool2(x)
    # block (0,0,0) of channel 0 holds x[0, z, y, x, 0] for z, y, x in {0, 1}
    blk = [x[0, z, y, xx, 0] for z in (0, 1) for y in (0, 1) for xx in (0, 1)]
    assert p[0, 0, 0, 0, 0] == sum(blk) / 8
    u = N.upsample2(p)
    assert u.shape == x.shape and u[1, 3, 2, 3, 2] == p[1, 1, 1, 1, 2]
    rng = np.random.default_rng(4)
    a = rng.standard_normal((2, 4, 6, 8, 3))
    c = rng.standard_normal((2, 2, 3, 4, 3))
    assert abs(np.sum(N.avgpool2(a) * c) - np.sum(a * N.avgpool2_backward(c))) < 1e-12
    assert abs(np.sum(N.upsample2(c) * a) - np.sum(c * N.upsample2_backward(a))) < 1e-12


def test_inputs_encode_rayleigh_and_coordinates():
    x = N.inputs([3.0, 6.0], 4)
    assert np.all(x[0, ..., 0] == -0.5) and np.all(x[1, ..., 0] == 1.0)
    c = np.array([-0.75, -0.25, 0.25, 0.75])
    assert np.array_equal(x[0, 1, 2, :, 1], c)   # x varies fastest
    assert np.array_equal(x[0, 1, :, 3, 2], c)
    assert np.array_equal(x[0, :, 0, 2, 3], c)


def test_network_shape_and_parameter_count():
    assert N.param_count() == sum(co * k ** 3 * ci + co for _, ci, co, k, _ in N.LAYERS)
    assert 1.8e6 < N.param_count() < 2.1e6  # "about 2 M parameters"
    theta = N.init_params(0)
    out, a = N.forward(theta, N.inputs([4.0], 8))
    assert out.shape == (1, 8, 8, 8, 4)
    assert a["botc"].shape == (1, 1, 1, 1, 128)


def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    theta = N.init_params(7)
    x = N.inputs([3.4, 5.1], 8)
    target = 0.3 * rng.standard_normal((2, 8, 8, 8, 4))
    loss, g = N.loss_and_gradient(theta, x, target)
    f = lambda th: N.mse(N.forward(th, x)[0], target)
    # coordinates in the first, a middle and the last layers, weights and biases
    offs, o = {}, 0
    for name, ci, co, k, _ in N.LAYERS:
        offs[name] = (o, co * k ** 3 * ci, co)
        o += co * k ** 3 * ci + co
    picks = []
    for name in ("enc1a", "enc2b", "bota", "botc", "dec3a", "dec1a", "dec1b", "head"):
        base, nw, co = offs[name]
        picks += [base + int(rng.integers(nw)), base + nw + int(rng.integers(co))]
    h = 1e-6
    for i in picks:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (f(theta + e) - f(theta - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_first_step_closed_form():
    """With m0 = v0 = 0 the bias-corrected moments of step 1 are g and g^2,
    so the step is lr g / (|g| + eps)."""
    rng = np.random.default_rng(6)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    z = np.zeros(50)
    t1, m, v = N.adam_step(th, z, z, g, 1, lr=1e-3)
    assert np.max(np.abs(t1 - (th - 1e-3 * g / (np.abs(g) + 1e-8)))) < 1e-15
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # a constant gradient keeps the bias-corrected moments at g and g^2, so
    # every step is lr g / (|g| + eps)
    th2, m2, v2 = t1, m, v
    for t in range(2, 6):
        th3, m2, v2 = N.adam_step(th2, m2, v2, g, t, lr=1e-3)
        assert np.max(np.abs(th3 - th2 + 1e-3 * g / (np.abs(g) + 1e-8))) < 1e-14
        th2 = th3
