"""The warm-start network's BF16 matrix-core kernels against the FP64 NumPy
oracle (oracle/nn_oracle.py).

Per layer, the GPU's own BF16 input activations are fed to the oracle, so
each convolution is checked alone: BF16 products are exact in FP32, the
matrix cores sum up to 27 * 192 of them in FP32 (relative error below
1e-4 of the sum of absolute terms), and the result is rounded once to BF16
(2^-9 relative); the bar is 2^-8 |ref| + 1e-4 sum|terms|.  The whole
network and its gradient carry about 30 such BF16 roundings (activations and
their gradients), about 2^-9 sqrt(30) ~ 1e-2 relative; their bars are 3e-2
(output) and 5e-2 (relative L2 error of each layer's gradient)."""
import numpy as np
import pytest

from gpu_helpers import log, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def net_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_04751_amd import network
    return network


@pytest.fixture(scope="module")
def N():
    from oracle import nn_oracle
    return nn_oracle


def to_bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def params(N, seed):
    """He-initialised weights rounded to BF16 (what the kernels use) and
    small random FP32 biases."""
    theta = N.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    P = N.unflatten(theta)
    for name, *_ in N.LAYERS:
        w, b = P[name]
        w[...] = to_bf16(w)
        b[...] = np.float32(0.05 * rng.standard_normal(b.shape))
    return theta


GRID, LRA = 16, [3.3, 5.2]


def layer_input(N, name, acts, x0):
    """Input of a layer built from the GPU's activations as the kernels see
    it (pooled tensors are rounded to BF16 by the pooling kernel)."""
    pools = {"enc2a": "enc1b", "enc3a": "enc2b", "bota": "enc3b"}
    cats = {"dec3a": ("enc3b", "botc"), "dec2a": ("enc2b", "dec3b"), "dec1a": ("enc1b", "dec2b")}
    order = [l[0] for l in N.LAYERS]
    if name == "enc1a":
        return x0
    if name in pools:
        return to_bf16(N.avgpool2(acts[pools[name]]))
    if name in cats:
        a, b = cats[name]
        return np.concatenate([acts[a], N.upsample2(acts[b])], axis=-1)
    return acts[order[order.index(name) - 1]]


@pytest.mark.parametrize("grid", [16, 32])
def test_each_layer_matches_oracle_on_gpu_inputs(net_mod, N, grid):
    """grid 32 puts the finest level on the LDS-staged brick convolution."""
    log(f"case: nn per-layer forward, grid {grid}")
    theta = params(N, 11)
    net = net_mod.WarmStartNet(grid, 2)
    net.set_params(torch.from_numpy(theta.astype(np.float32)))
    net.forward(LRA)
    acts = {}
    for i, name in enumerate(net_mod.LAYER_NAMES):
        acts[name] = to_np(net.activation(i, 2)).astype(np.float64)
    x0 = to_bf16(N.inputs(LRA, grid))
    P = N.unflatten(theta)
    for name, ci, co, k, relu in N.LAYERS:
        x = layer_input(N, name, acts, x0)
        w, b = P[name]
        ref = N.conv3d(x, w, b)
        bound_terms = N.conv3d(np.abs(x), np.abs(w), np.abs(b))
        if relu:
            ref = N.relu(ref)
        err = np.abs(acts[name] - ref)
        lim = 2.0 ** -8 * np.abs(ref) + 1e-4 * bound_terms
        worst = float(np.max(err - lim))
        log(f"{name}: max err {np.max(err):.2e} (max |ref| {np.max(np.abs(ref)):.2e})")
        assert worst <= 0, (name, worst)
    net.close()


def _sample_voxels(n, g, seed, extra=200):
    """Voxels (sample, z, y, x) of an n x g^3 grid: for every sample the 27
    points of {0, g/2, g-1}^3 (corners, edge and face centres, centre) and
    `extra` seeded random ones."""
    rng = np.random.default_rng(seed)
    pts = []
    for s in range(n):
        for z in (0, g // 2, g - 1):
            for y in (0, g // 2, g - 1):
                for x in (0, g // 2, g - 1):
                    pts.append((s, z, y, x))
        pts += [(s, *rng.integers(0, g, 3)) for _ in range(extra)]
    return np.array(pts, dtype=np.int64)


def test_each_layer_at_the_production_shape(net_mod, N):
    """Grid 64, batch 8 (the warm start's training shape): every launch
    variant of the forward pass at its production size -- the brick kernel
    with one output group on 64^3 (16 and 48 input channels), two groups on
    32^3, the 16^3 brick grid, the four-tile kernel of the 4-channel input
    layer, the split-k kernel on 8^3, the head on the vector units -- checked per layer on
    the GPU's own inputs at sampled voxels (every sample's corners, edge and
    face centres and 200 random voxels), which the oracle sums directly.
    Same per-element bar as the small grids: 2^-8 |ref| + 1e-4 sum|terms|."""
    grid, n = 64, 8
    log(f"case: nn per-layer forward, grid {grid}, batch {n}, sampled voxels")
    theta = params(N, 19)
    lra = list(np.linspace(3.1, 5.9, n))
    net = net_mod.WarmStartNet(grid, n)
    net.set_params(torch.from_numpy(theta.astype(np.float32)))
    net.forward(lra)
    acts = {}
    for i, name in enumerate(net_mod.LAYER_NAMES):
        acts[name] = to_np(net.activation(i, n)).astype(np.float64)
    net.close()
    x0 = to_bf16(N.inputs(lra, grid))
    P = N.unflatten(theta)
    for li, (name, ci, co, k, relu) in enumerate(N.LAYERS):
        x = layer_input(N, name, acts, x0)
        g = x.shape[1]
        pos = _sample_voxels(n, g, 100 + li)
        w, b = P[name]
        ref, mag = N.conv3d_at(x, w, b, pos)
        if relu:
            ref = N.relu(ref)
        got = acts[name][pos[:, 0], pos[:, 1], pos[:, 2], pos[:, 3], :]
        err = np.abs(got - ref)
        lim = 2.0 ** -8 * np.abs(ref) + 1e-4 * mag
        worst = float(np.max(err - lim))
        log(f"{name} ({g}^3, {len(pos)} voxels): max err {np.max(err):.2e} "
            f"(max |ref| {np.max(np.abs(ref)):.2e})")
        assert worst <= 0, (name, worst)


def test_network_output_matches_oracle(net_mod, N):
    log("case: nn full forward, grid 16 and 8")
    theta = params(N, 12)
    for grid in (16, 8):
        net = net_mod.WarmStartNet(grid, 2)
        net.set_params(torch.from_numpy(theta.astype(np.float32)))
        scale = [2.0, 1.0, 0.5, 1.0]
        out = to_np(net.forward(LRA, out_scale=scale)).astype(np.float64)
        ref, _ = N.forward(theta, to_bf16(N.inputs(LRA, grid)))
        ref = np.moveaxis(ref, -1, 1) * np.array(scale)[None, :, None, None, None]
        err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
        log(f"grid {grid}: normalised max error {err:.2e}")
        assert err < 3e-2
        net.close()


def gpu_cache(N, net_mod, net, n, x0):
    """The oracle's activation cache filled with the GPU's own activations
    (pooled inputs rounded to BF16 as the pooling kernel does)."""
    acts = {name: to_np(net.activation(i, n)).astype(np.float64)
            for i, name in enumerate(net_mod.LAYER_NAMES)}
    a = dict(acts)
    a["in"] = x0
    a["pool1"] = to_bf16(N.avgpool2(acts["enc1b"]))
    a["pool2"] = to_bf16(N.avgpool2(acts["enc2b"]))
    a["pool3"] = to_bf16(N.avgpool2(acts["enc3b"]))
    a["cat3"] = np.concatenate([acts["enc3b"], N.upsample2(acts["botc"])], axis=-1)
    a["cat2"] = np.concatenate([acts["enc2b"], N.upsample2(acts["dec3b"])], axis=-1)
    a["cat1"] = np.concatenate([acts["enc1b"], N.upsample2(acts["dec2b"])], axis=-1)
    return a, acts["head"]


def elementwise_excess(N, theta, a, dout, g, ref_g):
    """Element-by-element check of a gradient computed on the GPU's own
    activations.  The GPU stores every gradient tensor of the chain in BF16:
    each of the at most 20 roundings on the way from the loss to a parameter
    (16 layers, three pooling and three upsampling adjoints) changes a value
    by at most 2^-9 of itself, and the linear backward maps carry that change
    on by at most the absolute chain: the same backward pass run on |theta|,
    |activations| and |dout| (same ReLU masks).  Per element, |g - ref| must
    stay below 20 * 2^-9 of that absolute gradient (plus FP32 summation,
    1e-4 of it).  Returns the largest (|g - ref| - bound) / bound per layer
    (<= 0 passes) and the largest ratio |g - ref| / absolute gradient."""
    a_abs = {k: np.abs(v) for k, v in a.items()}
    A = N.backward(np.abs(theta), a_abs, np.abs(dout))
    bound = (20 * 2.0 ** -9 + 1e-4) * A + 1e-30
    out, o = {}, 0
    for name, ci, co, k, _ in N.LAYERS:
        m = co * k ** 3 * ci + co
        d = np.abs(g[o:o + m] - ref_g[o:o + m])
        out[name] = (float(np.max((d - bound[o:o + m]) / bound[o:o + m])),
                     float(np.max(d / (A[o:o + m] + 1e-30))))
        o += m
    return out


def per_layer_rel(N, g, ref_g):
    out, o = {}, 0
    for name, ci, co, k, _ in N.LAYERS:
        n = co * k ** 3 * ci + co
        a, b = g[o:o + n], ref_g[o:o + n]
        out[name] = (np.linalg.norm(a - b) / np.linalg.norm(b),
                     float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b))))
        o += n
    return out


def test_gradient_matches_oracle(net_mod, N):
    """Two checks of lbm_nn_gradient.  (1) The oracle's backward pass run on
    the GPU's own activations (same ReLU masks, same layer inputs) and on
    the GPU's output: the remaining difference is the BF16 rounding of the
    gradient tensors, about 10 roundings deep at the first layer, so each
    layer's relative L2 error stays below 2e-2.  (2) The pure oracle from
    the inputs: on a 16^3 grid the coarse levels hold 4^3 and 2^3 cells, and
    ReLU units whose input is within BF16 rounding of zero switch, so only
    the direction is held: cosine above 0.99 per layer, loss within 2e-2."""
    log("case: nn gradient, grid 16")
    theta = params(N, 13)
    rng = np.random.default_rng(14)
    tscale = [20.0, 20.0, 20.0, 1.0]
    targets = (0.02 * rng.standard_normal((3, 4, GRID, GRID, GRID))).astype(np.float32)
    index = [2, 0]
    net = net_mod.WarmStartNet(GRID, 2, target_scale=tscale)
    net.set_params(torch.from_numpy(theta.astype(np.float32)))
    loss, g = net.gradient(LRA, torch.from_numpy(targets).cuda(), index)
    g = to_np(g).astype(np.float64)
    tg = np.moveaxis(targets[index].astype(np.float64), 1, -1) * np.array(tscale)
    x0 = to_bf16(N.inputs(LRA, GRID))
    a, out = gpu_cache(N, net_mod, net, 2, x0)
    net.close()
    dout = 2.0 * (out - tg) / out.size
    ref_same = N.backward(theta, a, dout)
    same = per_layer_rel(N, g, ref_same)
    elem = elementwise_excess(N, theta, a, dout, g, ref_same)
    ref_loss, ref_g = N.loss_and_gradient(theta, x0, tg)
    pure = per_layer_rel(N, g, ref_g)
    log(f"loss {loss:.6e} ref {ref_loss:.6e}")
    for name in same:
        log(f"{name}: same activations rel {same[name][0]:.2e}, element/abs-chain "
            f"{elem[name][1]:.2e}; pure oracle rel {pure[name][0]:.2e} cosine "
            f"{pure[name][1]:.5f}")
    assert abs(loss - ref_loss) < 2e-2 * ref_loss
    bad = {k: v[0] for k, v in same.items() if not v[0] < 2e-2}
    assert not bad, bad
    bad = {k: v[0] for k, v in elem.items() if not v[0] <= 0}
    assert not bad, bad
    bad = {k: v[1] for k, v in pure.items() if not v[1] > 0.99}
    assert not bad, bad


def test_first_adam_step(net_mod, N):
    """Step 1 of Adam moves every parameter by lr g / (|g| + eps)."""
    log("case: nn adam step")
    theta = params(N, 15).astype(np.float32)
    rng = np.random.default_rng(16)
    targets = torch.from_numpy((0.1 * rng.standard_normal((2, 4, 8, 8, 8))).astype(np.float32))
    targets = targets.cuda()
    lr = 1e-3
    net = net_mod.WarmStartNet(8, 2, lr=lr)
    net.set_params(torch.from_numpy(theta))
    _, g = net.gradient(LRA, targets, [0, 1])
    net.train_step(LRA, targets, [0, 1])
    t1 = to_np(net.get_params()).astype(np.float64)
    g = to_np(g).astype(np.float64)
    expect = theta.astype(np.float64) - lr * g / (np.abs(g) + 1e-8)
    err = np.max(np.abs(t1 - expect) - 1e-6 * np.abs(theta))
    log(f"adam: max deviation {err:.2e} of lr {lr}")
    assert err < 1e-3 * lr
    net.close()


def test_training_lowers_the_loss(net_mod, N):
    """A few dozen steps on four smooth targets (one per Rayleigh number)."""
    log("case: nn training smoke")
    g = 16
    c = (np.arange(g) + 0.5) / g
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    lra = [3.0, 3.8, 4.6, 5.4]
    tg = np.stack([np.stack([np.sin(np.pi * x) * np.sin(2 * np.pi * z) * r / 6,
                             0 * x, -np.sin(2 * np.pi * x) * np.sin(np.pi * z) * r / 6,
                             0.5 - x + 0.1 * r * np.sin(np.pi * z)]) for r in lra])
    targets = torch.from_numpy(tg.astype(np.float32)).cuda()
    net = net_mod.WarmStartNet(g, 4, lr=2e-3)
    net.set_params(torch.from_numpy(N.init_params(3).astype(np.float32)))
    losses = [net.train_step(lra, targets, [0, 1, 2, 3]) for _ in range(60)]
    log(f"loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert np.isfinite(losses).all() and losses[-1] < 0.3 * losses[0]
    net.close()


def test_gradient_on_the_full_grid(net_mod, N):
    """lbm_nn_gradient on the 64^3 grid the warm start trains on (one
    sample), where every level has its production shape: the weight
    gradients of levels 0-2 come from the brick kernel (16, 32 and 64 output
    channels), the coarse convolutions from the split-k kernel.  The oracle's
    backward pass runs on the GPU's own activations, so the remaining
    difference is the BF16 rounding of the gradient tensors: relative L2
    error of each layer's gradient below 2e-2 (as on the 16^3 grid), and
    every element within its rounding bound (elementwise_excess).  The
    forward pass at this shape is checked layer by layer in
    test_each_layer_at_the_production_shape."""
    log("case: nn gradient, grid 64, batch 1")
    g = 64
    theta = params(N, 17)
    rng = np.random.default_rng(18)
    tscale = [20.0, 20.0, 20.0, 1.0]
    targets = (0.02 * rng.standard_normal((1, 4, g, g, g))).astype(np.float32)
    lra = [4.4]
    net = net_mod.WarmStartNet(g, 1, target_scale=tscale)
    net.set_params(torch.from_numpy(theta.astype(np.float32)))
    loss, grad = net.gradient(lra, torch.from_numpy(targets).cuda(), [0])
    grad = to_np(grad).astype(np.float64)
    tg = np.moveaxis(targets.astype(np.float64), 1, -1) * np.array(tscale)
    x0 = to_bf16(N.inputs(lra, g))
    a, out = gpu_cache(N, net_mod, net, 1, x0)
    net.close()
    dout = 2.0 * (out - tg) / out.size
    ref_same = N.backward(theta, a, dout)
    same = per_layer_rel(N, grad, ref_same)
    elem = elementwise_excess(N, theta, a, dout, grad, ref_same)
    for name in same:
        log(f"{name}: same activations rel {same[name][0]:.2e}, element/abs-chain "
            f"{elem[name][1]:.2e}")
    bad = {k: v[0] for k, v in same.items() if not v[0] < 2e-2}
    assert not bad, bad
    bad = {k: v[0] for k, v in elem.items() if not v[0] <= 0}
    assert not bad, bad


def test_gradient_of_a_repeated_batch(net_mod, N):
    """Nine copies of one 64^3 sample against that sample alone: the loss
    is a mean over the batch, so both calls have the same loss and the same
    gradient.  At nine samples each thread of the head's backward pass takes
    an odd number of voxel passes (the pass pairs end on a single voxel),
    and the weight gradients sum over nine times as many voxels.  The loss
    agrees to 1e-6 (each sample's forward pass is the same arithmetic, the
    FP64 loss sums are grouped differently); the gradients differ by the
    BF16 rounding of gradient tensors scaled by 1/9, so each layer's
    relative L2 difference stays below 2e-2, as against the oracle."""
    log("case: nn gradient, grid 64, batch 9 of one sample against batch 1")
    g = 64
    theta = params(N, 19)
    rng = np.random.default_rng(20)
    targets = torch.from_numpy(
        (0.02 * rng.standard_normal((1, 4, g, g, g))).astype(np.float32)).cuda()
    tscale = [20.0, 20.0, 20.0, 1.0]
    res = {}
    for n in (1, 9):
        net = net_mod.WarmStartNet(g, n, target_scale=tscale)
        net.set_params(torch.from_numpy(theta.astype(np.float32)))
        loss, grad = net.gradient([4.1] * n, targets, [0] * n)
        res[n] = (loss, to_np(grad).astype(np.float64))
        net.close()
    (l1, g1), (l9, g9) = res[1], res[9]
    rel = per_layer_rel(N, g9, g1)
    log(f"loss {l9:.9e} vs {l1:.9e}; " +
        ", ".join(f"{k} {v[0]:.1e}" for k, v in rel.items()))
    assert abs(l9 - l1) <= 1e-6 * l1
    bad = {k: v[0] for k, v in rel.items() if not v[0] < 2e-2}
    assert not bad, bad


def test_packed_weights_follow_adam(net_mod, N):
    """A training step re-packs the updated weights into their two BF16
    copies (the packed rows of the forward convolutions and the transposed
    ones of the input gradients).  After three steps, a second network given
    the same parameters (which packs them on their own) must compute the
    same output, loss and gradient, bit for bit."""
    log("case: nn packed copies after Adam, grid 16")
    rng = np.random.default_rng(21)
    targets = torch.from_numpy(
        (0.1 * rng.standard_normal((2, 4, GRID, GRID, GRID))).astype(np.float32)).cuda()
    a = net_mod.WarmStartNet(GRID, 2, lr=1e-2)
    a.set_params(torch.from_numpy(params(N, 22).astype(np.float32)))
    for _ in range(3):
        a.train_step(LRA, targets, [1, 0])
    b = net_mod.WarmStartNet(GRID, 2)
    b.set_params(a.get_params())
    res = []
    for net in (a, b):
        out = to_np(net.forward(LRA))
        loss, g = net.gradient(LRA, targets, [0, 1])
        res.append((out, loss, to_np(g)))
        net.close()
    (oa, la, ga), (ob, lb, gb) = res
    log(f"output max diff {np.abs(oa - ob).max():.1e}, loss {la:.9e} vs {lb:.9e}")
    assert np.array_equal(oa, ob)
    assert la == lb
    assert np.array_equal(ga, gb)


@pytest.mark.parametrize("grid", [16, 64])
def test_every_gradient_entry_is_written(net_mod, N, grid):
    """The gradient buffer is not cleared between calls: the head's sums and
    every layer's weight-gradient reduction write each entry once.  A call
    after one with other targets must therefore give, bit for bit, what a
    fresh network gives (an entry left unwritten would keep the first
    call's value; both networks stay open, so the second cannot reuse the
    first's memory).  Grid 16 reaches the tiled weight-gradient kernel (4^3
    and 2^3 levels) and the 8-cell one, grid 64 the brick ones at every
    level but the 8-cell bottleneck."""
    log(f"case: nn gradient entries all written, grid {grid}")
    rng = np.random.default_rng(23)
    t1, t2 = [torch.from_numpy((0.1 * rng.standard_normal((1, 4, grid, grid, grid)))
                               .astype(np.float32)).cuda() for _ in range(2)]
    theta = torch.from_numpy(params(N, 24).astype(np.float32))
    lra = [3.9]
    a = net_mod.WarmStartNet(grid, 1)
    b = net_mod.WarmStartNet(grid, 1)
    a.set_params(theta)
    b.set_params(theta)
    a.gradient(lra, t1, [0])
    la, ga = a.gradient(lra, t2, [0])
    lb, gb = b.gradient(lra, t2, [0])
    ga, gb = to_np(ga), to_np(gb)
    a.close()
    b.close()
    log(f"loss {la:.9e} vs {lb:.9e}; entries differing {int((ga != gb).sum())} of {ga.size}")
    assert la == lb
    assert np.array_equal(ga, gb)
