"""Pins of the FP64 warm-start network oracle: convolution against a library
routine, adjoint pairs, central finite differences of the loss, the closed
form of the first Adam step, and exact bfloat16 rounding.  CPU only."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn_oracle as net


def test_conv3x3_matches_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 9, 7))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = net.conv3x3(x, w, b)
    for n in range(2):
        for co in range(4):
            ref = b[co] + sum(correlate2d(x[n, ci], w[co, ci], mode="same", boundary="fill")
                              for ci in range(3))
            assert np.max(np.abs(y[n, co] - ref)) < 1e-12


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 8, 6))
    y = rng.standard_normal((2, 3, 4, 3))
    assert abs(np.sum(net.avgpool2(x) * y) - np.sum(x * net.avgpool2_backward(y))) < 1e-12
    z = rng.standard_normal((2, 3, 8, 6))
    assert abs(np.sum(net.upsample2(y) * z) - np.sum(y * net.upsample2_backward(z))) < 1e-12


def test_parameter_count_about_two_million():
    n = net.n_params(32, 4)
    assert 1.8e6 < n < 2.1e6


@pytest.mark.parametrize("levels", [2, 3])
def test_gradients_match_central_differences(levels):
    rng = np.random.default_rng(2 + levels)
    c0, s = 2, 8
    params = net.init_params(3, c0, levels)
    # small non-zero biases so every bias gradient is exercised
    params = [p + 0.05 * rng.standard_normal(p.shape) for p in params]
    x = rng.uniform(0, 1, size=(2, 1, s, s))
    target = rng.standard_normal((2, 2, s, s))
    loss, grads, _ = net.loss_and_grads(params, x, target, levels)
    flat = net.flatten(params)
    gflat = net.flatten(grads)
    idx = rng.choice(flat.size, size=60, replace=False)
    h = 1e-6
    for k in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[k] += h
        fm[k] -= h
        lp = net.loss_and_grads(net.unflatten(fp, c0, levels), x, target, levels)[0]
        lm = net.loss_and_grads(net.unflatten(fm, c0, levels), x, target, levels)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gflat[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, fd, gflat[k])


def test_first_adam_step_closed_form():
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -0.25, 2.0])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    p2, m2, v2 = net.adam_step(p, g, m, v, 1, lr=0.01)
    # bias correction makes the first step lr * g / (|g| + eps)
    assert np.allclose(p2[0], p[0] - 0.01 * g[0] / (np.abs(g[0]) + 1e-8), atol=1e-15)
    assert np.allclose(m2[0], 0.1 * g[0]) and np.allclose(v2[0], 0.001 * g[0] ** 2)


def test_bf16_rounding_ties_to_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.0e-3])
    r = net.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # halfway, even mantissa below
    assert r[2] == 1.0 + 2 ** -6             # halfway, rounds up to even
    assert r[3] == -2.5
    assert abs(r[4] - 3.0e-3) <= 2 ** -8 * 3.0e-3  # half an ulp (7 stored bits)


def test_preprocess_constant_frames_and_clipping():
    I = np.full((2, 8, 8), 3.0)
    I[1] = -1.0                                 # negative counts count as zero
    x = net.preprocess(I)
    assert x.shape == (2, 1, 4, 4)
    assert np.allclose(x[0], np.log(13.0) / 10.0, atol=1e-15)
    assert np.all(x[1] == 0.0)
    J = np.zeros((1, 4, 4))
    J[0, 2, 3] = np.e - 1.0                     # one count in block (1, 1),
    x = net.preprocess(J)[0, 0]                 # which moves to (0, 0)
    assert abs(x[0, 0] - 0.1) < 1e-15 and np.count_nonzero(x) == 1
    # the zero-frequency pixel of a 16 x 16 frame lands at the centre block
    # (4, 4) of the 8 x 8 input, its negative-frequency neighbours (pixel 15)
    # in the block before it
    K = np.zeros((1, 16, 16))
    K[0, 0, 0] = np.e - 1.0
    K[0, 15, 15] = np.e ** 2 - 1.0
    x = net.preprocess(K)[0, 0]
    assert abs(x[4, 4] - 0.1) < 1e-15 and abs(x[3, 3] - 0.2) < 1e-15
    assert np.count_nonzero(x) == 2


def test_patches_reproduce_constants_and_interior_linear_ramps():
    s = 6
    a = np.arange(s, dtype=float)
    y = np.zeros((1, 2, s, s))
    y[0, 0] = 2.0 + 0.5 * a[:, None] - 0.25 * a[None, :]
    y[0, 1] = -1.0
    z = net.patches(y)[0]
    # bilinear interpolation is exact for affine fields away from the clamp
    u = np.arange(1, 2 * s - 1)
    c = u / 2.0 - 0.25
    ref = 2.0 + 0.5 * c[:, None] - 0.25 * c[None, :]
    assert np.max(np.abs(z.real[1:-1, 1:-1] - ref)) < 1e-13
    assert np.all(z.imag == -1.0)
    # the clamped border rows repeat the first input row
    assert np.allclose(z.real[0], z.real[0, :] * 0 + (2.0 + 0.0 - 0.25 * np.clip(
        np.arange(2 * s) / 2.0 - 0.25, 0, s - 1)))


# ---------------------------------------------------------------------------
# the bfloat16 rounding hook, pinned by an independent engine: the same
# network built from torch's CPU convolutions (float64) and differentiated by
# torch's autograd, with the roundings placed as custom autograd steps.  A
# rounding missing, misplaced (skip concatenation, second convolution of a
# level, head input) or applied to the bias gradient moves some values by a
# bfloat16 ulp (~4e-3 relative) and fails the 1e-10 bar.
# ---------------------------------------------------------------------------
def _torch_rounded_network(levels):
    torch = pytest.importorskip("torch")
    F = torch.nn.functional

    def bf16(t):
        # float64 -> float32 -> bfloat16 (nearest even) -> float64
        return t.float().to(torch.bfloat16).to(torch.float64)

    class RoundInput(torch.autograd.Function):
        """bfloat16 input of a 3x3 convolution; the gradient passes as is."""
        @staticmethod
        def forward(ctx, t):
            return bf16(t)

        @staticmethod
        def backward(ctx, g):
            return g

    class RoundOutputGrad(torch.autograd.Function):
        """Identity forward; the output gradient entering the convolution's
        weight and data gradients is rounded to bfloat16."""
        @staticmethod
        def forward(ctx, t):
            return t.clone()

        @staticmethod
        def backward(ctx, g):
            return bf16(g)

    def conv3(x, w, b):
        y = RoundOutputGrad.apply(F.conv2d(RoundInput.apply(x), w, padding=1))
        # the bias is added after the rounding step, so its gradient is the
        # unrounded output gradient
        return y + b[None, :, None, None]

    def forward(params, x):
        it = iter(range(0, len(params), 2))
        h, skips = x, []
        for l in range(levels):
            i = next(it)
            h = torch.relu(conv3(h, params[i], params[i + 1]))
            i = next(it)
            h = torch.relu(conv3(h, params[i], params[i + 1]))
            skips.append(h)
            if l < levels - 1:
                h = F.avg_pool2d(h, 2)
        for l in range(levels - 2, -1, -1):
            u = torch.cat([F.interpolate(h, scale_factor=2, mode="nearest"), skips[l]], dim=1)
            i = next(it)
            h = torch.relu(conv3(u, params[i], params[i + 1]))
            i = next(it)
            h = torch.relu(conv3(h, params[i], params[i + 1]))
        i = next(it)
        return F.conv2d(h, params[i], params[i + 1])     # 1x1 head, not rounded

    return torch, forward


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_bf16_activation_hook_against_torch_autograd(levels):
    torch, tforward = _torch_rounded_network(levels)
    rng = np.random.default_rng(40 + levels)
    c0, s = 3, 8
    params = net.init_params(41, c0, levels)
    params = [p + 0.05 * rng.standard_normal(p.shape) for p in params]
    x = rng.uniform(0, 1, size=(2, 1, s, s))
    target = rng.standard_normal((2, 2, s, s))
    loss, grads, y = net.loss_and_grads(params, x, target, levels, act_round=net.bf16_round)
    tp = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in params]
    ty = tforward(tp, torch.tensor(x))
    tl = torch.mean((ty - torch.tensor(target)) ** 2)
    tl.backward()
    yt = ty.detach().numpy()
    assert np.max(np.abs(y - yt)) <= 1e-10 * np.max(np.abs(yt))
    assert abs(loss - tl.item()) <= 1e-12 * abs(loss)
    for k, (g, t) in enumerate(zip(grads, tp)):
        gt = t.grad.numpy()
        assert np.max(np.abs(g - gt)) <= 1e-10 * max(np.max(np.abs(gt)), 1e-30), k
    # the rounding is not a no-op on this network: without it the output moves
    y0 = net.forward(params, x, levels)[0]
    assert np.max(np.abs(y0 - y)) > 1e-4 * np.max(np.abs(y))


def test_bf16_hook_is_a_no_op_on_bfloat16_exact_networks():
    """Integer weights, inputs and biases on one level (no pooling) keep
    every activation and gradient a small integer (exact in bfloat16):
    rounded and unrounded runs agree bit for bit, so the hook changes
    nothing but the rounding."""
    levels, c0, s = 1, 2, 4
    rng = np.random.default_rng(7)
    params = [rng.integers(-1, 2, size=p.shape).astype(np.float64)
              for p in net.init_params(0, c0, levels)]
    x = rng.integers(0, 2, size=(1, 1, s, s)).astype(np.float64)
    y_r, cache_r = net.forward(params, x, levels, act_round=net.bf16_round)
    y_u, cache_u = net.forward(params, x, levels)
    assert np.max(np.abs(y_u)) < 128 and np.array_equal(y_r, y_u)
    dy = rng.integers(-2, 3, size=y_u.shape).astype(np.float64)
    g_r = net.backward(params, cache_r, dy, levels)
    g_u = net.backward(params, cache_u, dy, levels)
    for a, b in zip(g_r, g_u):
        assert np.max(np.abs(b)) < 256 and np.array_equal(a, b)
