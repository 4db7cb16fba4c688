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
