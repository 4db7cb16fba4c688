"""FP64 CPU oracle of the warm-start network (forward, backward, Adam).

TEST INFRASTRUCTURE ONLY, like dm_oracle: the GPU library never calls it.

The paper notes that the initial guesses of the probe and object may come
from pre-existing results rather than random ones (Section III).  This form
predicts an initial object from the diffraction frames with a small U-Net
style encoder-decoder:

  input   1 x S x S: log1p of the 2x2-binned intensities, divided by 10
  encoder level l = 0..L-1 (C_l = C0 * 2^l channels): two 3x3 convolutions
          (zero padding, stride 1), each followed by ReLU; 2x2 average pooling
          between levels
  decoder level l = L-2..0: nearest-neighbour 2x upsampling, channel concat
          [upsampled, skip of level l], two 3x3 convolutions with ReLU
  head    1x1 convolution C0 -> 2 (real and imaginary part of the patch)
  loss    mean squared error over every output value

Convolution here is cross-correlation: y[co,i,j] = b[co] +
sum_{ci,di,dj} w[co,ci,di,dj] x[ci, i+di-1, j+dj-1] (3x3) or
y[co,i,j] = b[co] + sum_ci w[co,ci,0,0] x[ci,i,j] (1x1).

Parameters are a list [W, b, W, b, ...] in the order enc0a, enc0b, enc1a, ...,
enc(L-1)b, dec(L-2)a, dec(L-2)b, ..., dec0a, dec0b, head.
"""
from __future__ import annotations

import numpy as np


def layer_shapes(c0: int = 32, levels: int = 4, c_in: int = 1, c_out: int = 2):
    """[(cout, cin, k)] of every convolution in parameter order."""
    ch = [c0 * 2 ** l for l in range(levels)]
    shapes = []
    prev = c_in
    for l in range(levels):
        shapes.append((ch[l], prev, 3))
        shapes.append((ch[l], ch[l], 3))
        prev = ch[l]
    for l in range(levels - 2, -1, -1):
        shapes.append((ch[l], ch[l + 1] + ch[l], 3))
        shapes.append((ch[l], ch[l], 3))
    shapes.append((c_out, ch[0], 1))
    return shapes


def n_params(c0: int = 32, levels: int = 4) -> int:
    return sum(co * ci * k * k + co for co, ci, k in layer_shapes(c0, levels))


def init_params(seed: int, c0: int = 32, levels: int = 4):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, seeded."""
    rng = np.random.default_rng(seed)
    params = []
    for co, ci, k in layer_shapes(c0, levels):
        params.append(rng.standard_normal((co, ci, k, k)) * np.sqrt(2.0 / (ci * k * k)))
        params.append(np.zeros(co))
    return params


def flatten(params) -> np.ndarray:
    return np.concatenate([p.ravel() for p in params])


def unflatten(flat, c0: int = 32, levels: int = 4):
    out, o = [], 0
    for co, ci, k in layer_shapes(c0, levels):
        n = co * ci * k * k
        out.append(np.asarray(flat[o:o + n], dtype=np.float64).reshape(co, ci, k, k))
        o += n
        out.append(np.asarray(flat[o:o + co], dtype=np.float64))
        o += co
    return out


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) through float32 bits."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r << 16).astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# building blocks (written out; batch axis first, NCHW)
# ---------------------------------------------------------------------------
def conv3x3(x, w, b):
    n, ci, h, wd = x.shape
    xp = np.zeros((n, ci, h + 2, wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((n, w.shape[0], h, wd))
    for di in range(3):
        for dj in range(3):
            y += np.einsum("oc,nchw->nohw", w[:, :, di, dj], xp[:, :, di:di + h, dj:dj + wd])
    return y + b[None, :, None, None]


def conv3x3_backward(x, w, dy):
    n, ci, h, wd = x.shape
    xp = np.zeros((n, ci, h + 2, wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for di in range(3):
        for dj in range(3):
            dw[:, :, di, dj] = np.einsum("nohw,nchw->oc", dy, xp[:, :, di:di + h, dj:dj + wd])
            dxp[:, :, di:di + h, dj:dj + wd] += np.einsum("oc,nohw->nchw", w[:, :, di, dj], dy)
    return dxp[:, :, 1:-1, 1:-1], dw, dy.sum(axis=(0, 2, 3))


def conv1x1(x, w, b):
    return np.einsum("oc,nchw->nohw", w[:, :, 0, 0], x) + b[None, :, None, None]


def conv1x1_backward(x, w, dy):
    dx = np.einsum("oc,nohw->nchw", w[:, :, 0, 0], dy)
    dw = np.einsum("nohw,nchw->oc", dy, x)[:, :, None, None]
    return dx, dw, dy.sum(axis=(0, 2, 3))


def avgpool2(x):
    n, c, h, w = x.shape
    return x.reshape(n, c, h // 2, 2, w // 2, 2).mean(axis=(3, 5))


def avgpool2_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=2), 2, axis=3) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)


def upsample2_backward(dy):
    n, c, h, w = dy.shape
    return dy.reshape(n, c, h // 2, 2, w // 2, 2).sum(axis=(3, 5))


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------
def _ident(v):
    return v


def forward(params, x, levels: int = 4, act_round=None):
    """Returns (y, cache).  x: [N][1][S][S].

    act_round, if given, is applied to the input of every 3x3 convolution
    (the form in which the matrix cores take bfloat16 activations); the
    cache keeps the rounded inputs, which the backward pass then uses."""
    r = act_round or _ident
    it = iter(range(0, len(params), 2))
    cache = {"enc_in": [], "enc_mid": [], "enc_out": [], "dec_in": [], "dec_mid": [],
             "dec_out": [], "act_round": act_round}
    h = x
    skips = []
    for l in range(levels):
        i = next(it)
        cache["enc_in"].append(r(h))
        a = np.maximum(conv3x3(r(h), params[i], params[i + 1]), 0.0)
        cache["enc_mid"].append(a)
        i = next(it)
        h = np.maximum(conv3x3(r(a), params[i], params[i + 1]), 0.0)
        cache["enc_out"].append(h)
        skips.append(h)
        if l < levels - 1:
            h = avgpool2(h)
    for l in range(levels - 2, -1, -1):
        u = np.concatenate([upsample2(h), skips[l]], axis=1)
        cache["dec_in"].append(r(u))
        i = next(it)
        a = np.maximum(conv3x3(r(u), params[i], params[i + 1]), 0.0)
        cache["dec_mid"].append(a)
        i = next(it)
        h = np.maximum(conv3x3(r(a), params[i], params[i + 1]), 0.0)
        cache["dec_out"].append(h)
    i = next(it)
    cache["head_in"] = h
    y = conv1x1(h, params[i], params[i + 1])
    return y, cache


def backward(params, cache, dy, levels: int = 4):
    """Gradients (list like params) of a loss whose gradient w.r.t. y is dy.
    With the forward pass's act_round, the inputs of every 3x3 convolution
    and the gradients at its output are rounded the same way (the bias
    gradients sum the unrounded output gradients)."""
    r = cache.get("act_round") or _ident

    def back3(x, w, dz):
        # weight and data gradients from the rounded output gradient; the
        # bias gradient sums it unrounded
        dx, dw, _ = conv3x3_backward(x, w, r(dz))
        return dx, dw, dz.sum(axis=(0, 2, 3))

    grads = [None] * len(params)
    i = len(params) - 2
    dh, grads[i], grads[i + 1] = conv1x1_backward(cache["head_in"], params[i], dy)
    dskip = [None] * levels
    for k, l in enumerate(range(0, levels - 1)):
        # decoder levels in reverse order of the forward pass: 0, 1, ..., L-2
        pos = levels - 2 - l            # index in the forward decoder lists
        dh = dh * (cache["dec_out"][pos] > 0)
        i -= 2
        da, grads[i], grads[i + 1] = back3(r(cache["dec_mid"][pos]), params[i], dh)
        da = da * (cache["dec_mid"][pos] > 0)
        i -= 2
        du, grads[i], grads[i + 1] = back3(cache["dec_in"][pos], params[i], da)
        c_up = du.shape[1] - cache["enc_out"][l].shape[1]
        dskip[l] = du[:, c_up:]
        dh = upsample2_backward(du[:, :c_up])
    for l in range(levels - 1, -1, -1):
        if l < levels - 1:
            dh = avgpool2_backward(dh) + dskip[l]
        dh = dh * (cache["enc_out"][l] > 0)
        i -= 2
        da, grads[i], grads[i + 1] = back3(r(cache["enc_mid"][l]), params[i], dh)
        da = da * (cache["enc_mid"][l] > 0)
        i -= 2
        dh, grads[i], grads[i + 1] = back3(cache["enc_in"][l], params[i], da)
    return grads


def mse(y, target):
    return float(np.mean((y - target) ** 2)), 2.0 * (y - target) / y.size


def loss_and_grads(params, x, target, levels: int = 4, act_round=None):
    y, cache = forward(params, x, levels, act_round)
    loss, dy = mse(y, target)
    return loss, backward(params, cache, dy, levels), y


# ---------------------------------------------------------------------------
# input and output maps between frames and the network
# ---------------------------------------------------------------------------
def preprocess(I):
    """x[n][0] = log1p(2x2 block sums of max(I, 0)) / 10, with the block
    image rolled by S/2 = F/4 along both axes so that the block holding the
    zero frequency (pixel [0][0] of the unshifted DFT) sits at [S/2][S/2];
    I: [N][F][F]."""
    I = np.maximum(np.asarray(I, dtype=np.float64), 0.0)
    n, f, _ = I.shape
    s = I.reshape(n, f // 2, 2, f // 2, 2).sum(axis=(2, 4))
    s = np.roll(s, (f // 4, f // 4), axis=(1, 2))
    return (np.log1p(s) / 10.0)[:, None]


def patches(y):
    """Complex patches [N][2S][2S] from y [N][2][S][S] (real, imaginary) by
    bilinear 2x upsampling: output pixel u samples the input at u/2 - 1/4
    (pixel centres), clamped to [0, S-1]."""
    y = np.asarray(y, dtype=np.float64)
    n, _, s, _ = y.shape
    c = np.clip(np.arange(2 * s) / 2.0 - 0.25, 0.0, s - 1.0)
    i0 = np.floor(c).astype(int)
    i1 = np.minimum(i0 + 1, s - 1)
    f = c - i0
    z = y[:, 0] + 1j * y[:, 1]
    rows = z[:, i0, :] * (1 - f)[None, :, None] + z[:, i1, :] * f[None, :, None]
    return rows[:, :, i0] * (1 - f)[None, None, :] + rows[:, :, i1] * f[None, None, :]


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), step t >= 1; returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mh = mm / (1 - b1 ** t)
        vh = vv / (1 - b2 ** t)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v
