"""CPU emulation of the BF16x3 precision form of the DM view update.

TEST INFRASTRUCTURE ONLY, like dm_oracle: the GPU library never calls it.

The 2-D DFT of a frame is computed as two dense complex matrix products with
the DFT matrix W (W[a][b] = exp(-2 pi i ab / F), symmetric): T = Z W along
rows, then W T along columns; the inverse uses conj(W).  Every real product
a*b inside those matrix products is replaced by the three-term split
product

    x32 = float32(x),  hi(x) = bf16(x32),  lo(x) = bf16(x32 - hi(x))
    a*b ~ hi(a) hi(b) + hi(a) lo(b) + lo(a) hi(b)

(the lo*lo term is dropped) and summed exactly here (float64; the GPU sums
in float32 on its matrix units).  Each matrix product's result is rounded to
float32, as the GPU stores it.  The complex products use the four real
products Re = Ar Br - Ai Bi, Im = Ar Bi + Ai Br.  W enters as float64 ->
float32 -> split.  The 1/F^2 of the inverse and the modulus scale
sqrt(I / sum_k |.|^2) are applied together to the spectrum, in float64,
before the result is rounded to float32 and split for the inverse
products.

Everything else of the iteration (exit waves, the modulus projection, the
object and probe updates of Eqs. 4-5, the error norms of Eq. 6) is
dm_oracle's float64 arithmetic; this module only swaps the transforms.
"""
from __future__ import annotations

import numpy as np

from . import dm_oracle as dm
from .cnn_oracle import bf16_round


def split(x):
    """(hi, lo) bfloat16 pieces (as float64) of float32(x); x real."""
    x32 = np.asarray(x, dtype=np.float32).astype(np.float64)
    hi = bf16_round(x32)
    lo = bf16_round((x32 - hi).astype(np.float32))
    return hi, lo


def rmatmul3(A, B):
    """Three-term split product of real matrices, summed exactly (float64)."""
    ah, al = split(A)
    bh, bl = split(B)
    return ah @ bh + ah @ bl + al @ bh


def cmatmul3(A, B):
    """Complex product from four split real products, rounded to complex64."""
    A = np.asarray(A, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    re = rmatmul3(A.real, B.real) - rmatmul3(A.imag, B.imag)
    im = rmatmul3(A.real, B.imag) + rmatmul3(A.imag, B.real)
    return (re + 1j * im).astype(np.complex64).astype(np.complex128)


def dft_matrix(f: int, sign: int = -1) -> np.ndarray:
    """W[a][b] = exp(sign * 2 pi i ab / f) in float64, rounded to complex64."""
    a = np.arange(f)
    w = np.exp(sign * 2j * np.pi * np.outer(a, a) / f)
    return w.astype(np.complex64).astype(np.complex128)


def dft2(z):
    """Forward 2-D DFT of each [F][F] frame of z (any leading axes)."""
    z = np.asarray(z, dtype=np.complex128)
    f = z.shape[-1]
    W = dft_matrix(f, -1)
    flat = z.reshape(-1, f, f)
    out = np.empty_like(flat)
    for i, fr in enumerate(flat):
        out[i] = cmatmul3(W, cmatmul3(fr, W))
    return out.reshape(z.shape)


def idft2_unscaled(u):
    """conj(W) u conj(W) per frame, no 1/F^2 (the caller folds it in)."""
    u = np.asarray(u, dtype=np.complex128)
    f = u.shape[-1]
    Wc = dft_matrix(f, +1)
    flat = u.reshape(-1, f, f)
    out = np.empty_like(flat)
    for i, fr in enumerate(flat):
        out[i] = cmatmul3(cmatmul3(Wc, fr), Wc)
    return out.reshape(u.shape)


def view_update(psi, P, O, pos, I, beta):
    """Eq. 3 with the split-product transforms; float64 elsewhere."""
    psi = np.asarray(psi, dtype=np.complex128)
    f = psi.shape[-1]
    phi = dm.exit_waves(P, O, pos)
    z = 2.0 * phi - psi
    spec = dft2(z)
    # modulus projection with the inverse's 1/F^2 folded into the scale
    proj = dm.constrained_ft(spec, I) / float(f * f)
    proj = proj.astype(np.complex64).astype(np.complex128)
    return psi + beta * (idft2_unscaled(proj) - phi)


def iterate(psi, P, O, pos, I, beta):
    """One DM iteration in dm_oracle's order with the split-product views."""
    psi_new = view_update(psi, P, O, pos, I, beta)
    O_new, _ = dm.object_update(psi_new, P, O, pos)
    P_new, _ = dm.probe_update(psi_new, O_new, P, pos)
    return psi_new, P_new, O_new
