"""Pins of the BF16x3 emulation (CPU only): the split's exactness bound, exact
products of bfloat16-representable matrices, the proven per-output error
bound of the split DFT, exact special cases, and closeness of one emulated
DM step to the float64 one."""
import numpy as np

from oracle import bf16x3_oracle as b3
from oracle import dm_oracle as dm
from paper_1808_10375_amd import synth


def test_split_pieces_are_bf16_and_reconstruct_within_2_to_minus_16():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(10000) * 10.0 ** rng.uniform(-6, 6, 10000)
    hi, lo = b3.split(x)
    for piece in (hi, lo):
        bits = piece.astype(np.float32).view(np.uint32)
        assert np.all((bits & 0xFFFF) == 0)
    x32 = x.astype(np.float32).astype(np.float64)
    assert np.all(np.abs(x32 - (hi + lo)) <= 2.0 ** -16 * np.abs(x32))
    # a value that is already bfloat16 has no low piece
    hi2, lo2 = b3.split(hi)
    assert np.array_equal(hi2, hi) and np.all(lo2 == 0.0)


def test_products_of_bf16_matrices_are_exact():
    rng = np.random.default_rng(1)
    A = b3.split(rng.standard_normal((7, 9)))[0]
    B = b3.split(rng.standard_normal((9, 5)))[0]
    assert np.array_equal(b3.rmatmul3(A, B), A @ B)


def test_split_dft_within_the_proven_bound():
    # per real product |ab - (hh + hl + lh)| <= 3 * 2^-16 |a||b| (+ rounding of
    # the float32 inputs), so each output of a 1-D complex DFT is off by at
    # most about 4 * 3 * 2^-16 * sum_k |z_k| (four real products per complex
    # product, |Re W|, |Im W| <= 1); the float32 results add 2^-24 relative
    rng = np.random.default_rng(2)
    f = 32
    z = (rng.standard_normal((f, f)) + 1j * rng.standard_normal((f, f)))
    W = b3.dft_matrix(f)
    got = b3.cmatmul3(z, W)
    exact = z @ np.exp(-2j * np.pi * np.outer(np.arange(f), np.arange(f)) / f)
    bound = 4 * 3 * 2.0 ** -16 * np.sum(np.abs(z), axis=1, keepdims=True) + 1e-6
    assert np.all(np.abs(got - exact) <= bound)
    # the emulation is not secretly exact: split errors are visible
    assert np.max(np.abs(got - exact)) > 1e-8


def test_split_dft_exact_special_cases():
    f = 16
    delta = np.zeros((f, f), complex)
    delta[0, 0] = 1.0
    assert np.array_equal(b3.dft2(delta), np.ones((f, f)))   # row/col 0 of W are 1
    ones = np.ones((f, f), complex)
    out = b3.dft2(ones)
    assert out[0, 0] == f * f
    assert np.max(np.abs(out.ravel()[1:])) <= 4 * 3 * 2.0 ** -16 * f * f


def test_emulated_step_close_to_float64_step():
    c = synth.random_case(3, n_frames=6, frame=16, n_modes=2, obj_h=40, obj_w=36,
                          perturb=0.3)
    args = (c["psi"], c["P"], c["O"], c["pos"], c["I"], c["beta"])
    psi_e, P_e, O_e = b3.iterate(*args)
    psi_x, P_x, O_x, _ = dm.iterate(*args)

    def rel(a, b):
        return np.linalg.norm(a - b) / np.linalg.norm(b)
    for a, b in ((psi_e, psi_x), (P_e, P_x)):
        r = rel(a, b)
        assert 1e-9 < r < 1e-4, r
