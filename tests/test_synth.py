"""Checks of the seeded scan generator (shapes, ranges, recipes).  CPU only."""
import numpy as np
import pytest

from paper_1808_10375_amd import synth


def test_grf_object_ranges():
    r = synth.streams(0)
    O = synth.grf_object(128, 128, r[0], r[1])
    ph = np.angle(O)
    assert abs(ph.min() + 1.0) < 1e-12 and abs(ph.max() - 1.0) < 1e-12
    a = np.abs(O)
    assert a.min() >= 0.8 and a.max() < 1.0


def test_hermite_gauss_modes_orthogonal_with_weights():
    w = [1.0, 0.5, 0.25, 0.12, 0.06]
    P = synth.hermite_gauss_modes(128, 16.0, synth.HG_ORDERS[:5], w)
    g = np.einsum("aij,bij->ab", P.conj(), P)
    nrm = np.sqrt(np.real(np.diag(g)))
    off = np.abs(g) / np.outer(nrm, nrm) - np.eye(5)
    assert np.max(np.abs(off)) < 1e-8
    assert np.allclose(np.real(np.diag(g)), w, rtol=1e-12)


def test_single_mode_raster_shapes_and_bounds():
    s = synth.single_mode_raster_32(0)
    assert s.I.shape == (100, 32, 32) and s.I.dtype == np.float32
    assert s.P0.shape == (1, 32, 32) and s.O0.shape == (128, 128)
    assert s.pos.min() >= 0 and s.pos.max() <= 128 - 32
    # noise-free: intensities are exactly |FFT(P O)|^2 of the true fields
    assert np.all(s.I >= 0)
    # deterministic
    assert np.array_equal(synth.single_mode_raster_32(0).I, s.I)


def test_fermat_spiral_step_and_bounds():
    pos = synth.fermat_positions(2500, 5.88, (512, 512), 128)
    assert pos.min() >= 0 and pos.max() <= 1024 - 128
    d = np.sqrt(((pos[:, None, :] - pos[None, :, :]) ** 2).sum(-1).astype(float))
    np.fill_diagonal(d, np.inf)
    nn = d.min(axis=1)
    assert 8.5 < nn.mean() < 11.5


def test_poisson_budget_small_spiral():
    s = synth.spiral_scan(7, 200, 3, [1.0, 0.5, 0.25], photons=1e5)
    assert s.I.shape == (200, 128, 128)
    mean = float(np.mean(np.sum(s.I.astype(np.float64), axis=(1, 2))))
    assert abs(mean / 1e5 - 1.0) < 0.01
    assert np.all(s.I == np.round(s.I))
    # Parseval-scaled cold start
    tot = 128 * 128 * float(np.sum(np.abs(s.P0.astype(np.complex128)) ** 2))
    assert abs(tot / mean - 1.0) < 1e-5


def test_uneven_scan_sizes_in_range():
    sizes = synth.uneven_scan_sizes()
    assert len(sizes) == 16 and min(sizes) >= 200 and max(sizes) <= 3000


def test_flyscan_strip_positions_in_bounds():
    full = synth.raster_positions(100, 100, 12.0, 814.0)
    assert full.min() >= 0 and full.max() <= 3072 - 256
