"""Seeded synthetic ptychography scans.

This module only *simulates measurements*: objects, probes, scan positions and
far-field intensities built from them.  It holds none of the reconstruction's
arithmetic (no projection, no update, no error norm) and is the one module that
both the FP64 CPU oracle's tests and the GPU path's tests and benchmark import,
so both sides always receive bit-identical inputs.

Forward model: the recorded intensity of view j is the incoherent sum over
probe modes of the squared modulus of the far-field transform of the exit wave
P_m * O_window_j (Section II, Eqs. 1-2 of the paper).  The transform here is
numpy's unnormalised forward FFT with exp(-2*pi*i*k*n/F), detector DC at [0,0]
(no fftshift); the reconstruction must use the same convention.

Workload shapes follow the paper's cases, restated as synthetic scans:
  single_mode_raster_32   single mode, 32x32 frames, 10x10 jittered raster, 128x128 object,
            noise-free
  multimode_spiral_128    5 Hermite-Gaussian modes, 128x128 frames, 2500-point Fermat spiral,
            1024x1024 object, Poisson noise at 1e5 photons per frame
  flyscan_raster_256      fly scan: 256x256 frames, 100x100 raster, 3072x3072 object, 8
            sub-positions of motion blur, Poisson noise at 1e6 photons/frame,
            reconstructed with 8 modes (Section II: fly-scan blur read as
            incoherent illumination)
  flyscan_raster_188      the paper's frame size: 188x188 frames, 100x100 raster, 1280x1280
            object, 8 sub-positions of motion blur, 1e6 photons/frame, 4 modes
  weak_scaling_200        the per-node shape of the paper's weak scaling: 200x200 frames,
            71x71 raster (5041 points), 1000x1000 object, zone-plate probe, single mode
  uneven_spirals_128      16 scans of 200-3000 frames, 3 modes, 128x128 frames, 1024^2 objects
The paper measured real beamline data that is not available; these seeded
scans stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import os

import numpy as np

try:  # multi-threaded FFT for generating large scans; numpy's as a fallback
    import scipy.fft as _sfft

    def _fft2(a):
        return _sfft.fft2(a, axes=(-2, -1), workers=-1)

    def _ifft2(a):
        return _sfft.ifft2(a, axes=(-2, -1), workers=-1)
except Exception:  # pragma: no cover
    def _fft2(a):
        return np.fft.fft2(a, axes=(-2, -1))

    def _ifft2(a):
        return np.fft.ifft2(a, axes=(-2, -1))


GOLDEN_ANGLE_DEG = 137.508


@dataclass
class Scan:
    """One synthetic scan, in the layouts the library takes.

    I      float32 [N][F][F]  measured intensities, DC at [0, 0]
    pos    int32   [N][2]     (y, x) top-left corner of each view's window
    P0     complex64 [M][F][F] initial probe modes (cold start)
    O0     complex64 [H][W]    initial object (cold start)
    P_true / O_true            the fields the data was simulated from
    """
    I: np.ndarray
    pos: np.ndarray
    P0: np.ndarray
    O0: np.ndarray
    beta: float = 0.8
    P_true: Optional[np.ndarray] = None
    O_true: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_frames(self):
        return int(self.I.shape[0])

    @property
    def frame(self):
        return int(self.I.shape[1])

    @property
    def n_modes(self):
        return int(self.P0.shape[0])

    @property
    def obj_shape(self):
        return tuple(int(s) for s in self.O0.shape)

    def subset(self, views) -> "Scan":
        """The same scan restricted to the listed views (in that order); the
        initial guesses, object size and ground truth are kept."""
        idx = np.asarray(views, dtype=np.int64)
        return Scan(np.ascontiguousarray(self.I[idx]), np.ascontiguousarray(self.pos[idx]),
                    self.P0, self.O0, self.beta, self.P_true, self.O_true,
                    f"{self.name}[{len(idx)} views]", dict(self.meta))


# --------------------------------------------------------------------------
# random streams
# --------------------------------------------------------------------------
def streams(seed: int, n: int = 8):
    """Independent PCG64 generators spawned from one seed."""
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


# --------------------------------------------------------------------------
# objects
# --------------------------------------------------------------------------
def grf_object(h: int, w: int, rng_amp, rng_phase, sigma: float = 4.0,
               phase_range: float = 1.0, amp_lo: float = 0.8,
               amp_hi: float = 1.0) -> np.ndarray:
    """Complex object: iid U(amp_lo, amp_hi) amplitude and a Gaussian random
    field phase (white N(0,1) noise, periodic Gaussian filter of std `sigma`
    px, affinely mapped onto exactly [-phase_range, +phase_range] rad)."""
    amp = rng_amp.uniform(amp_lo, amp_hi, size=(h, w))
    white = rng_phase.standard_normal((h, w))
    fy = np.fft.fftfreq(h)[:, None]
    fx = np.fft.fftfreq(w)[None, :]
    transfer = np.exp(-2.0 * math.pi ** 2 * sigma ** 2 * (fy ** 2 + fx ** 2))
    field_ = np.real(_ifft2(_fft2(white) * transfer))
    lo, hi = field_.min(), field_.max()
    phase = -phase_range + 2.0 * phase_range * (field_ - lo) / (hi - lo)
    return (amp * np.exp(1j * phase)).astype(np.complex128)


# --------------------------------------------------------------------------
# probes
# --------------------------------------------------------------------------
def _centred_grid(f: int):
    c = (f - 1) / 2.0
    y, x = np.mgrid[0:f, 0:f].astype(np.float64)
    return y - c, x - c


def quadratic_phase(f: int, alpha: Optional[float] = None) -> np.ndarray:
    """exp(i*alpha*r^2) about the frame centre; alpha = pi/(F/2)^2 by default
    (a phase of pi at the frame edge)."""
    if alpha is None:
        alpha = math.pi / (f / 2.0) ** 2
    y, x = _centred_grid(f)
    return np.exp(1j * alpha * (x * x + y * y))


def gaussian_probe(f: int, sigma: float, alpha: Optional[float] = None):
    y, x = _centred_grid(f)
    amp = np.exp(-(x * x + y * y) / (2.0 * sigma * sigma))
    return amp * quadratic_phase(f, alpha)


def _hermite(n: int, t: np.ndarray) -> np.ndarray:
    """Physicists' Hermite polynomial H_n by its three-term recurrence."""
    h0 = np.ones_like(t)
    if n == 0:
        return h0
    h1 = 2.0 * t
    for k in range(1, n):
        h0, h1 = h1, 2.0 * t * h1 - 2.0 * k * h0
    return h1


def hermite_gauss_modes(f: int, waist: float, orders, weights,
                        alpha: Optional[float] = None) -> np.ndarray:
    """Orthogonal Hermite-Gaussian probe modes HG_{n,m} (n along x, m along
    y), Gram-Schmidt orthonormalised on the pixel grid, then scaled so that
    mode k carries intensity fraction weights[k] / weights[0] of mode 0."""
    y, x = _centred_grid(f)
    g = np.exp(-(x * x + y * y) / (waist * waist))
    raw = [(_hermite(n, math.sqrt(2.0) * x / waist)
            * _hermite(m, math.sqrt(2.0) * y / waist) * g).astype(np.complex128)
           for (n, m) in orders]
    basis = []
    for v in raw:
        for b in basis:
            v = v - np.vdot(b, v) * b
        v = v / np.linalg.norm(v)
        basis.append(v)
    qp = quadratic_phase(f, alpha)
    modes = np.stack([math.sqrt(wt) * b * qp for b, wt in zip(basis, weights)])
    return modes


def subpixel_shift(p: np.ndarray, dy: float, dx: float) -> np.ndarray:
    """Shift a frame by a (sub)pixel amount with a Fourier phase ramp."""
    f0, f1 = p.shape[-2:]
    ky = np.fft.fftfreq(f0)[:, None]
    kx = np.fft.fftfreq(f1)[None, :]
    ramp = np.exp(-2j * math.pi * (ky * dy + kx * dx))
    return _ifft2(_fft2(p) * ramp)


# --------------------------------------------------------------------------
# scan positions (integer top-left corners, rounded with floor(x + 0.5))
# --------------------------------------------------------------------------
def _round(v):
    return np.floor(np.asarray(v, dtype=np.float64) + 0.5).astype(np.int64)


def raster_positions(ny: int, nx: int, step: float, origin: float,
                     jitter: float = 0.0, rng=None) -> np.ndarray:
    iy, ix = np.mgrid[0:ny, 0:nx]
    y = origin + step * iy.ravel().astype(np.float64)
    x = origin + step * ix.ravel().astype(np.float64)
    if jitter > 0:
        y = y + rng.uniform(-jitter, jitter, size=y.shape)
        x = x + rng.uniform(-jitter, jitter, size=x.shape)
    return np.stack([_round(y), _round(x)], axis=1).astype(np.int32)


def fermat_positions(n: int, c: float, centre_yx, frame: int) -> np.ndarray:
    """Fermat spiral of probe centres r = c*sqrt(k), theta = k*golden angle,
    converted to the top-left corners of frame x frame windows."""
    k = np.arange(n, dtype=np.float64)
    r = c * np.sqrt(k)
    th = np.deg2rad(GOLDEN_ANGLE_DEG) * k
    cy = centre_yx[0] + r * np.sin(th) - frame / 2.0
    cx = centre_yx[1] + r * np.cos(th) - frame / 2.0
    return np.stack([_round(cy), _round(cx)], axis=1).astype(np.int32)


# --------------------------------------------------------------------------
# measurements
# --------------------------------------------------------------------------
def _windows(obj: np.ndarray, pos: np.ndarray, f: int) -> np.ndarray:
    return np.stack([obj[y:y + f, x:x + f] for (y, x) in pos])


def far_field_intensity(probes: np.ndarray, obj: np.ndarray, pos: np.ndarray,
                        chunk: int = 256) -> np.ndarray:
    """I_j = sum_m |FFT2(P_m * O_window_j)|^2 (float64), computed in chunks;
    with object modes obj [L][H][W], the sum also runs over l (Eq. 1)."""
    if obj.ndim == 3:
        return sum(far_field_intensity(probes, o, pos, chunk) for o in obj)
    f = probes.shape[-1]
    out = np.empty((len(pos), f, f), dtype=np.float64)

    def one(s):
        w = _windows(obj, pos[s:s + chunk], f)            # [c][F][F]
        ex = probes[None, :, :, :] * w[:, None, :, :]     # [c][M][F][F]
        out[s:s + chunk] = np.sum(np.abs(_fft2(ex)) ** 2, axis=1)

    starts = range(0, len(pos), chunk)
    if len(starts) < 4:
        for s in starts:
            one(s)
    else:
        # chunks are independent (each writes its own rows), so threads give
        # the same array; numpy's FFT releases the interpreter lock
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex_pool:
            list(ex_pool.map(one, starts))
    return out


def poisson_counts(intensity: np.ndarray, photons_per_frame: float, rng):
    """One global scale so the mean expected count per frame equals
    `photons_per_frame`, then Poisson sampling (float32 counts)."""
    scale = photons_per_frame / float(np.mean(np.sum(intensity, axis=(1, 2))))
    counts = rng.poisson(intensity * scale)
    return counts.astype(np.float32), scale


def cold_start(f: int, n_modes: int, mean_frame_sum: float, rng,
               envelope: np.ndarray, mode_weights, obj_shape) -> tuple:
    """Cold-start guesses.  O0 = 1 + 0i.  Mode 0 is the config's Gaussian
    amplitude envelope with flat phase; mode k >= 1 is that envelope blurred by
    a Gaussian of std k px times a random phase screen U(-0.1, 0.1) rad
    (differently blurred modes, as the paper suggests in Section III).  The
    modes are scaled to the weights and jointly to the measured total
    intensity (F^2 * sum_k ||P_k||^2 = mean_j sum_q I_j, by Parseval)."""
    modes = []
    for k in range(n_modes):
        if k == 0:
            m = envelope.astype(np.complex128)
        else:
            fy = np.fft.fftfreq(f)[:, None]
            fx = np.fft.fftfreq(f)[None, :]
            blur = np.exp(-2.0 * math.pi ** 2 * k * k * (fy ** 2 + fx ** 2))
            m = np.real(_ifft2(_fft2(envelope) * blur)).astype(np.complex128)
            m = m * np.exp(1j * rng.uniform(-0.1, 0.1, size=(f, f)))
        m = m / np.linalg.norm(m) * math.sqrt(mode_weights[k])
        modes.append(m)
    P0 = np.stack(modes)
    total = f * f * float(np.sum(np.abs(P0) ** 2))
    P0 = P0 * math.sqrt(mean_frame_sum / total)
    O0 = np.ones(obj_shape, dtype=np.complex128)
    return P0.astype(np.complex64), O0.astype(np.complex64)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------
def single_mode_raster_32(seed: int = 0) -> Scan:
    """Single mode, 32x32 frames, 10x10 raster (step 8 px, origin 12 px,
    U(-1,1) px jitter), 128x128 object, noise-free intensities."""
    r = streams(seed)
    f, h = 32, 128
    O = grf_object(h, h, r[0], r[1])
    P = gaussian_probe(f, 6.0)[None]
    pos = raster_positions(10, 10, 8.0, 12.0, jitter=1.0, rng=r[2])
    I = far_field_intensity(P, O, pos).astype(np.float32)
    y, x = _centred_grid(f)
    env = np.exp(-(x * x + y * y) / (2 * 36.0))
    P0, O0 = cold_start(f, 1, float(np.mean(np.sum(I, axis=(1, 2)))), r[3],
                        env, [1.0], (h, h))
    return Scan(I, pos, P0, O0, 0.8, P.astype(np.complex64),
                O.astype(np.complex64), "single_mode_raster_32")


HG_ORDERS = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1)]


def spiral_scan(seed: int, n_frames: int, n_modes: int, weights,
                frame: int = 128, obj: int = 1024, photons: float = 1e5,
                c: float = 5.88, name: str = "") -> Scan:
    """Multi-mode Hermite-Gaussian probe (waist F/8, quadratic phase
    pi/(F/2)^2), Fermat-spiral scan of mean step ~10 px centred in the object,
    Poisson counts at `photons` per frame."""
    r = streams(seed)
    O = grf_object(obj, obj, r[0], r[1])
    waist = frame / 8.0
    P = hermite_gauss_modes(frame, waist, HG_ORDERS[:n_modes], weights)
    pos = fermat_positions(n_frames, c, (obj / 2.0, obj / 2.0), frame)
    I_exact = far_field_intensity(P, O, pos)
    I, _ = poisson_counts(I_exact, photons, r[2])
    y, x = _centred_grid(frame)
    env = np.exp(-(x * x + y * y) / (waist * waist))
    P0, O0 = cold_start(frame, n_modes, float(np.mean(np.sum(I, axis=(1, 2)))),
                        r[3], env, weights, (obj, obj))
    return Scan(I, pos, P0, O0, 0.8, P.astype(np.complex64),
                O.astype(np.complex64), name)


def multimode_spiral_128(seed: int = 1, n_frames: int = 2500) -> Scan:
    """5 HG modes (weights 1, .5, .25, .12, .06), 128x128 frames, 2500-point
    Fermat spiral (mean step 10 px), 1024x1024 object, 1e5 photons/frame."""
    return spiral_scan(seed, n_frames, 5, [1.0, 0.5, 0.25, 0.12, 0.06],
                       name="multimode_spiral_128")


def flyscan_raster_256(seed: int = 2, n_frames: int = 10000, n_modes: int = 8,
            obj: int = 3072, sub_positions: int = 8) -> Scan:
    """Fly scan: 256x256 frames on a 100x100 raster (step 12 px, origin
    814 px), 3072x3072 object, HG00 source probe (waist 32 px, quadratic
    phase pi/128^2), motion blur from `sub_positions` sub-positions along x at
    offsets (s - 3.5) * 1.5 px summed incoherently, 1e6 photons/frame,
    reconstructed with `n_modes` modes.  `n_frames` < 10000 takes the first
    rows of the raster (a strip of the same scan)."""
    r = streams(seed)
    f = 256
    O = grf_object(obj, obj, r[0], r[1])
    src = hermite_gauss_modes(f, 32.0, [(0, 0)], [1.0])[0]
    origin = 814.0 * obj / 3072.0 if obj != 3072 else 814.0
    full = raster_positions(100, 100, 12.0, origin)
    pos = full[:n_frames]
    shifts = [(s - (sub_positions - 1) / 2.0) * 1.5 for s in range(sub_positions)]
    probes = np.stack([subpixel_shift(src, 0.0, dx) for dx in shifts])
    I_exact = far_field_intensity(probes, O, pos, chunk=64)
    I, _ = poisson_counts(I_exact, 1e6, r[2])
    y, x = _centred_grid(f)
    env = np.exp(-(x * x + y * y) / (32.0 * 32.0))
    weights = [1.0 / (k + 1) for k in range(n_modes)]
    P0, O0 = cold_start(f, n_modes, float(np.mean(np.sum(I, axis=(1, 2)))),
                        r[3], env, weights, (obj, obj))
    return Scan(I, pos, P0, O0, 0.8, probes.astype(np.complex64),
                O.astype(np.complex64), "flyscan_raster_256")


def flyscan_raster_188(seed: int = 3, n_frames: int = 10000, n_modes: int = 4,
                       obj: int = 1280, sub_positions: int = 8) -> Scan:
    """Fly scan at the paper's own frame size (188 = 4 x 47; its measured
    gold nano-crystal scan has 10000 such frames): 188x188 frames on a
    100x100 raster (step 9 px, origin 100 px), 1280x1280 object, HG00 source
    probe (waist 23.5 px = F/8, quadratic phase pi/94^2), motion blur from
    `sub_positions` sub-positions along x at offsets (s - 3.5) * 1.1 px summed
    incoherently, 1e6 photons/frame, reconstructed with `n_modes` modes.
    `n_frames` < 10000 takes the first rows of the raster."""
    r = streams(seed)
    f = 188
    O = grf_object(obj, obj, r[0], r[1])
    src = hermite_gauss_modes(f, f / 8.0, [(0, 0)], [1.0])[0]
    full = raster_positions(100, 100, 9.0, 100.0)
    pos = full[:n_frames]
    shifts = [(s - (sub_positions - 1) / 2.0) * 1.1 for s in range(sub_positions)]
    probes = np.stack([subpixel_shift(src, 0.0, dx) for dx in shifts])
    I_exact = far_field_intensity(probes, O, pos, chunk=64)
    I, _ = poisson_counts(I_exact, 1e6, r[2])
    y, x = _centred_grid(f)
    env = np.exp(-(x * x + y * y) / (f / 8.0) ** 2)
    weights = [1.0 / (k + 1) for k in range(n_modes)]
    P0, O0 = cold_start(f, n_modes, float(np.mean(np.sum(I, axis=(1, 2)))),
                        r[3], env, weights, (obj, obj))
    return Scan(I, pos, P0, O0, 0.8, probes.astype(np.complex64),
                O.astype(np.complex64), "flyscan_raster_188")


def zone_plate_probe(f: int, r_in: float, r_out: float, defocus: float) -> np.ndarray:
    """Probe behind a zone plate with a central stop: an annular pupil
    r_in <= |k| / (F/2) <= r_out with a defocus phase defocus * (|k| / (F/2))^2
    rad, propagated to the sample plane by an inverse FFT and centred in the
    frame; unit L2 norm."""
    ky = np.fft.fftfreq(f)[:, None] * 2.0
    kx = np.fft.fftfreq(f)[None, :] * 2.0
    r = np.sqrt(ky * ky + kx * kx)
    pupil = ((r >= r_in) & (r <= r_out)).astype(np.complex128)
    pupil *= np.exp(1j * defocus * r * r)
    p = np.fft.fftshift(np.fft.ifft2(pupil))
    return p / np.linalg.norm(p)


def weak_scaling_200(seed: int = 4, side: int = 71, obj: int = 1000) -> Scan:
    """The per-node shape of the paper's weak-scaling runs (Section IV:
    synthesized single-mode data, 200x200 diffraction patterns through a
    zone plate, about 5000 points per node): 200x200 frames, a side x side
    raster (71 x 71 = 5041 points, step 10 px, centred), obj x obj object
    (amplitude and phase from two independent random fields), zone-plate
    probe (annular pupil 0.1..0.6 of the detector half-width, defocus 60 rad
    at its edge: an RMS spot radius of 18 px against the 10 px step),
    Poisson 1e6 photons/frame, single-mode reconstruction from a Gaussian
    cold start."""
    r = streams(seed)
    f = 200
    O = grf_object(obj, obj, r[0], r[1])
    P = zone_plate_probe(f, 0.1, 0.6, 60.0)[None]
    origin = (obj - f - 10.0 * (side - 1)) / 2.0
    pos = raster_positions(side, side, 10.0, origin)
    I_exact = far_field_intensity(P, O, pos, chunk=128)
    I, _ = poisson_counts(I_exact, 1e6, r[2])
    y, x = _centred_grid(f)
    env = np.exp(-(x * x + y * y) / (2.0 * 18.0 ** 2))
    P0, O0 = cold_start(f, 1, float(np.mean(np.sum(I, axis=(1, 2)))), r[3], env, [1.0],
                        (obj, obj))
    return Scan(I, pos, P0, O0, 0.8, P.astype(np.complex64), O.astype(np.complex64),
                "weak_scaling_200")


def uneven_scan_sizes(seed: int = 1000, n_scans: int = 16, lo: int = 200,
                  hi: int = 3000):
    rng = streams(seed, 1)[0]
    return [int(v) for v in rng.integers(lo, hi + 1, size=n_scans)]


def uneven_spirals_128(seed: int = 1000, n_scans: int = 16, sizes=None):
    """16 scans of uneven size N_s ~ U{200..3000}, 3 HG modes (weights 1,
    .5, .25), 128x128 frames, 1024^2 objects, Fermat spirals, 1e5 photons."""
    if sizes is None:
        sizes = uneven_scan_sizes(seed, n_scans)
    return [spiral_scan(seed + 1 + s, n, 3, [1.0, 0.5, 0.25],
                        name=f"uneven_spirals_128.scan{s}") for s, n in enumerate(sizes)]


# --------------------------------------------------------------------------
# small generic cases for tests
# --------------------------------------------------------------------------
def random_case(seed: int, n_frames: int, frame: int, n_modes: int,
                obj_h: int, obj_w: int, consistent: bool = False,
                beta: float = 0.8, perturb: Optional[float] = None,
                n_obj_modes: int = 1) -> dict:
    """A small random state (psi, P, O) with random positions and positive
    intensities.  With consistent=True the intensities and psi are exactly
    those of (P, O), i.e. a fixed point of the reconstruction.  With
    `perturb`, psi is the exit wave of (P, O) plus complex Gaussian noise of
    that relative size (a state near the physical one, whose overlap
    updates are well conditioned).  With n_obj_modes = L > 1 the object is
    [L][H][W] (mode l scaled by 0.6^l) and psi [N][L M][F][F], frame l M + k
    holding the pair (probe mode k, object mode l)."""
    if n_obj_modes > 1:
        return _random_case_obj_modes(seed, n_frames, frame, n_modes, obj_h, obj_w,
                                      consistent, beta, perturb, n_obj_modes)
    r = streams(seed)
    P = (r[0].standard_normal((n_modes, frame, frame))
         + 1j * r[0].standard_normal((n_modes, frame, frame)))
    O = grf_object(obj_h, obj_w, r[1], r[2], sigma=1.5)
    ys = r[3].integers(0, obj_h - frame + 1, size=n_frames)
    xs = r[3].integers(0, obj_w - frame + 1, size=n_frames)
    pos = np.stack([ys, xs], axis=1).astype(np.int32)
    P = P.astype(np.complex64).astype(np.complex128)
    O = O.astype(np.complex64).astype(np.complex128)
    if consistent:
        psi = P[None] * _windows(O, pos, frame)[:, None]
        I = far_field_intensity(P, O, pos)
    elif perturb is not None:
        ex = P[None] * _windows(O, pos, frame)[:, None]
        noise = (r[4].standard_normal(ex.shape) + 1j * r[4].standard_normal(ex.shape))
        psi = ex + perturb * np.abs(ex) * noise
        I = far_field_intensity(P, O, pos) * r[5].uniform(
            0.5, 1.5, size=(n_frames, frame, frame))
    else:
        psi = (r[4].standard_normal((n_frames, n_modes, frame, frame))
               + 1j * r[4].standard_normal((n_frames, n_modes, frame, frame)))
        I = far_field_intensity(P, O, pos) * r[5].uniform(
            0.5, 1.5, size=(n_frames, frame, frame))
    return dict(psi=psi.astype(np.complex64), P=P.astype(np.complex64),
                O=O.astype(np.complex64), I=I.astype(np.float32), pos=pos,
                beta=beta)


def _random_case_obj_modes(seed, n_frames, frame, n_modes, obj_h, obj_w, consistent,
                           beta, perturb, L):
    """random_case with L object modes (see there)."""
    r = streams(seed + 7919 * L, 16)
    base = random_case(seed, n_frames, frame, n_modes, obj_h, obj_w, beta=beta)
    P = base["P"].astype(np.complex128)
    pos = base["pos"]
    O = np.stack([base["O"].astype(np.complex128)]
                 + [0.6 ** l * grf_object(obj_h, obj_w, r[2 * l], r[2 * l + 1], sigma=1.5)
                    for l in range(1, L)])
    O = O.astype(np.complex64).astype(np.complex128)
    ex = np.concatenate([P[None] * _windows(O[l], pos, frame)[:, None] for l in range(L)],
                        axis=1)                                   # [N][L M][F][F]
    I = far_field_intensity(P, O, pos)
    if consistent:
        psi = ex
    elif perturb is not None:
        noise = r[14].standard_normal(ex.shape) + 1j * r[14].standard_normal(ex.shape)
        psi = ex + perturb * np.abs(ex) * noise
        I = I * r[15].uniform(0.5, 1.5, size=I.shape)
    else:
        psi = r[14].standard_normal(ex.shape) + 1j * r[14].standard_normal(ex.shape)
        I = I * r[15].uniform(0.5, 1.5, size=I.shape)
    return dict(psi=psi.astype(np.complex64), P=P.astype(np.complex64),
                O=O.astype(np.complex64), I=I.astype(np.float32), pos=pos, beta=beta)
