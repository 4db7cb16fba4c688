"""Write <case>_trajectory.npz: the FP64 oracle's 100-iteration run from the
cold start on a strip of a benchmark scan, and the same run from a starting
probe perturbed at the FP32 rounding level (the oracle's own spread, against
which the GPU's trajectory is judged).  Cases:

  spiral_300     the first 300 views of the 2500-view, 5-mode, 128x128
                 spiral scan (Poisson 1e5 photons per frame)
  flyscan188_40  a block of 5 x 8 views (rows 0-4, columns 0-7) of the
                 10000-view, 4-mode, 188x188 fly-scan raster (the paper's
                 frame size; Poisson 1e6)

Beside the error curves and the final probe and object it stores how far
the perturbed run ends from the base run: in the probe, in the object
(weighted by the Eq. 5 denominator), both also without the ambiguities (the
object after the best complex scale, the probe through its mode-summed
power, which a unitary mix of the modes leaves alone), and in the modelled
intensities
sum_k |F[P_k O_j]|^2 of every view, which, unlike P and O, are free of the
ambiguities of the problem (a complex scale c with P -> cP, O -> O/c, and a
linear phase ramp moved between probe and object).

Calls only the oracle and the seeded input generator.

    python tests/golden/make_trajectories.py [case ...]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import dm_oracle as oracle  # noqa: E402
from paper_1808_10375_amd import synth  # noqa: E402

N_ITER = 100
PERTURB = 6e-8   # relative size of the complex noise put on the starting probe
CASES = {
    "spiral_300": lambda: synth.multimode_spiral_128(1, n_frames=300),
    "flyscan188_40": lambda: synth.flyscan_raster_188(3, n_frames=500).subset(
        [100 * r + c for r in range(5) for c in range(8)]),
}


def out_path(case):
    return os.path.join(HERE, f"{case}_trajectory.npz")


def perturbed_probe(P0):
    rng = np.random.default_rng(5)
    noise = rng.standard_normal(P0.shape) + 1j * rng.standard_normal(P0.shape)
    return P0.astype(np.complex128) * (1 + PERTURB * noise)


def trajectory(s, P0):
    psi = oracle.init_views(P0, s.O0, s.pos)
    P = np.asarray(P0, dtype=np.complex128)
    O = s.O0.astype(np.complex128)
    I = s.I.astype(np.float64)
    hist = []
    t0 = time.time()
    for it in range(N_ITER):
        psi, P, O, e = oracle.iterate(psi, P, O, s.pos, I, s.beta)
        hist.append([e["eps_probe"], e["eps_obj"], e["eps_psi"]])
        if it % 10 == 9:
            print(f"  iteration {it + 1}: eps_P {e['eps_probe']:.4e} "
                  f"({time.time() - t0:.0f} s)", flush=True)
    # Eq. 5 denominator of the last object update (the weight the views put
    # on every object pixel)
    _, den = oracle.object_update(psi, P, O, s.pos)
    return np.array(hist), P, O, den


def modelled_intensity(P, O, pos):
    """sum_k |F[P_k O_window_j]|^2 of every view (the forward model, Eq. 1)."""
    return np.sum(np.abs(oracle.dft2(oracle.exit_waves(P, O, pos))) ** 2, axis=1)


def aligned_distances(P, O, P_ref, O_ref, w):
    """How far (P, O) lies from (P_ref, O_ref) once the ambiguities of
    Eqs. 1-5 are removed.  The exit waves P_k O are unchanged by a complex
    scale (P, O) -> (P / c, c O) and the intensities of Eq. 1 by a unitary
    mix of the probe modes; so O is compared after the scale c that brings
    it closest to O_ref (least squares weighted by w, the Eq. 5
    denominator), and the probe through its mode-summed power
    sum_k |P_k / c|^2, which no mix changes.  O and O_ref cover the same
    box of pixels as w.  Returns (probe power distance, weighted object
    distance), both relative L2."""
    c = np.sum(w * np.conj(O) * O_ref) / np.sum(w * np.abs(O) ** 2)
    d_O = float(np.sqrt(np.sum(w * np.abs(c * O - O_ref) ** 2) / np.sum(w * np.abs(O_ref) ** 2)))
    pw = np.sum(np.abs(P / c) ** 2, axis=0)
    pw_ref = np.sum(np.abs(P_ref) ** 2, axis=0)
    d_P = float(np.linalg.norm(pw - pw_ref) / np.linalg.norm(pw_ref))
    return d_P, d_O


def make(case):
    s = CASES[case]()
    print("oracle run from the cold start", flush=True)
    h, P, O, den = trajectory(s, s.P0)
    print("oracle run from the perturbed start", flush=True)
    hp, Pp, Op, _ = trajectory(s, perturbed_probe(s.P0))
    cov = den > 0
    ys, xs = np.nonzero(cov)
    y0, y1, x0, x1 = ys.min(), ys.max() + 1, xs.min(), xs.max() + 1
    w = den[y0:y1, x0:x1]

    def rel(a, b, wt=1.0):
        return float(np.sqrt(np.sum(wt * np.abs(a - b) ** 2) / np.sum(wt * np.abs(b) ** 2)))

    out = out_path(case)
    model_spread = rel(modelled_intensity(Pp, Op, s.pos), modelled_intensity(P, O, s.pos))
    sP, sO = aligned_distances(Pp, Op[y0:y1, x0:x1], P, O[y0:y1, x0:x1], w)
    np.savez_compressed(
        out, eps=h, eps_perturbed=hp, P=P.astype(np.complex64),
        O_box=O[y0:y1, x0:x1].astype(np.complex64), den_box=w.astype(np.float32),
        box=np.array([y0, y1, x0, x1]), perturb=PERTURB,
        P_spread=rel(Pp, P), O_spread_weighted=rel(Op[y0:y1, x0:x1], O[y0:y1, x0:x1], w),
        P_spread_aligned=sP, O_spread_aligned=sO, model_spread=model_spread)
    print(f"wrote {out}: eps_P(50) {h[49, 0]:.4e} eps_P(100) {h[99, 0]:.4e}; "
          f"spread P {rel(Pp, P):.3e} O(weighted) {rel(Op[y0:y1, x0:x1], O[y0:y1, x0:x1], w):.3e} "
          f"without the ambiguities: probe power {sP:.3e} O(weighted) {sO:.3e}; "
          f"modelled intensities {model_spread:.3e}",
          flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        make(name)
