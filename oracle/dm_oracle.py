"""FP64 CPU oracle for one multi-mode difference-map (DM) iteration.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import this module.  The GPU library never
calls it, and it shares no code, tables or constants with the GPU path.

It follows Section II of Dong, Fang et al., "High-Performance Multi-Mode
Ptychography Reconstruction on Distributed GPUs" (arXiv:1808.10375), step by
step, in complex128.  The formulas below are written for one object mode
(M_O = 1, the paper knows no case where more help), so the mode index k runs
over probe modes; an object of shape [L][H][W] gives L object modes, the
views then carry the pairs (k, l) of Eqs. 1-5 at index l*M + k, F_c sums over
all pairs, Eq. 5 updates every O_l with its own views and Eq. 4 sums over l:

  exit wave       phi_{j,k} = P_k * O[window_j]                       (Eq. 2)
  view update     psi <- psi + beta * (F^-1 F_c[2 phi - psi] - phi)   (Eq. 3)
  constrained FT  F_c keeps the phase and rescales every mode by
                  sqrt(I_j / sum_k |F[.]_k|^2)                   (definition of
                                                                  F_c, Eq. 3)
  object update   O = sum_j sum_k conj(P_k) psi_{j,k} / sum_j sum_k |P_k|^2,
                  accumulated by embedding each view's window into the
                  object, one view after another (Eq. 5 and the embedding
                  procedure of Section III)
  probe update    P_k = sum_j conj(O[window_j]) psi_{j,k}
                        / sum_j |O[window_j]|^2                         (Eq. 4)
  convergence     relative L2 change between iterations             (Eq. 6)

Readings where the paper is silent (each also listed in the design notes):
  * order: views first, then the object from (psi', P_old), then the probe
    from (psi', O_new); one object/probe pass per iteration.  Section III
    describes swapping the P and O updates as an optimisation: from the
    order the equations are written in (probe first) to object first, which
    lets the object embedding of one batch of views overlap the view update
    of the next.  The swapped order is the default here; probe first is the
    option probe_first.
  * F is the unnormalised forward DFT with exp(-2 pi i k n / F); F^-1 carries
    1/F^2; DC sits at index [0, 0] (no fftshift).
  * where sum_k |F[.]_k|^2 == 0 every mode's spectrum is 0 there, and the
    projected value is 0.
  * zero denominators in Eqs. 4-5 (pixels no view covers) keep the previous
    value; no regulariser is added.
  * the window of view j is rows y_j..y_j+F-1, columns x_j..x_j+F-1 of the
    object, with (y_j, x_j) an integer top-left corner.
  * err = eps_P: Eq. 6 with the mode sum inside both norms; eps_P per mode,
    eps_psi and eps_O (over covered object pixels) are reported beside it.

Array layouts (same as the library's): psi [N][M][F][F], P [M][F][F],
O [H][W], I [N][F][F], pos [N][2] as (y, x).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "dft2", "idft2", "exit_waves", "constrained_ft", "view_update",
    "object_update", "probe_update", "rel_change", "iterate", "init_views",
    "run", "mode_gram", "orthogonalize_modes",
]


# ---------------------------------------------------------------------------
# transforms (the FFT library routine serves as the DFT step)
# ---------------------------------------------------------------------------
def dft2(x: np.ndarray) -> np.ndarray:
    """Unnormalised 2-D DFT over the last two axes, kernel exp(-2 pi i (ku+lv)/F)."""
    return np.fft.fft2(np.asarray(x, dtype=np.complex128), axes=(-2, -1))


def idft2(x: np.ndarray) -> np.ndarray:
    """Inverse 2-D DFT with the 1/F^2 factor, kernel exp(+2 pi i (ku+lv)/F)."""
    return np.fft.ifft2(np.asarray(x, dtype=np.complex128), axes=(-2, -1))


# ---------------------------------------------------------------------------
# Eq. 2: exit waves
# ---------------------------------------------------------------------------
def windows(O: np.ndarray, pos: np.ndarray, f: int) -> np.ndarray:
    """O[y_j : y_j+F, x_j : x_j+F] for every view j -> [N][F][F]."""
    return np.stack([O[y:y + f, x:x + f] for (y, x) in np.asarray(pos)])


def exit_waves(P: np.ndarray, O: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """phi_{j,k} = P_k * O[window_j] (Eq. 2) -> [N][M][F][F]; with object
    modes O [L][H][W], phi_{j,(k,l)} = P_k * O_l[window_j] at index l*M + k
    -> [N][L*M][F][F]."""
    P = np.asarray(P, dtype=np.complex128)
    O = np.asarray(O, dtype=np.complex128)
    if O.ndim == 2:
        return P[None, :, :, :] * windows(O, pos, P.shape[-1])[:, None, :, :]
    return np.concatenate([exit_waves(P, O[l], pos) for l in range(O.shape[0])], axis=1)


# ---------------------------------------------------------------------------
# F_c: constrained Fourier transform (modulus projection)
# ---------------------------------------------------------------------------
def constrained_ft(spectra: np.ndarray, I: np.ndarray) -> np.ndarray:
    """Replace the computed amplitude by the measured one, keeping the phase:
    every mode k of view j is multiplied by sqrt(I_j / sum_k |spectra_k|^2).

    spectra [N][M][F][F] (already transformed; with object modes the second
    axis runs over all L*M pairs (k, l)), I [N][F][F] -> same shape.
    Where the mode sum is zero all modes are zero and the result is zero."""
    spectra = np.asarray(spectra, dtype=np.complex128)
    I = np.maximum(np.asarray(I, dtype=np.float64), 0.0)
    s = np.sum(np.abs(spectra) ** 2, axis=1)                 # [N][F][F]
    scale = np.zeros_like(s)
    nz = s > 0
    scale[nz] = np.sqrt(I[nz] / s[nz])
    return spectra * scale[:, None, :, :]


# ---------------------------------------------------------------------------
# Eq. 3: view update
# ---------------------------------------------------------------------------
def view_update(psi, P, O, pos, I, beta, chunk: int = 64):
    """psi' = psi + beta * (F^-1 F_c[2 phi - psi] - phi), phi = P*O (Eq. 3).

    Processed in chunks of views only to bound memory; every view is
    independent of the others."""
    psi = np.asarray(psi, dtype=np.complex128)
    out = np.empty_like(psi)
    for s in range(0, psi.shape[0], chunk):
        sl = slice(s, s + chunk)
        phi = exit_waves(P, O, pos[sl])
        z = 2.0 * phi - psi[sl]
        z_proj = idft2(constrained_ft(dft2(z), I[sl]))
        out[sl] = psi[sl] + beta * (z_proj - phi)
    return out


# ---------------------------------------------------------------------------
# Eq. 5: object update by embedding, view after view
# ---------------------------------------------------------------------------
def object_update(psi, P, O_old, pos):
    """O = sum_j sum_k conj(P_k) psi_{j,k} / sum_j sum_k |P_k|^2 (Eq. 5).

    Numerator and denominator are accumulated by embedding each view's
    F x F window into the object, in ascending j.  Pixels with a zero
    denominator keep O_old.  Returns (O_new, denominator).  With object
    modes (O_old [L][H][W]) object mode l takes the views of the pairs
    (k, l), psi[:, l*M:(l+1)*M]; the denominator is the same for every l."""
    psi = np.asarray(psi, dtype=np.complex128)
    P = np.asarray(P, dtype=np.complex128)
    if np.ndim(O_old) == 3:
        m = P.shape[0]
        parts = [object_update(psi[:, l * m:(l + 1) * m], P, O_old[l], pos)
                 for l in range(O_old.shape[0])]
        return np.stack([o for o, _ in parts]), parts[0][1]
    f = P.shape[-1]
    num = np.zeros(O_old.shape, dtype=np.complex128)
    den = np.zeros(O_old.shape, dtype=np.float64)
    p_conj = np.conj(P)
    p_pow = np.sum(np.abs(P) ** 2, axis=0)
    for j, (y, x) in enumerate(np.asarray(pos)):
        num[y:y + f, x:x + f] += np.sum(p_conj * psi[j], axis=0)
        den[y:y + f, x:x + f] += p_pow
    O_new = np.array(O_old, dtype=np.complex128)
    cov = den > 0
    O_new[cov] = num[cov] / den[cov]
    return O_new, den


# ---------------------------------------------------------------------------
# Eq. 4: probe update
# ---------------------------------------------------------------------------
def probe_update(psi, O, P_old, pos):
    """P_k = sum_j conj(O[window_j]) psi_{j,k} / sum_j |O[window_j]|^2 (Eq. 4).

    Pixels with a zero denominator keep P_old.  Returns (P_new, denominator).
    With object modes (O [L][H][W]) both sums also run over l:
    P_k = sum_l sum_j conj(O_l[window_j]) psi_{j,(k,l)}
          / sum_l sum_j |O_l[window_j]|^2."""
    psi = np.asarray(psi, dtype=np.complex128)
    O = np.asarray(O, dtype=np.complex128)
    objs = O[None] if O.ndim == 2 else O
    m = P_old.shape[0]
    f = P_old.shape[-1]
    num = np.zeros(P_old.shape, dtype=np.complex128)
    den = np.zeros(P_old.shape[-2:], dtype=np.float64)
    for l, Ol in enumerate(objs):
        for j, (y, x) in enumerate(np.asarray(pos)):
            w = Ol[y:y + f, x:x + f]
            num += np.conj(w)[None] * psi[j, l * m:(l + 1) * m]
            den += np.abs(w) ** 2
    P_new = np.array(P_old, dtype=np.complex128)
    ok = den > 0
    P_new[:, ok] = num[:, ok] / den[ok]
    return P_new, den


# ---------------------------------------------------------------------------
# Eq. 6: relative L2 change
# ---------------------------------------------------------------------------
def rel_change(new, old, mask=None) -> float:
    """sqrt(sum |new - old|^2 / sum |new|^2), sums over `mask` if given
    (Eq. 6 with sums in place of integrals).  0/0 is reported as 0."""
    new = np.asarray(new, dtype=np.complex128)
    old = np.asarray(old, dtype=np.complex128)
    if mask is not None:
        new, old = new[..., mask], old[..., mask]
    num = float(np.sum(np.abs(new - old) ** 2))
    den = float(np.sum(np.abs(new) ** 2))
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return float(np.sqrt(num / den))


# ---------------------------------------------------------------------------
# one iteration and a run
# ---------------------------------------------------------------------------
def iterate(psi, P, O, pos, I, beta, probe_first: bool = False):
    """One DM iteration: views (Eq. 3), then object (Eq. 5) from the new
    views and the old probe, then probe (Eq. 4) from the new views and the
    new object (Section III's swapped order).  With probe_first, the order
    before that swap: probe (Eq. 4) from the new views and the old object,
    then object (Eq. 5) from the new views and the new probe.
    Returns (psi', P', O', errors)."""
    pos = np.asarray(pos)
    P = np.asarray(P, dtype=np.complex128)
    O = np.asarray(O, dtype=np.complex128)
    psi_new = view_update(psi, P, O, pos, I, beta)
    if probe_first:
        P_new, _ = probe_update(psi_new, O, P, pos)
        O_new, den_o = object_update(psi_new, P_new, O, pos)
    else:
        O_new, den_o = object_update(psi_new, P, O, pos)
        P_new, _ = probe_update(psi_new, O_new, P, pos)
    errors = {
        "eps_psi": rel_change(psi_new, psi),
        "eps_obj": rel_change(O_new, O, den_o > 0),
        "eps_probe": rel_change(P_new, P),
        "eps_probe_mode": [rel_change(P_new[k], P[k])
                           for k in range(P.shape[0])],
    }
    return psi_new, P_new, O_new, errors


# ---------------------------------------------------------------------------
# orthogonal probe modes (the mixed-state treatment the multi-mode method of
# Section II builds on; the paper cites it and does not spell it out)
# ---------------------------------------------------------------------------
def mode_gram(P) -> np.ndarray:
    """G[k, l] = sum_r conj(P_k(r)) P_l(r): the overlap (Gram) matrix of the
    probe modes, M x M Hermitian positive semi-definite."""
    P = np.asarray(P, dtype=np.complex128)
    flat = P.reshape(P.shape[0], -1)
    return np.conj(flat) @ flat.T


def orthogonalize_modes(psi, P):
    """Replace the probe modes by orthogonal ones spanning the same space:
    with G = V diag(lam) V^H (eigenvalues descending), the new modes are
    Q_a = sum_k V[k, a] P_k, whose Gram matrix is diag(lam).  The views get
    the same unitary mix, psi'_{j,a} = sum_k V[k, a] psi_{j,k}, so the
    iteration continues from an equivalent state: the intensity model
    sum_k |F[P_k O]|^2 (Eq. 1), the mode sum of F_c, the object update and
    the probe update are all unchanged by a unitary mix of the modes.

    Each column of V is given a fixed phase: its entry of largest modulus
    (the first such) is made real and positive.  The eigenvectors come from
    the library routine numpy.linalg.eigh.
    Returns (psi', Q, lam, V)."""
    psi = np.asarray(psi, dtype=np.complex128)
    P = np.asarray(P, dtype=np.complex128)
    lam, V = np.linalg.eigh(mode_gram(P))
    lam, V = lam[::-1].copy(), V[:, ::-1].copy()
    for a in range(V.shape[1]):
        k = int(np.argmax(np.abs(V[:, a])))
        V[:, a] *= np.conj(V[k, a]) / abs(V[k, a])
    Q = np.einsum("ka,kyx->ayx", V, P)
    # views [N][L*M][F][F]: the probe modes are mixed within each object mode
    n, c = psi.shape[:2]
    m = P.shape[0]
    psi_new = np.einsum("ka,jlkyx->jlayx", V,
                        psi.reshape(n, c // m, m, *psi.shape[2:])).reshape(psi.shape)
    return psi_new, Q, lam, V


def init_views(P0, O0, pos) -> np.ndarray:
    """Initial views psi = P0 * O0 at every scan position (Section II)."""
    return exit_waves(P0, O0, pos)


def run(P0, O0, pos, I, beta, n_iter: int):
    """Initial views from (P0, O0), then n_iter iterations.
    Returns (psi, P, O, list of per-iteration error dicts)."""
    psi = init_views(P0, O0, pos)
    P = np.asarray(P0, dtype=np.complex128)
    O = np.asarray(O0, dtype=np.complex128)
    history = []
    for _ in range(n_iter):
        psi, P, O, e = iterate(psi, P, O, pos, I, beta)
        history.append(e)
    return psi, P, O, history
