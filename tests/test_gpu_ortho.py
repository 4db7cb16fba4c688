"""GPU parity of the orthogonal probe modes (dm_orthogonalize_modes): the
eigenmodes of the probe modes' overlap matrix, with the views mixed by the
same unitary, against the FP64 oracle's orthogonalize_modes (numpy's eigh),
and the mode-count rule of Section II run on those eigen-powers.

Both sides form the overlaps in FP64 from the same FP32 modes; the GPU
rounds its mixed modes to FP32 once, so the bar is 1e-6 relative L2 (a few
FP32 roundings), tighter than the iteration's 1e-5."""
import sys

import numpy as np
import pytest

from oracle import dm_oracle as oracle
from paper_1808_10375_amd import modes, synth

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def correlated_case(seed, n, f, m, h, w):
    """A random state whose probe modes overlap strongly: mode k is a lower
    triangular mix of independent random modes, with well separated
    eigenvalues of the overlap matrix."""
    c = synth.random_case(seed, n, f, m, h, w)
    rng = np.random.default_rng(seed + 100)
    L = np.tril(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    L[np.diag_indices(m)] = 2.0 ** -np.arange(m) * 3.0
    P = np.einsum("kl,lyx->kyx", L, c["P"].astype(np.complex128))
    c["P"] = P.astype(np.complex64)
    return c


def gpu_ortho(c):
    torch = _torch()
    from paper_1808_10375_amd import dm
    dev = torch.device("cuda:0")
    Pt = torch.from_numpy(c["P"]).to(dev)
    Ot = torch.from_numpy(c["O"]).to(dev)
    ctx = dm.DMContext(torch.from_numpy(c["I"]).to(dev), c["pos"], Pt, Ot, beta=c["beta"])
    ctx.set_state(torch.from_numpy(c["psi"]).to(dev), Pt, Ot, 0)
    lam = ctx.orthogonalize_modes()
    psi, P, O, _ = ctx.state()
    out = psi.cpu().numpy(), P.cpu().numpy(), O.cpu().numpy(), np.array(lam)
    ctx.free()
    return out


@pytest.mark.parametrize("seed,n,f,m,h,w", [
    (1, 7, 32, 3, 70, 53),
    (2, 5, 64, 5, 90, 100),
    (3, 3, 16, 16, 40, 40),     # the largest mode count
    (4, 4, 128, 2, 150, 140),
    (5, 3, 188, 4, 200, 210),   # a frame of the paper's size
])
def test_orthogonalize_matches_oracle(seed, n, f, m, h, w):
    say(f"case ortho seed={seed} N={n} F={f} M={m}")
    c = correlated_case(seed, n, f, m, h, w)
    psi_g, P_g, O_g, lam_g = gpu_ortho(c)
    psi_o, Q_o, lam_o, V_o = oracle.orthogonalize_modes(c["psi"], c["P"])
    assert rel(P_g, Q_o) <= TOL, rel(P_g, Q_o)
    assert rel(psi_g, psi_o) <= TOL, rel(psi_g, psi_o)
    assert np.allclose(lam_g, lam_o, rtol=1e-10, atol=1e-12 * lam_o[0])
    # the object is untouched; the new modes are orthogonal with powers lam
    assert np.array_equal(O_g, c["O"])
    G = oracle.mode_gram(P_g)
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() <= 1e-6 * lam_o[0]
    assert np.allclose(np.diag(G).real, lam_o, rtol=1e-6)


def test_single_mode_and_orthogonal_modes_are_left_alone():
    say("case ortho: one mode; orthogonal HG modes")
    c = synth.random_case(7, 5, 32, 1, 60, 60)
    psi_g, P_g, _, lam = gpu_ortho(c)
    assert np.array_equal(P_g, c["P"]) and np.array_equal(psi_g, c["psi"])
    assert abs(lam[0] - np.sum(np.abs(c["P"].astype(np.complex128)) ** 2)) <= 1e-12 * lam[0]
    # Hermite-Gaussian modes with distinct weights: already the eigenmodes
    hg = synth.hermite_gauss_modes(64, 8.0, [(0, 0), (1, 0), (0, 1)], [1.0, 0.4, 0.1])
    c = synth.random_case(8, 4, 64, 3, 90, 90)
    c["P"] = hg.astype(np.complex64)
    _, P_g, _, lam = gpu_ortho(c)
    assert rel(P_g, c["P"]) <= TOL
    assert lam[0] > lam[1] > lam[2]


def test_iteration_is_unchanged_by_the_mix():
    """One DM iteration from the orthogonalised state gives the same object
    as one from the original state (Eq. 5 and F_c are invariant under a
    unitary mix of the modes), and probes related by the same mix."""
    torch = _torch()
    from paper_1808_10375_amd import dm
    say("case ortho: iteration invariance F=64 M=3")
    c = correlated_case(11, 9, 64, 3, 120, 110)
    dev = torch.device("cuda:0")
    Pt = torch.from_numpy(c["P"]).to(dev)
    Ot = torch.from_numpy(c["O"]).to(dev)
    psit = torch.from_numpy(c["psi"]).to(dev)
    ctx = dm.DMContext(torch.from_numpy(c["I"]).to(dev), c["pos"], Pt, Ot, beta=c["beta"])
    ctx.set_state(psit, Pt, Ot, 0)
    ctx.iterate(1)
    _, P1, O1, _ = ctx.state()
    ctx.set_state(psit, Pt, Ot, 0)
    ctx.orthogonalize_modes(want_power=False)
    ctx.iterate(1)
    _, P2, O2, _ = ctx.state()
    ctx.free()
    _, _, _, V = oracle.orthogonalize_modes(c["psi"], c["P"])
    den = oracle.object_update(c["psi"].astype(np.complex128), c["P"].astype(np.complex128),
                               c["O"].astype(np.complex128), c["pos"])[1]
    w = np.sqrt(den)
    assert rel(O2.cpu().numpy() * w, O1.cpu().numpy() * w) <= 1e-5
    P1m = np.einsum("ka,kyx->ayx", V, P1.cpu().numpy().astype(np.complex128))
    assert rel(P2.cpu().numpy(), P1m) <= 1e-5


def test_mode_rule_on_eigen_powers():
    """Section II's 1% rule on the powers of the eigenmodes: probes that are
    arbitrary unitary mixes of Hermite-Gaussian modes with weights 1, 0.3,
    0.05, 0.004 (the last below 1%).  The plain per-mode powers of the mixes
    hide the weak mode; the eigen-powers recover the weights, and the search
    stops at the fourth mode."""
    torch = _torch()
    from paper_1808_10375_amd import dm
    weights = [1.0, 0.3, 0.05, 0.004]
    orders = [(0, 0), (1, 0), (0, 1), (2, 0)]
    f = 64
    hg = synth.hermite_gauss_modes(f, 8.0, orders, weights).astype(np.complex128)
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5)
    plain = {}

    def run(m):
        say(f"case mode rule M={m}")
        z = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        U, _ = np.linalg.qr(z)
        P = np.einsum("kl,lyx->kyx", U, hg[:m]).astype(np.complex64)
        c = synth.random_case(20 + m, 4, f, m, 100, 100)
        Pt = torch.from_numpy(P).to(dev)
        Ot = torch.from_numpy(c["O"]).to(dev)
        ctx = dm.DMContext(torch.from_numpy(c["I"]).to(dev), c["pos"], Pt, Ot)
        plain[m] = ctx.mode_power()
        lam = ctx.orthogonalize_modes()
        ctx.free()
        return lam

    chosen, hist = modes.choose_mode_count(run, max_modes=4)
    assert chosen == 3 and [h[0] for h in hist] == [1, 2, 3, 4]
    share = np.array(weights) / sum(weights)
    assert np.allclose(hist[-1][1], share, rtol=1e-5)
    assert min(modes.mode_fractions(plain[4])) > 0.01
