"""The entry point that allocates nothing (dm_orthogonalize_modes_noalloc,
scratch in a static device array) against the context entry point it is a
variant of (dm_orthogonalize_modes, scratch in the caller's workspace): two
calls in a row on one GPU, the second smaller, each equal to the context
call bit for bit (same kernels and launch shapes) and to the FP64 oracle
within 1e-6."""
import sys

import numpy as np
import pytest

from oracle import dm_oracle as oracle
from paper_1808_10375_amd import synth

pytestmark = pytest.mark.gpu


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


def case(seed, n, f, m, h, w):
    c = synth.random_case(seed, n, f, m, h, w)
    rng = np.random.default_rng(seed + 7)
    L = np.tril(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    L[np.diag_indices(m)] = 1.5 ** -np.arange(m) * 2.0
    c["P"] = np.einsum("kl,lyx->kyx", L, c["P"].astype(np.complex128)).astype(np.complex64)
    return c


def with_context(c, dev):
    torch = _torch()
    from paper_1808_10375_amd import dm
    Pt = torch.from_numpy(c["P"]).to(dev)
    Ot = torch.from_numpy(c["O"]).to(dev)
    ctx = dm.DMContext(torch.from_numpy(c["I"]).to(dev), c["pos"], Pt, Ot, beta=c["beta"])
    ctx.set_state(torch.from_numpy(c["psi"]).to(dev), Pt, Ot, 0)
    lam = ctx.orthogonalize_modes()
    psi, P, _, _ = ctx.state()
    out = psi.cpu().numpy(), P.cpu().numpy(), np.array(lam)
    ctx.free()
    return out


def test_noalloc_matches_context_call_twice():
    torch = _torch()
    from paper_1808_10375_amd import dm
    dev = torch.device("cuda:0")
    # second call smaller in every size: views, frame, modes
    for k, (seed, n, f, m, h, w) in enumerate([(31, 9, 64, 5, 100, 90), (32, 4, 32, 3, 60, 50)]):
        say(f"case noalloc call {k + 1}: N={n} F={f} M={m}")
        c = case(seed, n, f, m, h, w)
        psi_c, P_c, lam_c = with_context(c, dev)
        Pt = torch.from_numpy(c["P"]).to(dev)
        psit = torch.from_numpy(c["psi"]).to(dev)
        powt = torch.full((m,), -1.0, dtype=torch.float64, device=dev)
        dm.dm_orthogonalize_modes_noalloc(Pt, psit, powt)
        torch.cuda.synchronize()
        P_n, psi_n, lam_n = Pt.cpu().numpy(), psit.cpu().numpy(), powt.cpu().numpy()
        assert np.array_equal(P_n, P_c) and np.array_equal(psi_n, psi_c)
        assert np.array_equal(lam_n, lam_c)
        psi_o, Q_o, lam_o, _ = oracle.orthogonalize_modes(c["psi"], c["P"])
        assert rel(P_n, Q_o) <= 1e-6 and rel(psi_n, psi_o) <= 1e-6
        assert np.allclose(lam_n, lam_o, rtol=1e-10)


def test_noalloc_probe_only_and_limits():
    torch = _torch()
    from paper_1808_10375_amd import dm
    dev = torch.device("cuda:0")
    say("case noalloc probe only, F=16 M=2")
    c = case(33, 1, 16, 2, 30, 30)
    Pt = torch.from_numpy(c["P"]).to(dev)
    dm.dm_orthogonalize_modes_noalloc(Pt)
    torch.cuda.synchronize()
    _, Q_o, _, _ = oracle.orthogonalize_modes(c["psi"], c["P"])
    assert rel(Pt.cpu().numpy(), Q_o) <= 1e-6
    # beyond the static scratch: refused before any launch
    big = torch.zeros((17, 16, 16), dtype=torch.complex64, device=dev)
    with pytest.raises(dm.DMError) as ex:
        dm.dm_orthogonalize_modes_noalloc(big)
    assert ex.value.status == dm.DM_E_UNSUPPORTED and "16 modes" in str(ex.value)
    assert bool(torch.all(big == 0))
