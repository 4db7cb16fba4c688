"""GPU parity with several object modes (Eqs. 1-5 with l over L > 1 object
modes; dm_desc.n_obj_modes): one iteration from the same state on the GPU
and in the FP64 oracle, to the plain path's bars (1e-5 relative L2 for psi'
and P', O' weighted by the Eq. 5 denominator, 10x that unweighted), on the
three-kernel path that object modes run on."""
import sys

import numpy as np
import pytest

from oracle import dm_oracle as oracle
from paper_1808_10375_amd import synth
from test_gpu_parity import (PROBE_FIRST, gpu_one_step, one_step_case, psi_free_case, rel,
                             rel_weighted)

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    # (seed, N, F, M, L, H, W)
    (1, 17, 32, 2, 2, 90, 77),
    (2, 13, 64, 1, 3, 140, 150),
    (3, 9, 128, 3, 2, 220, 200),
    (4, 5, 256, 2, 2, 300, 290),
    (5, 21, 16, 4, 4, 60, 50),      # the most object modes, 16 pairs
    (6, 7, 64, 16, 2, 120, 110),    # the most pairs (32)
]


@pytest.mark.parametrize("seed,n,f,m,L,h,w", CASES)
def test_one_step_object_modes(seed, n, f, m, L, h, w):
    say(f"case object modes seed={seed} N={n} F={f} M={m} L={L} obj={h}x{w}")
    one_step_case(synth.random_case(seed, n, f, m, h, w, n_obj_modes=L))


@pytest.mark.parametrize("seed,n,f,m,L,h,w", [(12, 13, 64, 2, 2, 150, 140),
                                              (13, 5, 256, 2, 2, 300, 290)])
def test_psi_free_update_object_modes(seed, n, f, m, L, h, w):
    """DM_FLAG_PSI_ERROR_LAST with L object modes: every frame (k, l) of a
    view takes the scale beta g - 1/F^2 and psi' = (2 - beta) P_k O_l + the
    inverse, over three iterations against the oracle and the same call
    without the flag."""
    from paper_1808_10375_amd import dm
    psi_free_case(seed, n, f, m, h, w, 1, dm.DM_FLAG_MULTIPASS if f <= 128 else 0,
                  n_obj_modes=L)


@pytest.mark.parametrize("seed,n,f,m,L,h,w", [(7, 11, 64, 2, 2, 130, 120),
                                              (8, 6, 128, 2, 3, 200, 190)])
def test_one_step_object_modes_probe_first(seed, n, f, m, L, h, w):
    say(f"case object modes probe first seed={seed} N={n} F={f} M={m} L={L}")
    one_step_case(synth.random_case(seed, n, f, m, h, w, n_obj_modes=L), flags=PROBE_FIRST)


def test_object_modes_fixed_point_and_beta_one():
    say("case object modes: consistent fixed point F=64 M=2 L=2, beta 1")
    c = synth.random_case(9, 15, 64, 2, 150, 140, consistent=True, n_obj_modes=2)
    psi_g, P_g, O_g, e, _ = gpu_one_step(c["psi"], c["P"], c["O"], c["I"], c["pos"], 0.8)
    den = oracle.object_update(c["psi"], c["P"].astype(np.complex128),
                               c["O"].astype(np.complex128), c["pos"])[1]
    assert rel(psi_g, c["psi"]) < 2e-6 and rel(P_g, c["P"]) < 2e-6
    assert rel_weighted(O_g, c["O"], den) < 2e-6
    assert e["eps_probe"] < 2e-6
    c = synth.random_case(10, 12, 32, 2, 80, 80, n_obj_modes=2, beta=1.0)
    one_step_case(c)


def test_object_modes_three_iterations_and_graph():
    """Three iterations in one call against three oracle iterations; the same
    with the iteration replayed as a hipGraph equals the eager launches bit
    for bit."""
    torch = _torch()
    from paper_1808_10375_amd import dm
    say("case object modes: 3 iterations, eager and graph, F=64 M=2 L=2")
    c = synth.random_case(11, 19, 64, 2, 150, 160, perturb=0.2, n_obj_modes=2)
    psi = c["psi"].astype(np.complex128)
    P, O = c["P"].astype(np.complex128), c["O"].astype(np.complex128)
    for _ in range(3):
        psi, P, O, e_o = oracle.iterate(psi, P, O, c["pos"], c["I"].astype(np.float64), 0.8)
    dev = torch.device("cuda:0")
    outs = []
    for flags in (0, dm.DM_FLAG_GRAPH):
        stream = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(stream):
            Pt = torch.from_numpy(c["P"]).to(dev)
            Ot = torch.from_numpy(c["O"]).to(dev)
            ctx = dm.DMContext(torch.from_numpy(c["I"]).to(dev), c["pos"], Pt, Ot, flags=flags,
                               stream=stream)
            ctx.set_state(torch.from_numpy(c["psi"]).to(dev), Pt, Ot, 0)
            ctx.iterate(3)
            stream.synchronize()
            psi_g, P_g, O_g, it = ctx.state()
            outs.append((psi_g.cpu().numpy(), P_g.cpu().numpy(), O_g.cpu().numpy(),
                         ctx.errors()))
            ctx.free()
    for a, b in zip(outs[0][:3], outs[1][:3]):
        assert np.array_equal(a, b)
    psi_g, P_g, O_g, e_g = outs[0]
    den = oracle.object_update(psi, P, O, c["pos"])[1]
    r = (rel(psi_g, psi), rel(P_g, P), rel_weighted(O_g, O, den))
    say(f"  rel L2 after 3: psi {r[0]:.2e} P {r[1]:.2e} O(weighted) {r[2]:.2e}")
    assert max(r) <= 1e-5, r
    assert abs(e_g["eps_probe"] - e_o["eps_probe"]) <= 1e-4 * e_o["eps_probe"]


def test_object_modes_orthogonalize():
    """Probe-mode orthogonalisation with two object modes mixes the probe
    modes inside each object mode's block of frames."""
    torch = _torch()
    from paper_1808_10375_amd import dm
    say("case object modes: orthogonal probe modes F=32 M=3 L=2")
    c = synth.random_case(12, 6, 32, 3, 70, 70, n_obj_modes=2)
    rng = np.random.default_rng(3)
    Lm = np.tril(rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3)))
    c["P"] = np.einsum("kl,lyx->kyx", Lm, c["P"].astype(np.complex128)).astype(np.complex64)
    dev = torch.device("cuda:0")
    Pt = torch.from_numpy(c["P"]).to(dev)
    Ot = torch.from_numpy(c["O"]).to(dev)
    ctx = dm.DMContext(torch.from_numpy(c["I"]).to(dev), c["pos"], Pt, Ot)
    ctx.set_state(torch.from_numpy(c["psi"]).to(dev), Pt, Ot, 0)
    lam = ctx.orthogonalize_modes()
    psi_g, P_g, O_g, _ = ctx.state()
    ctx.free()
    psi_o, Q_o, lam_o, _ = oracle.orthogonalize_modes(c["psi"], c["P"])
    assert rel(P_g.cpu().numpy(), Q_o) <= 1e-6
    assert rel(psi_g.cpu().numpy(), psi_o) <= 1e-6
    assert np.allclose(lam, lam_o, rtol=1e-10)
    assert np.array_equal(O_g.cpu().numpy(), c["O"])


def test_object_modes_limits():
    torch = _torch()
    from paper_1808_10375_amd import dm
    say("case object modes: refused forms")
    dev = torch.device("cuda:0")
    c = synth.random_case(13, 4, 64, 2, 80, 80, n_obj_modes=2)
    I = torch.from_numpy(c["I"]).to(dev)
    P = torch.from_numpy(c["P"]).to(dev)
    O = torch.from_numpy(c["O"]).to(dev)
    ctx = dm.DMContext(I, c["pos"], P, O)
    with pytest.raises(dm.DMError) as ex:
        ctx.warm_start(torch.zeros((4, 64, 64), dtype=torch.complex64, device=dev))
    assert ex.value.status == dm.DM_E_UNSUPPORTED
    with pytest.raises(dm.DMError) as ex:
        ctx.set_tuning(16, 4, dm.DM_VIEWS_STREAMED_MERGED)
    assert ex.value.status == dm.DM_E_ARG
    ctx.free()
    for kw in (dict(precision=dm.DM_BF16X3_DFT),):
        with pytest.raises(dm.DMError) as ex:
            dm.DMContext(torch.zeros((4, 128, 128), device=dev), c["pos"],
                         torch.zeros((2, 128, 128), dtype=torch.complex64, device=dev),
                         torch.zeros((2, 200, 200), dtype=torch.complex64, device=dev), **kw)
        assert ex.value.status in (dm.DM_E_UNSUPPORTED, dm.DM_E_ARG)
