"""GPU tests of the batched form: many scans of uneven size advanced by one
launch chain per iteration, its hipGraph replay, and launch tuning.

A batch must give each scan exactly what that scan gives alone (same kernels,
same summation order for equal tuning), a graph replay exactly what eager
launches give, and any tuning the oracle's result to the parity bar.
"""
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


def uneven_scans(seed=40, sizes=(23, 57, 11, 40), f=64, m=3, objs=(150, 200, 100, 170)):
    out = []
    for i, (n, h) in enumerate(zip(sizes, objs)):
        c = synth.random_case(seed + i, n, f, m, h, h + 10 * (i % 2), perturb=0.5,
                              beta=[0.8, 0.7, 1.0, 0.5][i % 4])
        out.append(dict(I=c["I"], pos=c["pos"], P0=c["P"], O0=c["O"], beta=c["beta"]))
    return out


def single(scan, flags=0, stream=None):
    torch = _torch()
    from paper_1808_10375_amd import dm
    dev = torch.device("cuda:0")
    return dm.DMContext(torch.from_numpy(scan["I"]).to(dev), scan["pos"],
                        torch.from_numpy(scan["P0"]).to(dev),
                        torch.from_numpy(scan["O0"]).to(dev), beta=scan["beta"], flags=flags,
                        stream=stream)


def test_batch_equals_each_scan_alone():
    _torch()
    from paper_1808_10375_amd import dm
    scans = uneven_scans()
    say(f"case batch of {len(scans)} scans, sizes {[len(s['pos']) for s in scans]}")
    b = dm.DMBatch(scans)
    assert b.n_scans == len(scans)
    b.iterate(3)
    for s, sc in enumerate(scans):
        ctx = single(sc)
        ctx.iterate(3)
        Ob, Pb = b.object(s).cpu().numpy(), b.probe(s).cpu().numpy()
        Os, Ps = ctx.object().cpu().numpy(), ctx.probe().cpu().numpy()
        eb = [e["eps_probe"] for e in b.error_history(s, 1, 3)]
        es = [e["eps_probe"] for e in ctx.error_history(1, 3)]
        say(f"  scan {s}: rel O {rel(Ob, Os):.1e} P {rel(Pb, Ps):.1e} "
            f"bitwise {np.array_equal(Ob, Os) and np.array_equal(Pb, Ps)}")
        assert rel(Ob, Os) <= 1e-6 and rel(Pb, Ps) <= 1e-6
        assert np.allclose(eb, es, rtol=1e-6)
        ctx.free()
    b.free()


def test_batch_matches_oracle_per_scan():
    _torch()
    from paper_1808_10375_amd import dm
    scans = uneven_scans(seed=50, sizes=(31, 9, 44), f=32, m=2, objs=(90, 64, 120))
    say("case batch of 3 scans vs oracle, 1 iteration from the initial views")
    b = dm.DMBatch(scans)
    b.iterate(1)
    for s, sc in enumerate(scans):
        psi0 = oracle.init_views(sc["P0"], sc["O0"], sc["pos"])
        _, P_o, O_o, e_o = oracle.iterate(psi0, sc["P0"], sc["O0"], sc["pos"],
                                          sc["I"].astype(np.float64), sc["beta"])
        den = oracle.object_update(oracle.view_update(psi0, sc["P0"], sc["O0"], sc["pos"],
                                                      sc["I"].astype(np.float64), sc["beta"]),
                                   sc["P0"], sc["O0"], sc["pos"])[1]
        Og, Pg = b.object(s).cpu().numpy(), b.probe(s).cpu().numpy()
        wrel = float(np.sqrt(np.sum(den * np.abs(Og - O_o) ** 2) / np.sum(den * np.abs(O_o) ** 2)))
        say(f"  scan {s}: rel P {rel(Pg, P_o):.1e} O(weighted) {wrel:.1e}")
        assert rel(Pg, P_o) <= 1e-5 and wrel <= 1e-5
        eg = b.error_history(s, 1, 1)[0]
        assert abs(eg["eps_probe"] - e_o["eps_probe"]) <= 1e-4 * e_o["eps_probe"]
    b.free()


def test_graph_replays_equal_eager_launches():
    torch = _torch()
    from paper_1808_10375_amd import dm
    scans = uneven_scans(seed=60, sizes=(17, 29), f=64, m=2, objs=(140, 120))
    say("case graph replay vs eager, 4 iterations with host work between replays")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = dm.DMBatch(scans, flags=dm.DM_FLAG_GRAPH, stream=stream)
    e = dm.DMBatch(scans)
    for it in range(4):
        g.iterate(1)
        e.iterate(1)
        stream.synchronize()
        torch.cuda.synchronize()
        _ = np.linalg.norm(np.ones(1000))  # eager host work between replays
        for s in range(len(scans)):
            a, b = g.object(s), e.object(s)
            torch.cuda.synchronize()
            assert torch.equal(a, b), (it, s)
            assert torch.equal(g.probe(s), e.probe(s)), (it, s)
        eg = [x["eps_probe"] for x in g.error_history(0, 1, it + 1)]
        ee = [x["eps_probe"] for x in e.error_history(0, 1, it + 1)]
        assert eg == ee
    g.free()
    e.free()


def test_probe_first_batch_graphs_equal_eager_and_oracle():
    """DM_FLAG_PROBE_FIRST on a batch of two scans: after one iteration the
    probe and object match the oracle in the same order; graph replays equal
    eager launches bitwise after one and after three iterations."""
    torch = _torch()
    from paper_1808_10375_amd import dm
    scans = uneven_scans(seed=75, sizes=(19, 26), f=64, m=2, objs=(150, 130))
    say("case probe-first batch: graph vs eager over 3 iterations, oracle after 1")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = dm.DMBatch(scans, flags=dm.DM_FLAG_GRAPH | dm.DM_FLAG_PROBE_FIRST, stream=stream)
    e = dm.DMBatch(scans, flags=dm.DM_FLAG_PROBE_FIRST)
    for n_it in (1, 2):
        g.iterate(n_it)
        e.iterate(n_it)
        stream.synchronize()
        torch.cuda.synchronize()
        for s, sc in enumerate(scans):
            og, oe, pg, pe = g.object(s), e.object(s), g.probe(s), e.probe(s)
            torch.cuda.synchronize()
            assert torch.equal(og, oe) and torch.equal(pg, pe), (n_it, s)
            if n_it != 1:
                continue
            psi0 = oracle.init_views(sc["P0"], sc["O0"], sc["pos"])
            psi, P, O, e_o = oracle.iterate(psi0, sc["P0"], sc["O0"], sc["pos"],
                                            sc["I"].astype(np.float64), sc["beta"],
                                            probe_first=True)
            den = oracle.object_update(psi, P, sc["O0"], sc["pos"])[1]
            Og = oe.cpu().numpy()
            wrel = float(np.sqrt(np.sum(den * np.abs(Og - O) ** 2) /
                                 np.sum(den * np.abs(O) ** 2)))
            say(f"  scan {s}: rel P {rel(pe.cpu().numpy(), P):.1e} O(weighted) {wrel:.1e}")
            assert rel(pe.cpu().numpy(), P) <= 1e-5 and wrel <= 1e-5
            eg = e.error_history(s, 1, 1)[0]
            assert abs(eg["eps_probe"] - e_o["eps_probe"]) <= 1e-4 * e_o["eps_probe"]
    g.free()
    e.free()


@pytest.mark.parametrize("f,objs", [(128, (200, 180)), (188, (300, 280))])
def test_graphs_with_psi_error_last_equal_eager_launches(f, objs):
    """DM_FLAG_PSI_ERROR_LAST with graph replay: each context keeps one graph
    without and one with the eps_psi partials (the last iteration of a
    call).  Calls of 3 and 2 iterations replayed against the same calls
    launched eagerly: bitwise equal states and errors, eps_psi NaN in every
    iteration but the last of each call; and within 1e-5 of the update that
    reads psi in every iteration (no flag).  F = 128 runs the merged
    streamed kernel, F = 188 the mixed-radix three-kernel path."""
    torch = _torch()
    from paper_1808_10375_amd import dm
    scans = uneven_scans(seed=70, sizes=(9, 14), f=f, m=2, objs=objs)
    say(f"case graphs with DM_FLAG_PSI_ERROR_LAST vs eager, F={f}, calls of 3 and 2 iterations")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = dm.DMBatch(scans, flags=dm.DM_FLAG_GRAPH | dm.DM_FLAG_PSI_ERROR_LAST,
                       stream=stream)
    e = dm.DMBatch(scans, flags=dm.DM_FLAG_PSI_ERROR_LAST)
    d = dm.DMBatch(scans)
    done = 0
    for n in (3, 2):
        g.iterate(n)
        e.iterate(n)
        d.iterate(n)
        stream.synchronize()
        torch.cuda.synchronize()
        done += n
        for s in range(len(scans)):
            og, oe, pg, pe, pd = g.object(s), e.object(s), g.probe(s), e.probe(s), d.probe(s)
            stream.synchronize()
            torch.cuda.synchronize()
            assert torch.equal(og, oe), (done, s)
            assert torch.equal(pg, pe), (done, s)
            assert rel(pg.cpu().numpy(), pd.cpu().numpy()) <= 1e-5
            hg = g.error_history(s, 1, done)
            he = e.error_history(s, 1, done)
            for k, (x, y) in enumerate(zip(hg, he)):
                last = (k + 1 == 3) or (k + 1 == done)
                assert np.isnan(x["eps_psi"]) != last, (done, s, k)
                assert x["eps_probe"] == y["eps_probe"] and x["eps_obj"] == y["eps_obj"]
                if last:
                    assert x["eps_psi"] == y["eps_psi"]
    g.free()
    e.free()
    d.free()


@pytest.mark.parametrize("tile,chunks,view_path", [(32, 16, 0), (16, 3, 0), (32, 64, 1),
                                                   (16, 16, 2), (32, 8, 3), (16, 8, 4),
                                                   (32, 16, 5)])
def test_tunings_keep_parity(tile, chunks, view_path):
    _torch()
    from paper_1808_10375_amd import dm
    c = synth.random_case(70, 27, 64, 3, 180, 170, perturb=0.5)
    say(f"case tuning tile={tile} chunks={chunks} view_path={view_path}")
    sc = dict(I=c["I"], pos=c["pos"], P0=c["P"], O0=c["O"], beta=c["beta"])
    ctx = single(sc, flags=dm.DM_FLAG_MULTIPASS if view_path == 1 else 0)
    ctx.set_tuning(tile, chunks, view_path)
    assert ctx.tuning() == {"obj_tile": tile, "probe_chunks": chunks, "view_path": view_path}
    ctx.iterate(1)
    psi0 = oracle.init_views(c["P"], c["O"], c["pos"])
    _, P_o, O_o, _ = oracle.iterate(psi0, c["P"], c["O"], c["pos"], c["I"].astype(np.float64),
                                    c["beta"])
    assert rel(ctx.probe().cpu().numpy(), P_o) <= 1e-5
    ctx.free()


def test_autotune_picks_a_valid_tuning_and_restores_the_start(tmp_path):
    _torch()
    from paper_1808_10375_amd import dm
    scans = uneven_scans(seed=80, sizes=(40, 25), f=64, m=2, objs=(160, 150))
    say("case autotune + cache")
    cache = str(tmp_path / "tune.jsonl")
    b = dm.DMBatch(scans)
    t = b.autotune(reps=3, cache_path=cache)
    say(f"  chosen {t}")
    assert t["obj_tile"] in (16, 32) and 1 <= t["probe_chunks"] <= 64
    assert b.iterations == 0
    b.iterate(2)
    ref = dm.DMBatch(scans)
    ref.set_tuning(t["obj_tile"], t["probe_chunks"], t["view_path"])
    ref.iterate(2)
    for s in range(2):
        assert rel(b.probe(s).cpu().numpy(), ref.probe(s).cpu().numpy()) == 0.0
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"obj_tile"' in lines[0]
    # a second autotune reads the cache
    again = dm.DMBatch(scans)
    assert again.autotune(reps=3, cache_path=cache) == t
    assert len(open(cache).read().strip().splitlines()) == 1
    for x in (b, ref, again):
        x.free()
