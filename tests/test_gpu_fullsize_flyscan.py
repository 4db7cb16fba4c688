"""The fly scans at full size, one iteration from the initial views in the
launch configuration the benchmark times (the library's default tuning for
the context): 10000 views x 8 modes x 256^2 frames on a 3072^2 object (psi
alone is 41.9 GB), and the paper's frame size, 10000 views x 4 modes x
188^2 frames on a 1280^2 object (mixed-radix transforms).

The whole FP64 iteration is too slow for a test, so the oracle is applied
where it can be computed one piece at a time:
  * psi' of sampled views: the view update (Eq. 3 with F_c) of view j
    depends only on psi_j, P, O[window_j] and I_j;
  * O' at sampled object pixels: the oracle's object update (Eq. 5) over
    every view that covers the pixel (the other views add nothing there),
    from the GPU's psi' of those views and the old probe;
  * P' at sampled probe pixels: the oracle's probe update (Eq. 4) over all
    10000 views on 1 x 1 frames cut at the pixel (each window corner moved
    by the pixel's offset), from the GPU's psi' and the GPU's new object.
Bar: 1e-5 relative (L2 over the sampled views; per sampled pixel)."""
import sys

import numpy as np
import pytest

from oracle import dm_oracle as oracle
from paper_1808_10375_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


CASES = {
    256: dict(make=lambda: synth.flyscan_raster_256(2), shape=(10000, 8, 256, 3072),
              obj_px=[(1500, 1500), (1000, 1800), (2000, 1100), (1234, 1777), (1900, 1950)],
              probe_px=[(128, 128), (120, 140), (100, 128), (128, 160), (150, 110)]),
    188: dict(make=lambda: synth.flyscan_raster_188(3), shape=(10000, 4, 188, 1280),
              obj_px=[(640, 640), (400, 800), (900, 300), (1000, 1000), (733, 457)],
              probe_px=[(94, 94), (80, 100), (60, 94), (94, 120), (110, 70)]),
}


@pytest.mark.parametrize("frame", [256, 188])
def test_flyscan_10000_views_full_size_sampled(frame):
    from paper_1808_10375_amd import dm
    cfg = CASES[frame]
    n, m, f, o = cfg["shape"]
    say(f"case fly scan full size: {n} views x {m} modes x {f}^2, {o}^2 object")
    s = cfg["make"]()
    assert (s.n_frames, s.n_modes, s.frame) == (n, m, f) and s.obj_shape == (o, o)
    dev = torch.device("cuda:0")
    ctx = dm.DMContext(torch.from_numpy(s.I).to(dev), s.pos, torch.from_numpy(s.P0).to(dev),
                       torch.from_numpy(s.O0).to(dev), beta=s.beta)
    say(f"  tuning {ctx.tuning()}")
    ctx.iterate(1)
    psi_t, P_t, O_t, it = ctx.state()
    torch.cuda.synchronize()
    ctx.free()
    assert it == 1
    pos = np.asarray(s.pos)
    P0 = s.P0.astype(np.complex128)
    O0 = s.O0.astype(np.complex128)

    # psi' of sampled views against the oracle's view update
    js = np.array([0, 1, 4321, 5050, 9998, 9999])
    psi0 = oracle.init_views(P0, O0, pos[js])
    psi_o = oracle.view_update(psi0, P0, O0, pos[js], s.I[js].astype(np.float64), s.beta)
    psi_g = psi_t[torch.as_tensor(js, device=dev)].cpu().numpy()
    r_psi = rel(psi_g, psi_o)
    say(f"  psi' of {len(js)} sampled views: rel L2 {r_psi:.2e}")
    assert r_psi <= TOL

    # O' at sampled object pixels: the oracle's Eq. 5 over the covering views
    O_g = O_t.cpu().numpy()
    worst = 0.0
    for (y, x) in cfg["obj_px"]:
        jj = np.nonzero((pos[:, 0] <= y) & (y < pos[:, 0] + f) &
                        (pos[:, 1] <= x) & (x < pos[:, 1] + f))[0]
        psi_jj = psi_t[torch.as_tensor(jj, device=dev)].cpu().numpy()
        O_ref, _ = oracle.object_update(psi_jj, P0, O0, pos[jj])
        del psi_jj
        ref = O_ref[y, x]
        e = abs(O_g[y, x] - ref) / abs(ref)
        worst = max(worst, e)
        say(f"  O'[{y},{x}]: {len(jj)} views, rel {e:.2e}")
    assert worst <= TOL

    # P' at sampled probe pixels: the oracle's Eq. 4 over all views, on the
    # 1 x 1 frames at (u, v) with the window corners moved by (u, v)
    P_g = P_t.cpu().numpy()
    worst = 0.0
    for (u, v) in cfg["probe_px"]:
        psi_uv = psi_t[:, :, u:u + 1, v:v + 1].cpu().numpy()
        P_ref, _ = oracle.probe_update(psi_uv, O_g, P0[:, u:u + 1, v:v + 1],
                                       pos + np.array([u, v]))
        e = rel(P_g[:, u, v], P_ref[:, 0, 0])
        worst = max(worst, e)
        say(f"  P'[:, {u}, {v}]: rel {e:.2e}")
    assert worst <= TOL
    del psi_t
