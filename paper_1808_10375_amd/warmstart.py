"""Learned warm start: training pairs from the DM solver, training of the
encoder-decoder on the GPU, and the warm-versus-cold comparison.

The paper allows the initial probe and object to come from pre-existing
results (Section III).  Here the pre-existing results are DM reconstructions
of synthetic scans: a network learns to map one diffraction frame to the
object under its window, and its patches, stitched with the object update
of Eq. 5, replace the flat initial object.  Plain DM from the flat object
stays the fallback and the reference the warm start is measured against.

Every arithmetic step of the reconstruction and of the network runs in
libdm's kernels (dm.py, dmnet.py).  Host code here only prepares training
targets from reconstructed objects (phase ramp, global phase and scale
normalisation, window extraction, 2x2 binning, the probe-footprint mask) and
bookkeeps.

    python -m paper_1808_10375_amd.warmstart --out report.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import synth

FRAME = 128
NET_SIZE = FRAME // 2
MODE_WEIGHTS = [1.0, 0.5, 0.25]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# training data
# ---------------------------------------------------------------------------
def training_scan(seed: int, n_frames: int = 256, obj: int = 384) -> synth.Scan:
    """A scan of the held-out family (3 HG modes, 128x128 frames, Fermat
    spiral of 10 px mean step, 1e5 photons) on a smaller object."""
    return synth.spiral_scan(seed, n_frames, 3, MODE_WEIGHTS, frame=FRAME, obj=obj,
                             name=f"warm_train.{seed}")


def illumination(P0: np.ndarray, pos: np.ndarray, shape) -> np.ndarray:
    """sum_j sum_k |P0_k|^2 placed at every window (the Eq. 5 weights)."""
    D = np.sum(np.abs(P0.astype(np.complex128)) ** 2, axis=0)
    f = D.shape[0]
    acc = np.zeros(shape)
    for y, x in pos:
        acc[y:y + f, x:x + f] += D
    return acc


def normalise_object(O: np.ndarray, weight: np.ndarray, floor: float = 0.01) -> np.ndarray:
    """Remove the global factor c of the (P, O) -> (cP, O/c) ambiguity: over
    well-lit pixels the mean of O becomes real and positive and its RMS
    amplitude 1 (the scale the flat initial object assumes).  Pixels whose
    illumination is below `floor` of the peak are not determined by the data
    (their Eq. 5 denominators are tiny) and are set to the flat value 1."""
    lit = weight >= 0.1 * weight.max()
    c = np.mean(O[lit])
    rms = math.sqrt(float(np.mean(np.abs(O[lit]) ** 2)))
    out = O * (np.conj(c) / abs(c)) / rms
    out[weight < floor * weight.max()] = 1.0
    return out


def remove_phase_ramp(O: np.ndarray, weight: np.ndarray) -> np.ndarray:
    """Remove the linear phase ramp that the data leave free (P e^{iq.r} with
    O e^{-iq.r} models the same intensities): q is the mean phase step
    between neighbouring well-lit pixels along each axis, which a zero-mean
    random phase field does not bias."""
    lit = weight >= 0.1 * weight.max()
    gx = np.sum((O[:, 1:] * np.conj(O[:, :-1]))[lit[:, 1:] & lit[:, :-1]])
    gy = np.sum((O[1:, :] * np.conj(O[:-1, :]))[lit[1:, :] & lit[:-1, :]])
    y, x = np.mgrid[0:O.shape[0], 0:O.shape[1]]
    return O * np.exp(-1j * (np.angle(gx) * x + np.angle(gy) * y))


def patch_targets(O: np.ndarray, pos: np.ndarray, f: int = FRAME) -> np.ndarray:
    """[N][2][f/2][f/2] float32: 2x2 averages of the object under each window."""
    out = np.empty((len(pos), 2, f // 2, f // 2), dtype=np.float32)
    for j, (y, x) in enumerate(pos):
        w = O[y:y + f, x:x + f].reshape(f // 2, 2, f // 2, 2).mean(axis=(1, 3))
        out[j, 0] = w.real
        out[j, 1] = w.imag
    return out


def lit_mask(P0: np.ndarray, level: float = 0.01) -> np.ndarray:
    """[f/2][f/2] weights in [0, 1] of the window's pixels in what one frame
    determines: sum_k |P0_k|^2 (2x2 averages) over `level` of its peak,
    clipped at 1.  Outside the probe's footprint a frame carries nothing
    about the object, and the Eq. 5 stitch weights it by |P0|^2 anyway."""
    d = np.sum(np.abs(P0.astype(np.complex128)) ** 2, axis=0)
    f = d.shape[0]
    d = d.reshape(f // 2, 2, f // 2, 2).mean(axis=(1, 3))
    return np.minimum(1.0, d / (level * d.max()))


def masked_targets(O: np.ndarray, pos: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Patch targets 1 + mask * (patch - 1): the object where the probe lights
    the window, the flat value 1 where it does not."""
    t = patch_targets(O, pos)
    t[:, 0] = 1.0 + mask * (t[:, 0] - 1.0)
    t[:, 1] = mask * t[:, 1]
    return t


def make_pairs(seeds, n_iter: int = 100, n_frames: int = 256, obj: int = 384,
               group: int = 16, net=None, device="cuda:0", targets: str = "dm-masked"):
    """(x [P][1][64][64], target [P][2][64][64]) on the device for the scans of
    `seeds`.  targets="dm-masked" (the default): the object that `n_iter` DM
    iterations reconstruct from the cold start (`group` scans per batch),
    its free phase ramp removed (remove_phase_ramp), in the gauge of the flat
    start (normalise_object) and masked to the probe's footprint
    (masked_targets).  targets="dm": the same reconstruction, normalised but
    neither de-ramped nor masked.  targets="truth": the synthetic scan's own
    object, normalised and masked."""
    import torch
    from .dm import DMBatch
    xs, ts = [], []
    for g0 in range(0, len(seeds), group):
        t0 = time.time()
        scans = [training_scan(s, n_frames, obj) for s in seeds[g0:g0 + group]]
        t1 = time.time()
        if targets.startswith("dm"):
            batch = DMBatch([dict(I=s.I, pos=s.pos, P0=s.P0, O0=s.O0) for s in scans],
                            device=device)
            batch.iterate(n_iter)
        for k, s in enumerate(scans):
            w = illumination(s.P0, s.pos, s.O0.shape)
            if targets == "dm":
                O = batch.object(k).cpu().numpy().astype(np.complex128)
                t = patch_targets(normalise_object(O, w), s.pos)
            elif targets == "dm-masked":
                O = batch.object(k).cpu().numpy().astype(np.complex128)
                O = normalise_object(remove_phase_ramp(O, w), w)
                t = masked_targets(O, s.pos, lit_mask(s.P0))
            else:
                O = s.O_true.astype(np.complex128)
                t = masked_targets(normalise_object(O, w), s.pos, lit_mask(s.P0))
            I = torch.as_tensor(s.I).to(device)
            xs.append(net.preprocess(I))
            ts.append(torch.as_tensor(t).to(device))
        if targets.startswith("dm"):
            batch.free()
        log(f"pairs: scans {g0}..{g0 + len(scans) - 1}: generate {t1 - t0:.1f} s, "
            f"targets {time.time() - t1:.1f} s")
    return torch.cat(xs), torch.cat(ts)


# ---------------------------------------------------------------------------
# training
# ---------------------------------------------------------------------------
def train(net, x, t, x_val, t_val, epochs: int, batch: int, seed: int = 0,
          log_every: int = 50, max_seconds: float = 1e30):
    """Adam over shuffled minibatches; returns the history of losses.  Stops
    early, at the end of a step, once `max_seconds` have passed."""
    import torch
    gen = torch.Generator(device="cpu").manual_seed(seed)
    n = x.shape[0]
    hist = []
    step = 0
    t_start = time.time()
    stopped = False
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(x.device)
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            want = (step % log_every == 0)
            loss = net.train_step(x[idx], t[idx], want_loss=want)
            if want:
                hist.append({"step": step, "loss": loss})
                log(f"train step {step} epoch {ep} loss {loss:.5f} "
                    f"({time.time() - t_start:.0f} s)")
            step += 1
            if time.time() - t_start > max_seconds:
                stopped = True
                break
        vl = validation_loss(net, x_val, t_val, batch)
        hist.append({"step": step, "epoch": ep, "val_loss": vl})
        log(f"epoch {ep}: validation loss {vl:.5f}")
        if stopped:
            log(f"training stopped by the time limit after {step} steps")
            break
    return hist, step, time.time() - t_start


def validation_loss(net, x, t, batch):
    tot, cnt = 0.0, 0
    for b0 in range(0, x.shape[0] - batch + 1, batch):
        loss, _ = net.loss_grad(x[b0:b0 + batch], t[b0:b0 + batch])
        tot += loss
        cnt += 1
    return tot / max(cnt, 1)


def predict_patches(net, I, batch: int):
    """Complex patches [N][F][F] for the frames I [N][F][F] (device)."""
    import torch
    out = torch.empty((I.shape[0], I.shape[1], I.shape[2]), dtype=torch.complex64,
                      device=I.device)
    for b0 in range(0, I.shape[0], batch):
        x = net.preprocess(I[b0:b0 + batch])
        out[b0:b0 + batch] = net.patches(net.forward(x))
    return out


# ---------------------------------------------------------------------------
# warm versus cold
# ---------------------------------------------------------------------------
def object_error(O: np.ndarray, O_true: np.ndarray, weight: np.ndarray) -> float:
    """Relative error of O against the truth over well-lit pixels, after the
    best complex scale factor."""
    lit = weight >= 0.1 * weight.max()
    a, b = O[lit].astype(np.complex128), O_true[lit].astype(np.complex128)
    c = np.vdot(a, b) / np.vdot(a, a)
    return float(np.linalg.norm(c * a - b) / np.linalg.norm(b))


def first_at_or_below(errs, level):
    for k, e in enumerate(errs):
        if e <= level:
            return k + 1
    return None


def compare(net, scans, n_iter: int, batch: int, device="cuda:0", checkpoints=(1, 10, 50)):
    """Run the scans as one batch from the flat object (cold) and from the
    stitched patches (warm), with the same initial probe; report the error
    histories and iterations to fixed error levels."""
    import torch
    from .dm import DMBatch, DM_FLAG_GRAPH
    res = {}
    weights = [illumination(s.P0, s.pos, s.O0.shape) for s in scans]
    # the network runs on the stream it was created on (the default one):
    # all patches are made there before the batch's own stream starts
    torch.cuda.synchronize(device)
    t0 = time.time()
    patches = [predict_patches(net, torch.as_tensor(s.I).to(device), batch) for s in scans]
    torch.cuda.synchronize(device)
    t_net = time.time() - t0
    stream = torch.cuda.Stream(device=device)
    for form in ("cold", "warm"):
        with torch.cuda.stream(stream):
            b = DMBatch([dict(I=s.I, pos=s.pos, P0=s.P0, O0=s.O0) for s in scans],
                        flags=DM_FLAG_GRAPH, stream=stream, device=device)
            t0 = time.time()
            if form == "warm":
                for k in range(len(scans)):
                    b.warm_start(k, patches[k])
                stream.synchronize()
            t_init = time.time() - t0 + (t_net if form == "warm" else 0.0)
            obj_err = {0: [object_error(b.object(k).cpu().numpy(), s.O_true, weights[k])
                           for k, s in enumerate(scans)]}
            done = 0
            for c in list(checkpoints) + [n_iter]:
                if c > done:
                    b.iterate(c - done)
                    done = c
                    obj_err[c] = [object_error(b.object(k).cpu().numpy(), s.O_true, weights[k])
                                  for k, s in enumerate(scans)]
            errs = [[e["eps_probe"] for e in b.error_history(k)] for k in range(len(scans))]
            b.free()
        res[form] = {"err": errs, "obj_err": obj_err, "init_s": t_init}
    levels = (1e-3, 1e-2, 2e-2, 3e-2, 1e-1)
    out = {"n_iter": n_iter, "scans": len(scans), "per_scan": []}
    for k in range(len(scans)):
        ec, ew = res["cold"]["err"][k], res["warm"]["err"][k]
        row = {
            "frames": int(scans[k].I.shape[0]),
            "err_at": {f: {str(i): e[i - 1] for i in (1, 2, 3, 5, 10, 20, 50, n_iter)
                           if i <= len(e)}
                       for f, e in (("cold", ec), ("warm", ew))},
            "iters_to": {f"{lv:g}": {"cold": first_at_or_below(ec, lv),
                                     "warm": first_at_or_below(ew, lv)} for lv in levels},
            # err <= 1e-3 is out of reach of Poisson data: the level is 1.1x the
            # cold start's err after n_iter iterations (the cold run stands in for
            # the converged reference on these scans)
            "iters_to_1.1x_final": {"level": 1.1 * ec[-1],
                                    "cold": first_at_or_below(ec, 1.1 * ec[-1]),
                                    "warm": first_at_or_below(ew, 1.1 * ec[-1])},
            "object_error": {f: {str(c): res[f]["obj_err"][c][k] for c in res[f]["obj_err"]}
                             for f in ("cold", "warm")},
        }
        out["per_scan"].append(row)
    out["warm_init_s"] = res["warm"]["init_s"]

    def med_iters(lv, f):
        v = [r["iters_to"][f"{lv:g}"][f] for r in out["per_scan"]]
        reached = [x for x in v if x is not None]
        return {"median": float(np.median(reached)) if reached else None,
                "reached": len(reached)}
    fin = {f: [r["iters_to_1.1x_final"][f] for r in out["per_scan"]] for f in ("cold", "warm")}
    out["iters_to_1.1x_final"] = {
        "median": {f: float(np.median([v if v is not None else n_iter + 1 for v in fin[f]]))
                   for f in fin},
        "saved_per_scan": [(c - w) if (c is not None and w is not None) else None
                           for c, w in zip(fin["cold"], fin["warm"])]}
    out["median"] = {
        "iters_to": {f"{lv:g}": {f: med_iters(lv, f) for f in ("cold", "warm")}
                     for lv in levels},
        "err_at": {f: {i: float(np.median([r["err_at"][f][i] for r in out["per_scan"]]))
                       for i in out["per_scan"][0]["err_at"][f]}
                   for f in ("cold", "warm")}}
    out["median_object_error"] = {
        f: {str(c): float(np.median(res[f]["obj_err"][c])) for c in res[f]["obj_err"]}
        for f in ("cold", "warm")}
    return out


def layer_shapes(c0: int = 32, levels: int = 4):
    """(cout, cin, k) of every convolution in the parameter order of dmnet.h."""
    ch = [c0 << l for l in range(levels)]
    out, prev = [], 1
    for l in range(levels):
        out += [(ch[l], prev, 3), (ch[l], ch[l], 3)]
        prev = ch[l]
    for l in range(levels - 2, -1, -1):
        out += [(ch[l], ch[l + 1] + ch[l], 3), (ch[l], ch[l], 3)]
    out.append((2, ch[0], 1))
    return out


def initial_params(seed: int, c0: int = 32, levels: int = 4) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, flat float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for co, ci, k in layer_shapes(c0, levels):
        parts.append((rng.standard_normal(co * ci * k * k) * math.sqrt(2.0 / (ci * k * k))))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train-scans", type=int, default=96)
    ap.add_argument("--val-scans", type=int, default=8)
    ap.add_argument("--train-frames", type=int, default=256)
    ap.add_argument("--train-obj", type=int, default=384)
    ap.add_argument("--dm-iters", type=int, default=100)
    ap.add_argument("--targets", choices=["dm-masked", "dm", "truth"], default="dm-masked")
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-iters", type=int, default=200)
    ap.add_argument("--eval-scans", type=int, default=16)
    ap.add_argument("--eval-sizes", type=str, default="",
                    help="comma-separated frame counts instead of U{200..3000}")
    ap.add_argument("--out", type=str, default="")
    ap.add_argument("--save-params", type=str, default="")
    ap.add_argument("--load-params", type=str, default="")
    ap.add_argument("--max-train-s", type=float, default=600.0)
    a = ap.parse_args(argv)
    import torch
    from .dmnet import DMNet
    dev = "cuda:0"
    net = DMNet(a.batch, size=NET_SIZE, base_ch=32, levels=4, lr=a.lr, device=dev)
    report = {"network": {"levels": 4, "channels": [32, 64, 128, 256],
                          "params": net.n_params, "input": [1, NET_SIZE, NET_SIZE],
                          "weights": "bf16 (fp32 master)", "accumulate": "fp32"}}
    if a.load_params:
        net.set_params(np.load(a.load_params, allow_pickle=False))
        report["training"] = {"loaded": a.load_params}
    else:
        net.set_params(initial_params(10000))
        t0 = time.time()
        seeds = list(range(10000, 10000 + a.train_scans))
        vseeds = list(range(20000, 20000 + a.val_scans))
        x, t = make_pairs(seeds, a.dm_iters, a.train_frames, a.train_obj, net=net, device=dev,
                          targets=a.targets)
        xv, tv = make_pairs(vseeds, a.dm_iters, a.train_frames, a.train_obj, net=net,
                            device=dev, targets=a.targets)
        t_pairs = time.time() - t0
        log(f"pairs: {x.shape[0]} training, {xv.shape[0]} validation ({t_pairs:.0f} s)")
        v0 = validation_loss(net, xv, tv, a.batch)
        hist, steps, t_train = train(net, x, t, xv, tv, a.epochs, a.batch,
                                     max_seconds=a.max_train_s)
        report["training"] = {
            "scans": a.train_scans, "frames_per_scan": a.train_frames,
            "object": a.train_obj, "targets": a.targets,
            "dm_iters": a.dm_iters if a.targets.startswith("dm") else None, "pairs": int(x.shape[0]),
            "validation_pairs": int(xv.shape[0]), "epochs": a.epochs, "batch": a.batch,
            "lr": a.lr, "steps": steps, "pairs_s": t_pairs, "train_s": t_train,
            "samples_per_s": steps * a.batch / t_train, "val_loss_initial": v0,
            "history": hist}
        # a target that predicts the flat initial object (1 + 0i) everywhere
        flat = torch.zeros_like(tv)
        flat[:, 0] = 1.0
        report["training"]["val_loss_flat_object"] = float(torch.mean((flat - tv) ** 2))
        del x, t
        if a.save_params:
            np.save(a.save_params, net.params().cpu().numpy())
    sizes = ([int(v) for v in a.eval_sizes.split(",")] if a.eval_sizes
             else synth.uneven_scan_sizes(1000, a.eval_scans))
    t0 = time.time()
    scans = synth.uneven_spirals_128(1000, len(sizes), sizes)
    log(f"evaluation scans generated ({time.time() - t0:.0f} s): {sizes}")
    report["evaluation"] = compare(net, scans, a.eval_iters, a.batch, dev)
    line = json.dumps(report)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(line + "\n")
    print(json.dumps({"median": report["evaluation"]["median"],
                      "iters_to_1.1x_final": report["evaluation"]["iters_to_1.1x_final"],
                      "median_object_error": report["evaluation"]["median_object_error"]}))


if __name__ == "__main__":
    main()
