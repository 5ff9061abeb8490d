"""Training and use of the CNN surrogate of the subimage stiffness.

The surrogate stands in for the FFT solve of Sec. 4 on each padded
subimage: a network maps the one-hot phase labels of the n^3 core to the 21
independent components of the subimage's stiffness C_R.  Training data are
subimages that the library's own FFT solver homogenizes (the same padding
p as at use), so the solver remains the reference for the network's error, and
at use a gate sends doubtful subimages back to it.

Everything numeric runs in the HIP library (network kernels, solver,
gather); this module only arranges data and calls the bindings.  Label
boxes and targets stay in device memory; the 48 symmetries of the cube
(axis permutations and reflections) multiply the training set, with the
stiffness transformed alongside each box.

Command line (trains and saves two networks for the spread gate):
    python -m paper_2208_02320_amd.surrogate --out DIR [--images K ...]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import time
from dataclasses import dataclass, field

import numpy as np

from . import hh, synth

UPPER = [(i, j) for i in range(6) for j in range(i, 6)]
VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]  # index pairs of 11,22,33,23,13,12
WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


# ---------------------------------------------------------------------------
# symmetries of the cube
# ---------------------------------------------------------------------------
def cube_symmetries():
    """The 48 signed axis permutations (p, s): x'_i = s_i x_{p(i)}, with
    physical axes 0 = x, 1 = y, 2 = z."""
    out = []
    for p in itertools.permutations(range(3)):
        for s in itertools.product((1, -1), repeat=3):
            out.append((tuple(p), tuple(s)))
    return out


def sym_matrix(p, s):
    Q = np.zeros((3, 3))
    for i in range(3):
        Q[i, p[i]] = s[i]
    return Q


def _voigt_to_tensor(C):
    T = np.zeros((3, 3, 3, 3))
    for I, (i, j) in enumerate(VOIGT):
        for J, (k, l) in enumerate(VOIGT):
            for a, b in ((i, j), (j, i)):
                for c, d in ((k, l), (l, k)):
                    T[a, b, c, d] = C[I, J]
    return T


def _tensor_to_voigt(T):
    return np.array([[T[i, j, k, l] for (k, l) in VOIGT] for (i, j) in VOIGT])


def c21_transform(p, s):
    """21 x 21 matrix taking the upper-triangle stiffness of a material to
    that of the material mapped by x -> Q x (C'_ijkl = Q_ia Q_jb Q_kc Q_ld C_abcd)."""
    Q = sym_matrix(p, s)
    T = np.zeros((21, 21))
    for m, (a, b) in enumerate(UPPER):
        C = np.zeros((6, 6))
        C[a, b] = C[b, a] = 1.0
        R = np.einsum("ia,jb,kc,ld,abcd->ijkl", Q, Q, Q, Q, _voigt_to_tensor(C))
        V = _tensor_to_voigt(R)
        T[:, m] = [V[i, j] for (i, j) in UPPER]
    return T


def transform_boxes(boxes, p, s):
    """Apply x -> Q x to label boxes (..., z, y, x) (a torch tensor or a
    numpy array): new physical axis i is old axis p(i), reversed where s_i < 0."""
    nd = boxes.ndim
    lead = list(range(nd - 3))
    # tensor dim of physical axis a is nd - 1 - a
    perm = lead + [nd - 1 - p[nd - 1 - d] for d in range(nd - 3, nd)]
    flips = [d for d in range(nd - 3, nd) if s[nd - 1 - d] < 0]
    if type(boxes).__module__.startswith("torch"):
        out = boxes.permute(*perm)
        if flips:
            out = out.flip(flips)
        return out.contiguous()
    out = np.transpose(boxes, perm)
    if flips:
        out = np.flip(out, axis=flips)
    return np.ascontiguousarray(out)


def mandel_weights():
    """Weights w such that sum w c^2 is the squared Frobenius norm of the
    Mandel-scaled matrix (the tensor norm)."""
    w = []
    for (i, j) in UPPER:
        f = (np.sqrt(2.0) if i >= 3 else 1.0) * (np.sqrt(2.0) if j >= 3 else 1.0)
        w.append(f * f * (1.0 if i == j else 2.0))
    return np.asarray(w)


def rel_error21(c, ref):
    """Per-item relative tensor-norm error of (m, 21) stiffnesses."""
    w = mandel_weights()
    c, ref = np.atleast_2d(c), np.atleast_2d(ref)
    return np.sqrt(((c - ref) ** 2 * w).sum(-1) / (ref ** 2 * w).sum(-1))


# ---------------------------------------------------------------------------
# data
# ---------------------------------------------------------------------------
@dataclass
class Dataset:
    boxes: object                 # device uint8 tensor (m, b, b, b)
    c21: np.ndarray               # (m, 21) FFT-solver stiffness of each padded box
    n: int                        # core edge
    pad: int
    seeds: list = field(default_factory=list)
    solve_seconds: float = 0.0

    @property
    def box(self):
        return self.n + 2 * self.pad

    def window(self, edge):
        """Offset of a network input window of ``edge`` in the boxes: the
        core (edge n) or the whole box (edge n + 2 pad)."""
        if edge == self.n:
            return self.pad
        if edge == self.box:
            return 0
        raise ValueError("network input edge %d fits neither the core nor the box" % edge)

    def split(self, count):
        """(first m - count items, last count items)."""
        m = self.c21.shape[0]
        a = Dataset(self.boxes[:m - count], self.c21[:m - count], self.n, self.pad, self.seeds)
        b = Dataset(self.boxes[m - count:], self.c21[m - count:], self.n, self.pad, self.seeds)
        return a, b


def label_images(ctx, seeds, size, n_sub, pad, sigma=2.0, tol=1e-5, log=print, labels=None):
    """Cut four-phase device images (one per seed, edge ``size``) into padded
    subimages and homogenize each with the FFT solver.  With ``labels`` (the
    c21 array of an earlier call with the same arguments) the images are only
    regenerated and cut: the device generator is deterministic."""
    import torch
    boxes, c21 = [], []
    t_solve = 0.0
    per = (size // n_sub) ** 3
    if labels is not None and labels.shape != (per * len(seeds), 21):
        raise ValueError("cached labels do not match the image recipe")
    for k, seed in enumerate(seeds):
        img = synth.four_phase_device(size, sigma=sigma, seed=seed, device="cuda:%d" % ctx.device)
        torch.cuda.synchronize()
        t0 = time.time()
        if labels is None:
            _, Cs, rep = ctx.hierarchical(img, synth.FOUR_PHASE["phases"], n_sub, pad, tol=tol)
            c21.append(Cs.copy())
        t_solve += time.time() - t0
        boxes.append(ctx.gather_subimages(img, n_sub, pad))
        del img
        if log and labels is None:
            log("labelled image %d/%d (seed %d): %d subimages, %.1fs" % (k + 1, len(seeds), seed, per,
                                                                      time.time() - t0))
    c21 = labels if labels is not None else np.concatenate(c21)
    return Dataset(torch.cat(boxes), c21, n_sub, pad, list(seeds), t_solve)


def fraction_stats(data, edge=None, nch=8):
    """Mean and inverse standard deviation of each label's fraction in the
    input windows of the data set (scale 0 for labels that never vary)."""
    import torch
    n = edge or data.n
    p = data.window(n)
    core = data.boxes[:, p:p + n, p:p + n, p:p + n]
    f = torch.stack([(core == c).float().mean(dim=(1, 2, 3)) for c in range(nch)], dim=1).double().cpu().numpy()
    mu, sd = f.mean(axis=0), f.std(axis=0)
    return mu, np.where(sd > 1e-6, 1.0 / np.maximum(sd, 1e-6), 0.0)


def interface_densities(boxes, offset, edge, chunk=256):
    """Interface density of the edge^3 window at (offset, offset, offset) of
    each box: the fraction of its face-adjacent voxel pairs (inside the
    window, along x, y and z) whose labels differ (device tensors in, FP64
    numpy out)."""
    import torch
    out = []
    pairs = 3.0 * edge * edge * (edge - 1)
    for a in range(0, boxes.shape[0], chunk):
        w = boxes[a:a + chunk, offset:offset + edge, offset:offset + edge, offset:offset + edge]
        d = ((w[..., 1:] != w[..., :-1]).sum(dim=(1, 2, 3)) + (w[:, :, 1:, :] != w[:, :, :-1, :]).sum(dim=(1, 2, 3)) +
             (w[:, 1:] != w[:, :-1]).sum(dim=(1, 2, 3)))
        out.append(d.to(torch.float64).cpu().numpy() / pairs)
    return np.concatenate(out)


def interface_stats(data, edge):
    """Mean and inverse standard deviation of the training windows'
    interface density (the gate's texture test)."""
    d = interface_densities(data.boxes, data.window(edge), edge)
    return float(d.mean()), float(1.0 / max(d.std(), 1e-6))


def symmetric_scaling(c21, syms=None):
    """Mean and standard deviation per component over the data set and all
    its symmetric images (floor 1e-3 of the largest)."""
    syms = syms or cube_symmetries()
    allc = np.concatenate([c21 @ c21_transform(p, s).T for p, s in syms])
    mean = allc.mean(axis=0)
    sd = allc.std(axis=0)
    return mean, np.maximum(sd, 1e-3 * sd.max())


# ---------------------------------------------------------------------------
# training
# ---------------------------------------------------------------------------
def train(ctx, data, nphase, epochs=20, batch=32, lr=1e-3, lr_final=2e-5, seed=0, augment=True, log=print,
          log_every=200, val=None, window="core"):
    """Train a network on ``data`` whose input is the core of each box
    (``window="core"``) or the whole box; returns (net, history)."""
    import torch
    syms = cube_symmetries() if augment else [((0, 1, 2), (1, 1, 1))]
    mats = [c21_transform(p, s) for p, s in syms]
    mean, scale = symmetric_scaling(data.c21, syms)
    edge = data.n if window == "core" else data.box
    offset = data.window(edge)
    net = hh.Net(ctx, nphase, edge, seed=seed)
    net.set_scaling(mean, scale)
    net.set_fraction_scaling(*fraction_stats(data, edge))
    net.set_interface_stats(*interface_stats(data, edge))
    dev = "cuda:%d" % ctx.device
    m = data.c21.shape[0]
    steps_per_epoch = max(1, m // batch)
    total = epochs * steps_per_epoch
    rng = np.random.default_rng(seed)
    hist = []
    step = 0
    t0 = time.time()
    for ep in range(epochs):
        order = rng.permutation(m)
        run = 0.0
        for j in range(steps_per_epoch):
            idx = order[j * batch:(j + 1) * batch]
            k = int(rng.integers(len(syms)))
            p, s = syms[k]
            ti = torch.from_numpy(idx).to(dev)
            lab = transform_boxes(data.boxes.index_select(0, ti), p, s)
            tgt = (data.c21[idx] @ mats[k].T - mean) / scale
            tdev = torch.from_numpy(tgt.astype(np.float32)).to(dev)
            frac = step / max(1, total - 1)
            rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * frac))
            loss = net.train_step(lab, tdev, rate, offset=offset)
            run += loss
            step += 1
            if log and log_every and step % log_every == 0:
                log("step %d/%d epoch %d loss %.4e lr %.2e (%.0fs)" % (step, total, ep, loss, rate,
                                                                     time.time() - t0))
        rec = dict(epoch=ep, loss=run / steps_per_epoch, seconds=time.time() - t0)
        if val is not None:
            e = rel_error21(predict(net, val), val.c21)
            rec.update(val_mean=float(e.mean()), val_p95=float(np.quantile(e, 0.95)))
        hist.append(rec)
        if log:
            log("epoch %d: %s" % (ep, json.dumps(rec)))
    return net, hist


def predict(net, data, chunk=512):
    off = data.window(net.n)
    out = []
    for a in range(0, data.c21.shape[0], chunk):
        out.append(net.predict(data.boxes[a:a + chunk], offset=off))
    return np.concatenate(out)


def save(net, path, meta=None):
    mean, scale = net.get_scaling()
    fmu, fsc = net.get_fraction_scaling()
    imu, isc = net.get_interface_stats()
    np.savez_compressed(path, params=net.get_params(), mean=mean, scale=scale, fmu=fmu, fsc=fsc,
                        imu=np.float64(imu), isc=np.float64(isc), n=net.n, nphase=net.nphase,
                        meta=json.dumps(meta or {}))


def add_gate_stats(ctx, paths, out_dir, log=print):
    """Interface statistics for networks saved before the texture test
    existed: the training windows are regenerated from the images named in
    each file's record (device generator, same seeds and partition) and the
    file is written again to out_dir with imu and isc added; every other
    array is kept as it was."""
    import torch
    cache = {}
    for path in paths:
        with np.load(path, allow_pickle=False) as z:
            arrays = {k: z[k] for k in z.files}
        meta = json.loads(str(arrays["meta"]))
        edge = int(arrays["n"])
        key = (tuple(meta["images"]), meta["size"], meta["n"], meta["pad"], edge)
        if key not in cache:
            d = []
            for seed in meta["images"]:
                img = synth.four_phase_device(meta["size"], sigma=2.0, seed=seed, device="cuda:%d" % ctx.device)
                boxes = ctx.gather_subimages(img, meta["n"], meta["pad"])
                off = meta["pad"] if edge == meta["n"] else 0
                d.append(interface_densities(boxes, off, edge))
                del img, boxes
                torch.cuda.empty_cache()
            d = np.concatenate(d)
            cache[key] = (float(d.mean()), float(1.0 / max(d.std(), 1e-6)), d.size)
        imu, isc, cnt = cache[key]
        arrays["imu"], arrays["isc"] = np.float64(imu), np.float64(isc)
        os.makedirs(out_dir, exist_ok=True)
        out = os.path.join(out_dir, os.path.basename(path))
        np.savez_compressed(out, **arrays)
        if log:
            log("%s: interface density %.5f +- %.5f over %d training windows -> %s" % (path, imu, 1.0 / isc, cnt, out))


def load(ctx, path):
    """The network of a saved file, read by the library (hh_net_load); its
    training record (``meta``) is read here."""
    net = hh.Net.load(ctx, path)
    with np.load(path, allow_pickle=False) as z:
        net.meta = json.loads(str(z["meta"]))
    return net


def default_weights(n=64, pad=8, directory=None):
    """Paths of the two shipped networks for four-phase subimages."""
    return [os.path.join(directory or WEIGHTS_DIR, "four_phase_n%d_p%d_%s.npz" % (n, pad, t)) for t in ("a", "b")]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=WEIGHTS_DIR)
    ap.add_argument("--images", type=int, default=40, help="training images (seeds 10000, 10001, ...)")
    ap.add_argument("--val-images", type=int, default=2, help="validation images (seeds 20000, ...)")
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--pad", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--seeds", default="1,2", help="one network per seed")
    ap.add_argument("--window", choices=("core", "box"), default="core")
    ap.add_argument("--labels", default=None, help="npz cache of the FFT labels (read if present, else written)")
    ap.add_argument("--gate-stats", nargs="*", default=None,
                    help="add interface statistics to these saved networks (written to --out)")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    ctx = hh.Context(0)
    if a.gate_stats:
        add_gate_stats(ctx, a.gate_stats, a.out, log=log)
        return
    seeds = list(range(10000, 10000 + a.images))
    vseeds = list(range(20000, 20000 + a.val_images))
    cached = None
    if a.labels and os.path.exists(a.labels):
        z = np.load(a.labels, allow_pickle=False)
        key = [a.size, a.n, a.pad, a.images, a.val_images]
        if list(z["key"]) != key or float(z["tol"]) != a.tol:
            raise SystemExit("label cache %s was made for another recipe" % a.labels)
        cached = (z["train"], z["val"])
        log("labels from %s" % a.labels)
    data = label_images(ctx, seeds, a.size, a.n, a.pad, tol=a.tol, log=log,
                        labels=None if cached is None else cached[0])
    val = label_images(ctx, vseeds, a.size, a.n, a.pad, tol=a.tol, log=log,
                       labels=None if cached is None else cached[1])
    if a.labels and cached is None:
        np.savez_compressed(a.labels, train=data.c21, val=val.c21, tol=a.tol,
                            key=np.array([a.size, a.n, a.pad, a.images, a.val_images]))
    os.makedirs(a.out, exist_ok=True)
    for sd in [int(x) for x in a.seeds.split(",")]:
        net, hist = train(ctx, data, 4, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=sd, log=log, val=val,
                          window=a.window)
        err = rel_error21(predict(net, val), val.c21)
        meta = dict(images=seeds, val_images=vseeds, size=a.size, n=a.n, pad=a.pad, window=a.window,
                    epochs=a.epochs, batch=a.batch, lr=a.lr, tol=a.tol, seed=sd, items=int(data.c21.shape[0]),
                    val_mean=float(err.mean()), val_p95=float(np.quantile(err, 0.95)), history=hist)
        path = os.path.join(a.out, "four_phase_n%d_p%d_%s_s%d.npz" % (a.n, a.pad, a.window, sd))
        save(net, path, meta)
        log("saved %s: validation error mean %.3e p95 %.3e" % (path, err.mean(), np.quantile(err, 0.95)))
        net.close()


if __name__ == "__main__":
    main()
