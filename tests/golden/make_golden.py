"""Writes the stored expected values used by the GPU parity tests.

Calls only the FP64 CPU oracle (oracle/) and the seeded input generator.
Usage:  python tests/golden/make_golden.py four_phase_256
        python tests/golden/make_golden.py hier_512_items [jobs]
        python tests/golden/make_golden.py uneven_2048_items [jobs]
        python tests/golden/make_golden.py paper_pores_16
        python tests/golden/make_golden.py study_48 [jobs]
The sampled workloads solve their items in ``jobs`` processes (one FFT
thread each).
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import galerkin as g, hier  # noqa: E402
from paper_2208_02320_amd import synth  # noqa: E402


def four_phase_256():
    """256^3 four-phase image (seed 1, sigma 2), six unit loads, CG to 1e-9."""
    lab = synth.four_phase(256, sigma=2.0, seed=1)
    t = time.time()
    r = g.homogenize(g.IsotropicMedium(lab, synth.FOUR_PHASE["phases"]), tol=1e-9, form="sym6")
    out = dict(image="synth.four_phase(256, sigma=2.0, seed=1)", tol=1e-9, form="sym6",
               C=r.C.tolist(), C_sym=r.C_sym.tolist(), iters=r.iters, seconds=time.time() - t)
    json.dump(out, open(os.path.join(HERE, "four_phase_256_seed1.json"), "w"), indent=1)


def _pool_map(fn, args, jobs):
    if jobs <= 1:
        return [fn(a) for a in args]
    with mp.get_context("fork").Pool(jobs) as pool:
        return pool.map(fn, args, chunksize=1)


_HIER = {}


def _hier_item(i):
    g.set_workers(1)
    lab = _HIER["lab"]
    origin = hier.partition(lab, 64)[i]
    t = time.time()
    box = hier.padded_box(lab, origin, 64, 8)
    r = g.homogenize(g.IsotropicMedium(box, synth.FOUR_PHASE["phases"]),
                     region=(8, 8, 8, 72, 72, 72), tol=1e-9, form="sym6")
    print("item", i, time.time() - t, flush=True)
    return dict(index=i, origin=list(origin), C=r.C.tolist(), C_sym=r.C_sym.tolist(),
                iters=r.iters, seconds=time.time() - t)


def hier_512_items(count=32, jobs=1):
    """Sampled subimages of the 512^3 four-phase image (seed 2) cut with
    n = 64 and 8 voxels of padding (80^3 boxes), homogenized over the
    central 64^3; items drawn without replacement over the image."""
    lab = synth.four_phase(512, sigma=2.0, seed=2)
    _HIER["lab"] = lab
    origins = hier.partition(lab, 64)
    rng = np.random.default_rng(0)
    pick = sorted(rng.choice(len(origins), size=count, replace=False).tolist())
    items = _pool_map(_hier_item, pick, jobs)
    out = dict(image="synth.four_phase(512, sigma=2.0, seed=2)", n=64, pad=8, tol=1e-9,
               form="sym6", items=items)
    json.dump(out, open(os.path.join(HERE, "four_phase_512_n64_p8_items.json"), "w"), indent=1)


def _uneven_item(i):
    g.set_workers(1)
    t = time.time()
    it = synth.uneven_batch(2048, seed=1234)[i]
    lab = synth.item_image(it)
    r = g.homogenize(g.IsotropicMedium(lab, it["phases"]), tol=1e-9, form="sym6")
    print("item", i, it["size"], time.time() - t, flush=True)
    return dict(index=i, size=it["size"], C=r.C.tolist(), C_sym=r.C_sym.tolist(), iters=r.iters,
                seconds=time.time() - t)


def uneven_2048_items(per_size=8, jobs=1):
    """Stratified sample of the uneven batch recipe (2048 items, sizes 32, 48,
    64, 96, seed 1234): the first ``per_size`` items of each size, six loads,
    whole box."""
    recipe = synth.uneven_batch(2048, seed=1234)
    picked = []
    for size in (32, 48, 64, 96):
        picked += [i for i, it in enumerate(recipe) if it["size"] == size][:per_size]
    items = _pool_map(_uneven_item, picked, jobs)
    out = dict(recipe="synth.uneven_batch(2048, seed=1234)", tol=1e-9, form="sym6", items=items)
    json.dump(out, open(os.path.join(HERE, "uneven_2048_items.json"), "w"), indent=1)


def paper_pores_16():
    """The paper's two phases of Sec. 2 at full contrast: quartz (K 36, G 45
    GPa) and pores of 1e-5 GPa, on a 16^3 image at 20 % porosity (sigma 1.5,
    seed 0); six unit loads, CG to 1e-9 (several thousand iterations)."""
    lab = synth.two_phase(16, 0.2, 1.5, seed=0)
    phases = [(36.0, 45.0), (1e-5, 1e-5)]
    t = time.time()
    r = g.homogenize(g.IsotropicMedium(lab, phases), tol=1e-9, form="sym6", maxit=200000)
    out = dict(image="synth.two_phase(16, 0.2, 1.5, seed=0)", phases=phases, tol=1e-9, form="sym6",
               C=r.C.tolist(), C_sym=r.C_sym.tolist(), iters=r.iters, seconds=time.time() - t)
    json.dump(out, open(os.path.join(HERE, "paper_pores_16.json"), "w"), indent=1)


def _study_run(np_):
    g.set_workers(1)
    n, p = np_
    lab = synth.four_phase(48, sigma=2.0, seed=21)
    t = time.time()
    h = hier.hierarchical(lab, synth.FOUR_PHASE["phases"], n, p, tol=1e-9, form="sym6")
    K_am, G_am = hier.arithmetic_mean_moduli(h.C_sub)
    print("study n", n, "pad", p, time.time() - t, flush=True)
    return dict(n=n, pad=p, C=h.C.tolist(), K_am=float(K_am), G_am=float(G_am), seconds=time.time() - t)


def study_48(jobs=1):
    """The error study of Sec. 5 in miniature: a 48^3 four-phase image (sigma
    2, seed 21), its plain stiffness, and the two-level scheme for subimage
    sizes 8, 12, 16 with 0 and 2 voxels of padding, with the arithmetic mean
    of the subimage moduli; CG to 1e-9."""
    lab = synth.four_phase(48, sigma=2.0, seed=21)
    t = time.time()
    ref = g.homogenize(g.IsotropicMedium(lab, synth.FOUR_PHASE["phases"]), tol=1e-9, form="sym6")
    runs = _pool_map(_study_run, [(n, p) for p in (0, 2) for n in (8, 12, 16)], jobs)
    out = dict(image="synth.four_phase(48, sigma=2.0, seed=21)", tol=1e-9, form="sym6", C_ref=ref.C_sym.tolist(),
               ref_seconds=time.time() - t, runs=runs)
    json.dump(out, open(os.path.join(HERE, "study_48.json"), "w"), indent=1)


if __name__ == "__main__":
    fn = {"four_phase_256": four_phase_256, "hier_512_items": hier_512_items,
          "uneven_2048_items": uneven_2048_items, "paper_pores_16": paper_pores_16,
          "study_48": study_48}[sys.argv[1]]
    if len(sys.argv) > 2:
        fn(jobs=int(sys.argv[2]))
    else:
        fn()
