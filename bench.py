"""Benchmark: voxel-iterations per second of the FFT elasticity solve.

Workload (one step): effective stiffness of one 256^3 four-phase rock-like
image (quartz/feldspar/clay/pore, fractions 0.55/0.15/0.10/0.20, smoothing
sigma 2 voxels, seed 1) under the six unit macroscopic strains, FP32 fields
and FFTs with FP64 reductions, CG to a relative residual of 1e-6.  Labels
are resident in device memory before the timed region.

voxel-iters = sum over the six loads of (voxels x CG iterations).

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (algorithmic bytes per launch / mean launch time from HIP events on
the library stream) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KCLS = ("zinv", "yinv", "x", "yfwd", "zfwd")


def algorithmic_bytes(nx, ny, nz, cbytes=8):
    """Bytes each pass class must move per system-iteration: the CG vectors as 3-vectors, the
    6-component spectrum in FP32 complex (cbytes per value), labels once per voxel."""
    nf = (nx // 2 + 1) * ny * nz  # half-spectrum frequencies
    V = nx * ny * nz
    return {
        "zinv": nf * cbytes * (3 + 3 + 3 + 6),   # read r, p; write p, spectrum
        "yinv": nf * cbytes * 12,                # read + write 6 components
        "x": nf * cbytes * 12 + V,               # read + write 6 components, labels
        "yfwd": nf * cbytes * 12,
        "zfwd": nf * cbytes * (6 + 3 + 3),       # read spectrum, r; write r
    }


SOLVER_SOURCES = ("fft.hpp", "hh_internal.hpp", "kernels.hpp", "solver_kernels.hpp", "solver_common.hip",
                  "sizes_f32_*.hip", "sizes_f64_*.hip")


def kernel_source_hash():
    """Short hash of the solver kernels' sources; profile-derived figures are
    used only while it matches the hash recorded with them."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = set()
    for pat in SOLVER_SOURCES:
        files.update(glob.glob(os.path.join(ROOT, "paper_2208_02320_amd", "csrc", pat)))
    for f in sorted(files):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel, n, plan):
    """HBM bytes per dispatch of a pass class from the committed counter
    profile (FETCH_SIZE/WRITE_SIZE scaled by the copy-kernel calibration),
    or None if the profile is missing, for another size, for another tile
    plan than the timed one, or stale."""
    path = os.path.join(ROOT, "profiles", "solver_passes_256cube_counters.md")
    if n != 256 or not os.path.exists(path):
        return None
    sha, val, prof_plan = None, None, None
    for line in open(path):
        w = line.split()
        if len(w) == 2 and w[0] == "source_sha256_16":
            sha = w[1]
        if len(w) == 4 and w[0] == "tile_plan":
            prof_plan = [int(x) for x in w[1:]]
        if len(w) == 3 and w[0] == "traffic_bytes_per_dispatch" and w[1] == kernel:
            val = float(w[2])
    return val if sha == kernel_source_hash() and prof_plan == list(plan) else None


def _mandel_rel_error(C, Cref):
    """||C - Cref||_F / ||Cref||_F with shear rows and columns times sqrt 2."""
    s = np.array([1.0, 1.0, 1.0, 2.0 ** 0.5, 2.0 ** 0.5, 2.0 ** 0.5])
    M = np.outer(s, s)
    Cref = np.asarray(Cref)
    return float(np.linalg.norm((np.asarray(C) - Cref) * M) / np.linalg.norm(Cref * M))


def _stored_oracle(name):
    """FP64 oracle results stored under tests/golden by a script that runs only
    the oracle and the seeded generator (tol 1e-9); None where absent."""
    path = os.path.join(ROOT, "tests", "golden", name)
    return json.load(open(path)) if os.path.exists(path) else None


def error_vs_stored_oracle(n, C):
    """Relative error of the timed result's stiffness against the stored FP64
    oracle result for the same seeded image.  None for sizes without one."""
    ref = _stored_oracle("four_phase_%d_seed1.json" % n)
    if ref is None:
        return None
    return {"rel_error": _mandel_rel_error(C, ref["C_sym"]), "bound": 1e-5,
            "oracle": "FP64 oracle at tol %g (%s)" % (ref["tol"], ref["image"])}


def sampled_error_vs_stored_oracle(name, C_of_item):
    """Largest relative error over the sampled items of a stored FP64 oracle
    result; C_of_item(index) gives the GPU stiffness of an item."""
    ref = _stored_oracle(name)
    if ref is None:
        return None
    errs = [_mandel_rel_error(C_of_item(it["index"]), it["C_sym"]) for it in ref["items"]]
    return {"max_rel_error": max(errs), "items": len(errs), "bound": 1e-5,
            "oracle": "FP64 oracle at tol %g, %s" % (ref["tol"], name)}


def cpu_baseline(lab, phases, iters=2):
    """FP64 oracle on a bounded sample of the same workload, in the form the GPU
    solves (symmetric projection, CG): load 1 of the same image, its right-hand
    side and the first ``iters`` CG iterations, once with one FFT thread and
    once with all host threads.  voxel-iters/s counts the CG iterations."""
    from oracle import galerkin as g
    med = g.IsotropicMedium(lab, phases)
    V = float(lab.size)
    allw = g.workers()
    runs = {}
    for w in (1, allw):
        g.set_workers(w)
        t = time.perf_counter()
        _, info = g.solve_load(med, g.unit_strain(0), tol=1e-6, maxit=iters, form="sym6")
        dt = time.perf_counter() - t
        runs[w] = (V * info.iters / dt, dt, info.iters)
    g.set_workers(allw)
    return {"value": runs[allw][0], "unit": "voxel-iters/s", "cores": allw, "kind": "oracle",
            "value_1_core": runs[1][0],
            "sample": "FP64 oracle (symmetric projection, CG, scipy.fft), load 1 of the same %s image: right-hand "
                      "side and the first %d CG iterations, %.1f s with %d FFT threads and %.1f s with 1; the "
                      "time includes the right-hand side" % ("x".join(map(str, lab.shape)), runs[allw][2],
                                                            runs[allw][1], allw, runs[1][1])}


def bench_hier(args):
    """Two-level scheme on a 512^3 four-phase image (seed 2): 512 subimages of
    64^3 with 8 voxels of padding (80^3 boxes) batched in one group, then the
    8^3 anisotropic intermediate image; Richardson over n = 32, 64, 128."""
    import torch
    from paper_2208_02320_amd import hh, synth
    N = args.hier_size
    lab = synth.four_phase(N, sigma=2.0, seed=2)
    phases = synth.FOUR_PHASE["phases"]
    dev = torch.from_numpy(lab).to("cuda:0")
    ctx = hh.Context(0)
    out = {}
    ns = [int(x) for x in args.hier_ns.split(",")]
    for n in ns:
        ctx.hierarchical(dev, phases, n, 8, tol=1e-6)  # warm-up (workspace, code objects)
        torch.cuda.synchronize()
        t = time.perf_counter()
        C, Cs, rep = ctx.hierarchical(dev, phases, n, 8, tol=1e-6)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        out[n] = dict(C=C, Cs=Cs, seconds=dt, items=rep["items"], voxel_iters=rep["voxel_iters"],
                      level2_iters=rep["iters"])
        print("bench: hier n=%d pad 8: %d subimages in %.3f s, %.3e voxel-iter/s" %
              (n, rep["items"], dt, rep["voxel_iters"] / dt), file=sys.stderr, flush=True)
    K = G = None
    if len(ns) >= 2:
        Cinf, slope = hh.richardson(ns, [out[n]["C"] for n in ns])
        K, G = hh.moduli(Cinf)
    three = None
    if not args.no_levels and 32 in out:
        # three levels: the intermediate image of n = 32 cut again into 2^3
        # blocks with 1 voxel of surround, then the last image
        t = time.perf_counter()
        C3, rep3 = ctx.hierarchical_levels(dev, phases, [(32, 8), (2, 1)], tol=1e-6)
        torch.cuda.synchronize()
        dt3 = time.perf_counter() - t
        K3, G3 = hh.moduli(C3)
        K2, G2 = hh.moduli(out[32]["C"])
        print("bench: three levels (32 pad 8, 2 pad 1): K %.4f G %.4f (two levels: K %.4f G %.4f) in %.3f s" %
              (K3, G3, K2, G2, dt3), file=sys.stderr, flush=True)
        three = {"levels": [[32, 8], [2, 1]], "K_G": [K3, G3], "seconds": dt3, "two_level_K_G": [K2, G2]}
    rates = {n: box_pass_rates(ctx, dev, phases, n, 8) for n in ns}
    for n in ns:
        print("bench: hier n=%d pass rates with every launch full (TB/s): %s" %
              (n, ", ".join("%s %.2f" % kv for kv in rates[n]["TBps"].items())), file=sys.stderr, flush=True)
    r = out[64] if 64 in out else out[ns[0]]
    line = {
        "metric": "subimages/s of the batched FFT solve in the two-level scheme",
        "value": r["items"] / r["seconds"], "unit": "subimages/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "hierarchical %d^3 four-phase, n = %d, pad 8 (%d^3 boxes), 6 loads, tol 1e-6"
                               % (N, 64 if 64 in out else ns[0], (64 if 64 in out else ns[0]) + 16)},
        "voxel_iters_per_s": r["voxel_iters"] / r["seconds"], "seconds": r["seconds"],
        "per_n": {n: {"subimages": out[n]["items"], "seconds": round(out[n]["seconds"], 4),
                      "subimages_per_s": round(out[n]["items"] / out[n]["seconds"], 2),
                      "voxel_iters_per_s": out[n]["voxel_iters"] / out[n]["seconds"],
                      "K_G": hh.moduli(out[n]["C"])} for n in ns},
        "richardson": {"K_inf": K, "G_inf": G},
        "pass_rates": rates,
        "error_vs_oracle": (sampled_error_vs_stored_oracle("four_phase_512_n64_p8_items.json",
                                                           lambda i: _full36(out[64]["Cs"][i]))
                            if N == 512 and 64 in out else None),
        "three_levels": three,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


PASS_BYTES = {"zinv": 120, "yinv": 96, "x": 96, "yfwd": 96, "zfwd": 96}  # per frequency and system-iteration


def box_pass_rates(ctx, img, phases, n, pad, iters=10):
    """HBM rate of each pass on the padded boxes of the two-level scheme with
    every launch full: the first boxes of the image (about 72 M voxels), their
    core as the averaging region, a tolerance out of reach and a fixed number
    of iterations, the second of two calls (the first tunes).  Algorithmic
    bytes of the system-iterations run over the summed launch times of each
    pass class (HIP events on the library's stream)."""
    b = n + 2 * pad
    pack = ctx.gather_subimages(img, n, pad)
    cnt = min(pack.shape[0], max(1, int(72e6 // b ** 3)))
    pack = pack[:cnt].contiguous().reshape(-1)
    core = [(pad, pad, pad, pad + n, pad + n, pad + n)] * cnt
    for _ in range(2):
        _, _, _, it, rep = ctx.homogenize_batch([(b, b, b)] * cnt, [phases] * cnt, regions=core, labels_pack=pack,
                                                tol=1e-14, profile=1, max_iter=iters, check=False)
    nf = b * b * (b // 2 + 1)
    sys_iters = float(np.sum(it))
    tb = {}
    for k, B in PASS_BYTES.items():
        byt = sys_iters * (nf * B + (b ** 3 if k == "x" else 0))
        tb[k] = round(byt / (rep["kernel_ms"][k] * 1e-3) / 1e12, 3)
    return {"boxes": cnt, "box": b, "system_iterations": sys_iters, "TBps": tb}


def _full36(c21):
    C = np.zeros((6, 6))
    k = 0
    for i in range(6):
        for j in range(i, 6):
            C[i, j] = C[j, i] = c21[k]
            k += 1
    return C


def bench_study(args):
    """The error study of Sec. 5 on a synthetic stand-in: a 300^3 four-phase
    image with a correlation length near the paper's rocks (smoothing sigma 8,
    seed 5), homogenized directly (the reference) and by the two-level scheme
    for subimage sizes 50, 60, 75, 100 with 0, 5 and 10 voxels of padding per
    side (with --study-size 1024: 64, 128, 256 and 0, 8, 16 voxels, boxes of
    compiled lengths only); the arithmetic mean of the subimage stiffnesses beside each, and the
    n^-1 extrapolation per padding.  Only sizes with at least three subimages
    per axis: with two, the intermediate image has only the mean and Nyquist
    frequencies, and its solve returns the arithmetic mean."""
    import torch
    from paper_2208_02320_amd import hh, synth
    N, sigma, seed = args.study_size, 8.0, 5
    if args.study_phases == "four":
        phases = synth.FOUR_PHASE["phases"]
        lab = synth.four_phase_device(N, sigma=sigma, seed=seed)
    else:  # two phases at porosity 0.15 (Table 1 spans 3.45 to 22.2 %)
        phases = synth.PAPER_TWO_PHASE if args.study_phases == "paper" else synth.APPENDIX_B_TWO_PHASE
        lab = synth.rocklike_device(N, [0.85, 0.15], sigma=sigma, seed=seed, low_to_high=[1, 0])
    torch.cuda.synchronize()
    ctx = hh.Context(0)
    t0 = time.perf_counter()
    ref = ctx.homogenize(lab, phases, tol=1e-6)
    t_ref = time.perf_counter() - t0
    Kr, Gr = hh.moduli(ref.C)
    print("bench: study %d^3 reference K %.4f G %.4f in %.2f s (iters %s)" % (N, Kr, Gr, t_ref, ref.report["iters"]),
          file=sys.stderr, flush=True)
    # subimage sizes and paddings: the 300^3 stand-in uses sizes near the paper's
    # (3 to 6 per axis); a power-of-two image (1024^3, whose plain solve is the
    # paper's brute-force scale) uses 64, 128, 256 with 0, 8, 16 voxels
    if N % 256 == 0:
        cand, pads = (64, 128, 256), (0, 8, 16)
    elif N % 300 == 0:
        cand, pads = (50, 60, 75, 100), (0, 5, 10)
    else:
        cand, pads = (16, 24, 32, 48, 64), (0, 4, 8)
    ns = [n for n in cand if N % n == 0 and N // n >= 3]
    runs = {}
    for pad in pads:
        for n in ns:
            if not hh.size_supported(n + 2 * pad, 0):
                continue  # box length without compiled passes
            t = time.perf_counter()
            C, Cs, rep = ctx.hierarchical(lab, phases, n, pad, tol=1e-6, check=False)
            dt = time.perf_counter() - t
            K, G = hh.moduli(C)
            Ka, Ga = hh.mean_moduli(Cs)
            if rep["status"] != 0:
                print("bench: study n=%d pad %d: status %d (level-2 iterations %s)" % (n, pad, rep["status"],
                                                                                    rep["iters"]),
                      file=sys.stderr, flush=True)
            if rep["retried"]:
                print("bench: study n=%d pad %d: %d subimages solved again with FP64 fields" % (n, pad, rep["retried"]),
                      file=sys.stderr, flush=True)
            runs[(n, pad)] = dict(C=C, K=K, G=G, K_am=Ka, G_am=Ga, seconds=dt, retried=rep["retried"],
                                  status=rep["status"])
            print("bench: study n=%d pad %d: K %.4f (%+.3f %%) G %.4f (%+.3f %%); mean of subimages K %+.3f %% "
                  "G %+.3f %%; %.2f s" % (n, pad, K, 100 * (K / Kr - 1), G, 100 * (G / Gr - 1),
                                         100 * (Ka / Kr - 1), 100 * (Ga / Gr - 1), dt), file=sys.stderr, flush=True)
    fits = {}
    for pad in pads:
        nsp = [n for n in ns if (n, pad) in runs]
        if len(nsp) < 2:
            continue
        Cinf, _ = hh.richardson(nsp, [runs[(n, pad)]["C"] for n in nsp])
        Ki, Gi = hh.moduli(Cinf)
        fits[pad] = {"n": nsp, "K_inf": Ki, "G_inf": Gi, "K_err_pct": 100 * (Ki / Kr - 1),
                     "G_err_pct": 100 * (Gi / Gr - 1)}
    total = time.perf_counter() - t0
    line = {
        "metric": "seconds for the two-level error study (reference solve + %d hierarchies)" % len(runs),
        "value": total, "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "error study, %d^3 %s (sigma %g, seed %d), n in %s, pad %s, tol 1e-6"
                               % (N, {"four": "four-phase", "paper": "two-phase, the paper's moduli",
                                      "appendixB": "two-phase, Appendix B moduli"}[args.study_phases],
                                  sigma, seed, ns, "/".join(str(p) for p in pads)), "phases": phases},
        "reference": {"K": Kr, "G": Gr, "seconds": t_ref, "iters": ref.report["iters"]},
        "runs": [{"n": n, "pad": pad, "K_err_pct": 100 * (r["K"] / Kr - 1), "G_err_pct": 100 * (r["G"] / Gr - 1),
                  "K_mean_err_pct": 100 * (r["K_am"] / Kr - 1), "G_mean_err_pct": 100 * (r["G_am"] / Gr - 1),
                  "seconds": r["seconds"], "fp64_retries": r["retried"], "status": r["status"]}
                 for (n, pad), r in sorted(runs.items(), key=lambda kv: (kv[0][1], kv[0][0]))],
        "richardson": fits,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_timing(args):
    """Computation time against size (the timing discussion of Sec. 4 and its
    log-log figure): (a) the plain solve of one n^3 four-phase image (sigma 8,
    seed 5) for n from 64 to 1024, timed on a second call (the first tunes and
    captures graphs), with a power-law fit t ~ n^a over n >= 128, where the
    six systems fill the GPU (1024^3 runs its loads in two memory waves); (b) the two-level scheme on a 900^3 image of the
    same recipe, pad 0, for every subimage size dividing 900 with at least
    three subimages per axis (75 to 300, the paper's partition grid), total
    solve time against n with its fit.  One-time tuning and graph setup are
    reported apart and left out of the fitted times."""
    import numpy as np
    import torch
    from paper_2208_02320_amd import hh, synth
    phases = synth.FOUR_PHASE["phases"]
    sigma, seed = 8.0, 5
    ctx = hh.Context(0)
    single = []
    for n in (64, 96, 128, 160, 192, 256, 320, 512, 1024):
        lab = synth.four_phase_device(n, sigma=sigma, seed=seed)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()  # the generator's temporaries
        first = ctx.homogenize(lab, phases, tol=1e-6).report
        t = time.perf_counter()
        rep = ctx.homogenize(lab, phases, tol=1e-6).report
        dt = time.perf_counter() - t
        single.append({"n": n, "seconds": dt, "device_seconds": rep["seconds"], "iters": rep["iters"],
                       "voxel_iters_per_s": rep["voxel_iters"] / dt, "setup_ms_first_call": first["setup_ms"]})
        print("bench: timing single n=%d: %.3f s, iters %s, %.3g voxel-iter/s" %
              (n, dt, rep["iters"], rep["voxel_iters"] / dt), file=sys.stderr, flush=True)
        del lab
    big = [r for r in single if r["n"] >= 128]
    a_single = float(np.polyfit(np.log([r["n"] for r in big]), np.log([r["seconds"] for r in big]), 1)[0])
    N = args.timing_size
    ctx.release_workspace()
    lab = synth.four_phase_device(N, sigma=sigma, seed=seed)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    hier = []
    for n in [n for n in range(75, N // 3 + 1) if N % n == 0]:
        t = time.perf_counter()
        C, _, rep = ctx.hierarchical(lab, phases, n, 0, tol=1e-6)
        dt = time.perf_counter() - t
        solve = dt - rep["setup_ms"] * 1e-3
        K, G = hh.moduli(C)
        hier.append({"n": n, "seconds": dt, "setup_ms": rep["setup_ms"], "solve_seconds": solve,
                     "subimages": (N // n) ** 3, "voxel_iters_per_s": rep["voxel_iters"] / solve, "K": K, "G": G})
        print("bench: timing hierarchy N=%d n=%d: %.2f s (setup %.0f ms), %.3g voxel-iter/s, K %.4f G %.4f" %
              (N, n, dt, rep["setup_ms"], rep["voxel_iters"] / solve, K, G), file=sys.stderr, flush=True)
    a_hier = float(np.polyfit(np.log([r["n"] for r in hier]), np.log([r["solve_seconds"] for r in hier]), 1)[0])
    # the plain solve of the same N^3 image, the reference of the scheme's error
    plain = None
    if hh.size_supported(N, 0):
        ctx.release_workspace()
        t = time.perf_counter()
        rp = ctx.homogenize(lab, phases, tol=1e-6)
        dtp = time.perf_counter() - t
        Kp, Gp = hh.moduli(rp.C)
        plain = {"seconds": dtp, "K": Kp, "G": Gp, "iters": rp.report["iters"]}
        for r in hier:
            r["K_err_pct"] = 100 * (r["K"] / Kp - 1)
            r["G_err_pct"] = 100 * (r["G"] / Gp - 1)
        print("bench: timing plain %d^3: %.2f s, K %.4f G %.4f" % (N, dtp, Kp, Gp), file=sys.stderr, flush=True)
    # M(n) = M_inf + c / n over the partition grid (Sec. 5 fit)
    A = np.stack([np.ones(len(hier)), 1.0 / np.array([r["n"] for r in hier], float)], axis=1)
    fit = {}
    for m in ("K", "G"):
        y = np.array([r[m] for r in hier])
        coef = np.linalg.lstsq(A, y, rcond=None)[0]
        fit[m] = {"M_inf": float(coef[0]), "c": float(coef[1]), "max_residual": float(np.abs(A @ coef - y).max())}
    line = {
        "metric": "time exponent of the plain solve (t ~ n^a, n = 128..1024)", "value": a_single, "unit": "exponent",
        "n_gpus": 1, "higher_is_better": False, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "timing: four-phase images (sigma %g, seed %d), tol 1e-6; plain solves n = 64..1024, "
                               "two-level scheme on %d^3, pad 0" % (sigma, seed, N)},
        "single": single, "hierarchy": hier, "hierarchy_time_exponent": a_hier, "hierarchy_n_inverse_fit": fit,
        "plain_reference": plain,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_contrast(args):
    """Iterations and accuracy against phase contrast (Sec. 2 gives pores of
    1e-5 GPa, chosen there for stability): a 64^3 two-phase quartz / pore
    image (porosity 0.2, sigma 2, seed 0), pore moduli from the benchmark
    2.25 / 1 GPa down to the paper's 1e-5 GPa; FP32 and FP64 fields at tol
    1e-6 against FP64 at tol 1e-9."""
    from paper_2208_02320_amd import hh, synth
    lab = synth.two_phase(64, 0.2, 2.0, 0)
    ctx = hh.Context(0)
    rows = []
    for Kp, Gp in ((2.25, 1.0), (0.1, 0.05), (1e-2, 5e-3), (1e-3, 5e-4), (1e-5, 1e-5)):
        ph = [synth.QUARTZ, (Kp, Gp)]
        row = {"pore_K": Kp, "pore_G": Gp, "contrast": max(synth.QUARTZ) / min(Kp, Gp)}
        ref = ctx.homogenize(lab, ph, tol=1e-9, precision=1, max_iter=50000, stall_limit=2000, check=False)
        row["fp64_tight"] = {"iters": max(ref.report["iters"]), "status": ref.report["status"],
                             "K_G": hh.moduli(ref.C)}
        for name, prec in (("fp32", 0), ("fp64", 1)):
            t = time.perf_counter()
            r = ctx.homogenize(lab, ph, tol=1e-6, precision=prec, max_iter=50000, stall_limit=2000, check=False)
            dt = time.perf_counter() - t
            err = float(np.linalg.norm(_mandel(r.C) - _mandel(ref.C)) / np.linalg.norm(_mandel(ref.C)))
            row[name] = {"iters": max(r.report["iters"]), "status": r.report["status"], "seconds": dt,
                         "rel_err_vs_tight": err}
        print("bench: contrast %.1e: fp32 %d it (status %d) err %.1e; fp64 %d it err %.1e; tight %d it" % (
            row["contrast"], row["fp32"]["iters"], row["fp32"]["status"], row["fp32"]["rel_err_vs_tight"],
            row["fp64"]["iters"], row["fp64"]["rel_err_vs_tight"], row["fp64_tight"]["iters"]),
            file=sys.stderr, flush=True)
        rows.append(row)
    line = {"metric": "CG iterations to tol 1e-6 at the paper's pore contrast (FP64 fields)",
            "value": rows[-1]["fp64"]["iters"], "unit": "iterations", "n_gpus": 1, "higher_is_better": False,
            "dtype": "f32/f64", "data": "synthetic",
            "config": {"workload": "64^3 two-phase quartz/pore (porosity 0.2, sigma 2, seed 0), pore moduli "
                                   "2.25 GPa down to 1e-5 GPa, 6 loads"},
            "rows": rows}
    print(json.dumps(line), flush=True)
    ctx.close()


def _mandel(C):
    d = np.array([1.0, 1.0, 1.0, np.sqrt(2.0), np.sqrt(2.0), np.sqrt(2.0)])
    return np.asarray(C).reshape(6, 6) * d[:, None] * d[None, :]


def bench_uneven(args):
    """2048 independent subimages of sizes 32/48/64/96 (seed 1234), 2-4 phases,
    contrast <= 50, six loads each, FP32, tol 1e-6, in one batched call."""
    import torch
    from paper_2208_02320_amd import hh, synth
    recipe = synth.uneven_batch(args.uneven_count, seed=1234)
    t = time.perf_counter()
    imgs = [synth.item_image(it) for it in recipe]
    print("bench: generated %d images in %.1f s" % (len(imgs), time.perf_counter() - t),
          file=sys.stderr, flush=True)
    pack = torch.from_numpy(np.concatenate([im.ravel() for im in imgs])).to("cuda:0")
    shapes = [im.shape for im in imgs]
    phs = [it["phases"] for it in recipe]
    ctx = hh.Context(0)
    ctx.homogenize_batch(shapes, phs, labels_pack=pack, tol=1e-6)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    C, Craw, st, iters, rep = ctx.homogenize_batch(shapes, phs, labels_pack=pack, tol=1e-6)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    # the same batch with its four shape groups solved concurrently (four lanes)
    ctx.homogenize_batch(shapes, phs, labels_pack=pack, tol=1e-6, lanes=4)  # warm-up of the lanes
    torch.cuda.synchronize()
    t = time.perf_counter()
    C4 = ctx.homogenize_batch(shapes, phs, labels_pack=pack, tol=1e-6, lanes=4)[0]
    torch.cuda.synchronize()
    dt_conc = time.perf_counter() - t
    print("bench: uneven %d items: %.3f s one group at a time, %.3f s with the groups on four lanes; identical: %s" %
          (len(imgs), dt, dt_conc, bool(np.array_equal(C, C4))), file=sys.stderr, flush=True)
    sizes = {}
    for im in imgs:
        sizes[im.shape[0]] = sizes.get(im.shape[0], 0) + 1
    line = {
        "metric": "voxel-iters/s of the batched uneven FFT solve",
        "value": rep["voxel_iters"] / dt, "unit": "voxel-iters/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%d subimages, sizes %s, 2-4 phases, 6 loads, tol 1e-6"
                               % (len(imgs), sizes)},
        "subimages_per_s": len(imgs) / dt, "seconds": dt, "status_ok": int((st == 0).sum()),
        "seconds_groups_on_four_lanes": dt_conc, "four_lanes_identical": bool(np.array_equal(C, C4)),
        "mean_iters": float(iters.mean()),
        "error_vs_oracle": (sampled_error_vs_stored_oracle("uneven_2048_items.json", lambda i: C[i])
                            if len(imgs) == 2048 else None),
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def conv_flops_per_item(n, nphase):
    """Multiply-adds x 2 of the four convolutions on one n^3 input (real
    input channels for the one-hot layer)."""
    cin, cout = (nphase, 32, 32, 64), (32, 32, 64, 64)
    f, d = 0, n
    for l in range(4):
        d //= 2
        f += 2 * d ** 3 * cout[l] * 27 * cin[l]
    return f


def bench_surrogate(args):
    """Two-level scheme with the CNN surrogate: 1024^3 four-phase image (device
    generator, seed 3) cut into 4096 subimages of 64^3 with 8 voxels of
    padding; two shipped networks predict every subimage stiffness, the gate
    sends doubtful ones to the FFT solver, then the 16^3 level-2 solve.  One
    step is the whole pipeline; the plain FFT hierarchy on the same image is
    timed once for the speed-up and is the reference of the C* error."""
    import torch
    from paper_2208_02320_amd import hh, surrogate, synth
    N, n, pad = args.sur_size, 64, 8
    phases = synth.FOUR_PHASE["phases"]
    ctx = hh.Context(0)
    paths = surrogate.default_weights(n, pad, args.weights_dir)
    for pth in paths:
        if not os.path.exists(pth):
            raise SystemExit("surrogate weights %s missing: train them with "
                             "python -m paper_2208_02320_amd.surrogate" % pth)
    na, nb = (surrogate.load(ctx, pth) for pth in paths)
    img = synth.four_phase_device(N, sigma=2.0, seed=3, device="cuda:0")
    torch.cuda.synchronize()
    kw = dict(spread_tol=args.spread_tol, bound_tol=args.bound_tol, tol=1e-6)
    print("bench: surrogate %d^3, warmup %d" % (N, args.warmup), file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        ctx.hierarchical_surrogate(img, phases, n, pad, na, nb, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        C, Cs, fb, rep = ctx.hierarchical_surrogate(img, phases, n, pad, na, nb, profile=1, **kw)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    items = rep["items"]
    print("bench: surrogate step %.3f s, fallback %d of %d" % (dt, int(fb.sum()), items), file=sys.stderr,
          flush=True)
    # network inference alone, for the MFMA roofline of the convolutions
    pack = ctx.gather_subimages(img, n, pad)
    na.predict(pack[:64], offset=pad)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    na.predict(pack, offset=pad)
    ev1.record()
    torch.cuda.synchronize()
    cnn_s = ev0.elapsed_time(ev1) * 1e-3
    flops = conv_flops_per_item(n, len(phases)) * items
    tflops = flops / cnn_s / 1e12
    del pack
    # the plain FFT hierarchy on the same image: speed and reference C*
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Cp, Csp, repp = ctx.hierarchical(img, phases, n, pad, tol=1e-6)
    torch.cuda.synchronize()
    dtp = time.perf_counter() - t1
    err = float(surrogate.rel_error21(hh.upper21(C), hh.upper21(Cp))[0])
    sub_err = surrogate.rel_error21(Cs, Csp)
    # the plain solve of the whole image (the paper's brute-force reference),
    # where the axis length is compiled; its loads run a few at a time at 1024^3
    brute = None
    if hh.size_supported(N, 0):
        torch.cuda.empty_cache()
        ctx.release_workspace()
        t2 = time.perf_counter()
        rb = ctx.homogenize(img, phases, tol=1e-6)
        torch.cuda.synchronize()
        Kb, Gb = hh.moduli(rb.C)
        Kh, Gh = hh.moduli(Cp)
        Ks, Gs = hh.moduli(C)
        brute = {"seconds": time.perf_counter() - t2, "K": Kb, "G": Gb,
                 "plain_hierarchy_rel_error": float(surrogate.rel_error21(hh.upper21(Cp), hh.upper21(rb.C))[0]),
                 "surrogate_rel_error": float(surrogate.rel_error21(hh.upper21(C), hh.upper21(rb.C))[0]),
                 "K_G_err_pct": {"plain_hierarchy": [100 * (Kh / Kb - 1), 100 * (Gh / Gb - 1)],
                                 "surrogate": [100 * (Ks / Kb - 1), 100 * (Gs / Gb - 1)]}}
        print("bench: brute-force %d^3 in %.1f s: K %.4f G %.4f; hierarchy error %.2e, surrogate error %.2e" %
              (N, brute["seconds"], Kb, Gb, brute["plain_hierarchy_rel_error"], brute["surrogate_rel_error"]),
              file=sys.stderr, flush=True)
    line = {
        "metric": "subimages/s of the two-level scheme with surrogate and FFT fallback",
        "value": items / dt, "unit": "subimages/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 network / f32 solver", "data": "synthetic",
        "config": {"workload": "hierarchical %d^3 four-phase (seed 3), n = 64, pad 8, CNN surrogate pair, "
                               "spread_tol %g, bound_tol %g, FFT fallback tol 1e-6" % (N, args.spread_tol,
                                                                                      args.bound_tol)},
        "fallback_fraction": float(fb.mean()),
        "rel_error_vs_plain": err,
        "subimage_rel_error": {"mean": float(sub_err.mean()), "p95": float(np.quantile(sub_err, 0.95)),
                               "max": float(sub_err.max())},
        "plain_subimages_per_s": items / dtp, "speedup_vs_plain": dtp / dt,
        "brute_force": brute,
        "roofline": {"bound": "mfma", "kernel": "network forward (4 BF16 convolutions + head)",
                     "achieved": round(tflops, 2), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(tflops / 2500.0, 5), "traffic": None,
                     "algorithmic_flops_per_item": conv_flops_per_item(n, len(phases)),
                     "seconds_for_%d_items" % items: cnn_s},
        "kernel_ms": rep["kernel_ms"],
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def surrogate_leg(ctx, img, phases, nets, steps=3, warmup=1, spread_tol=0.02, bound_tol=0.0, n=64, pad=8,
                  keep_plain=False):
    """The two-level scheme with the network pair, gate and FFT fallback on one
    device image, timed over ``steps`` calls after ``warmup``; the plain FFT
    hierarchy of the same image, timed once, is the reference of its C* error
    and of the speed-up (its C* under "_C_plain" with ``keep_plain``)."""
    import torch
    from paper_2208_02320_amd import hh, surrogate
    na, nb = nets
    kw = dict(spread_tol=spread_tol, bound_tol=bound_tol, tol=1e-6)
    for _ in range(warmup):
        ctx.hierarchical_surrogate(img, phases, n, pad, na, nb, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        C, Cs, fb, rep = ctx.hierarchical_surrogate(img, phases, n, pad, na, nb, **kw)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    t1 = time.perf_counter()
    Cp, Csp, repp = ctx.hierarchical(img, phases, n, pad, tol=1e-6)
    torch.cuda.synchronize()
    dtp = time.perf_counter() - t1
    sub = surrogate.rel_error21(Cs, Csp)
    acc = ~fb
    return {"subimages": int(rep["items"]), "subimages_per_s": rep["items"] / dt, "ms_per_step": dt * 1e3,
            "fallback_fraction": float(fb.mean()),
            "rel_error_vs_plain": float(surrogate.rel_error21(hh.upper21(C), hh.upper21(Cp))[0]),
            "subimage_rel_error_accepted": {"mean": float(sub[acc].mean()) if acc.any() else None,
                                            "max": float(sub[acc].max()) if acc.any() else None},
            "plain_subimages_per_s": rep["items"] / dtp, "plain_seconds": dtp, "speedup_vs_plain": dtp / dt,
            "K_G": hh.moduli(C), "plain_K_G": hh.moduli(Cp), **({"_C_plain": Cp} if keep_plain else {})}


def bench_surrogate_ood(args):
    """The shipped network pair (trained on sigma 2, fractions 0.55/0.15/0.10/
    0.20) on images it has not seen: a coarser texture (sigma 8), a different
    fraction mix (porosity 0.30) and a finer one (sigma 1.2).  Each line gives
    the gate's fallback fraction and the final C* error against the plain FFT
    hierarchy of the same image."""
    import torch
    from paper_2208_02320_amd import hh, surrogate, synth
    N = args.sur_size
    phases = synth.FOUR_PHASE["phases"]
    ctx = hh.Context(0)
    nets = [surrogate.load(ctx, pth) for pth in surrogate.default_weights(64, 8, args.weights_dir)]
    low = synth.FOUR_PHASE["low_to_high"]
    cases = [("training recipe (sigma 2, seed 3)", dict(fracs=synth.FOUR_PHASE["fracs"], sigma=2.0, seed=3)),
             ("sigma 8 (seed 5)", dict(fracs=synth.FOUR_PHASE["fracs"], sigma=8.0, seed=5)),
             ("porosity 0.30 (fractions 0.45/0.15/0.10/0.30, seed 6)", dict(fracs=[0.45, 0.15, 0.10, 0.30],
                                                                             sigma=2.0, seed=6)),
             ("sigma 1.2 (seed 7)", dict(fracs=synth.FOUR_PHASE["fracs"], sigma=1.2, seed=7))]
    rows = []
    for name, c in cases:
        img = synth.rocklike_device(N, c["fracs"], sigma=c["sigma"], seed=c["seed"], low_to_high=low)
        torch.cuda.synchronize()
        for net in nets:
            net.set_fraction_gate(args.frac_z)
        leg = surrogate_leg(ctx, img, phases, nets, steps=1, warmup=1, spread_tol=args.spread_tol,
                            bound_tol=args.bound_tol, keep_plain=True)
        Cp = leg.pop("_C_plain")
        leg["image"] = name
        # the same gate without its input-space tests (phase fractions, interface density)
        for net in nets:
            net.set_fraction_gate(0.0)
        C0, _, fb0, _ = ctx.hierarchical_surrogate(img, phases, 64, 8, nets[0], nets[1], spread_tol=args.spread_tol,
                                                   bound_tol=args.bound_tol, tol=1e-6)
        leg["without_input_tests"] = {
            "fallback_fraction": float(fb0.mean()),
            "rel_error_vs_plain": float(surrogate.rel_error21(hh.upper21(C0), hh.upper21(Cp))[0])}
        rows.append(leg)
        print("bench: surrogate on %s: fallback %.3f, C* error %.2e, %.0f subimages/s, %.0fx the plain hierarchy; "
              "without the input-space tests: fallback %.3f, C* error %.2e" %
              (name, leg["fallback_fraction"], leg["rel_error_vs_plain"], leg["subimages_per_s"],
               leg["speedup_vs_plain"], leg["without_input_tests"]["fallback_fraction"],
               leg["without_input_tests"]["rel_error_vs_plain"]), file=sys.stderr, flush=True)
        del img
        torch.cuda.empty_cache()
    line = {"metric": "C* error of the surrogate pipeline against the plain hierarchy, worst over the images",
            "value": max(r["rel_error_vs_plain"] for r in rows), "unit": "relative", "n_gpus": 1,
            "higher_is_better": False, "dtype": "bf16 network / f32 solver", "data": "synthetic",
            "config": {"workload": "surrogate pair on %d^3 four-phase images off its training recipe, n = 64, pad 8, "
                                   "spread_tol %g, bound_tol %g, input-test z_max %g" %
                                   (N, args.spread_tol, args.bound_tol, args.frac_z)},
            "images": rows}
    print(json.dumps(line), flush=True)
    for net in nets:
        net.close()
    ctx.close()


def bench_cnn(args):
    """Network kernels alone: inference over the 4096 padded 64^3 subimages of
    the 1024^3 surrogate workload, and Adam training steps at batch 32."""
    import torch
    from paper_2208_02320_amd import hh, surrogate, synth
    n, pad = 64, 8
    ctx = hh.Context(0)
    net = surrogate.load(ctx, surrogate.default_weights(n, pad, args.weights_dir)[0])
    img = synth.four_phase_device(args.sur_size, sigma=2.0, seed=3, device="cuda:0")
    pack = ctx.gather_subimages(img, n, pad)
    del img
    items = pack.shape[0]
    fl = conv_flops_per_item(n, 4)
    net.predict(pack[:64], offset=pad)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(args.steps):
        net.predict(pack, offset=pad)
    ev[1].record()
    torch.cuda.synchronize()
    inf_s = ev[0].elapsed_time(ev[1]) * 1e-3 / args.steps
    B = 32
    tgt = torch.zeros((B, 21), dtype=torch.float32, device="cuda:0")
    lab = pack[:B].contiguous()
    for _ in range(3):
        net.train_step(lab, tgt, 1e-6, offset=pad)
    nsteps = 20 * args.steps
    torch.cuda.synchronize()
    ev[2].record()
    for _ in range(nsteps):
        net.train_step(lab, tgt, 1e-6, offset=pad)
    ev[3].record()
    torch.cuda.synchronize()
    tr_s = ev[2].elapsed_time(ev[3]) * 1e-3 / nsteps
    inf_tf = fl * items / inf_s / 1e12
    line = {
        "metric": "subimages/s of network inference", "value": items / inf_s, "unit": "subimages/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": inf_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "CNN surrogate on %d padded 64^3 four-phase subimages (core input)" % items},
        "train_ms_per_step_batch32": tr_s * 1e3,
        "train_items_per_s": B / tr_s,
        "roofline": {"bound": "mfma", "kernel": "network forward (4 BF16 convolutions + head)",
                     "achieved": round(inf_tf, 2), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(inf_tf / 2500.0, 5), "traffic": None, "algorithmic_flops_per_item": fl},
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=("solve256", "hier", "uneven", "surrogate", "surrogate_ood", "cnn", "study",
                                               "contrast", "timing"),
                    default="solve256")
    ap.add_argument("--sur-size", type=int, default=1024)
    ap.add_argument("--weights-dir", default=None)
    ap.add_argument("--plan", default=None, help="fixed tile variants z,y,x of the default workload (else tuned)")
    ap.add_argument("--spread-tol", type=float, default=0.02)
    ap.add_argument("--bound-tol", type=float, default=0.0)
    ap.add_argument("--frac-z", type=float, default=5.0,
                    help="limit of the gate's input-space tests (phase fractions, interface density)")
    ap.add_argument("--hier-size", type=int, default=512)
    ap.add_argument("--hier-ns", default="32,64,128", help="subimage sizes of the hier workload")
    ap.add_argument("--no-levels", action="store_true", help="hier workload without the three-level run")
    ap.add_argument("--study-size", type=int, default=300)
    ap.add_argument("--study-phases", choices=("four", "paper", "appendixB"), default="four",
                    help="four-phase benchmark moduli, or two phases at porosity 0.15 with the paper's "
                         "moduli (Sec. 2) or Appendix B's")
    ap.add_argument("--timing-size", type=int, default=900)
    ap.add_argument("--uneven-count", type=int, default=2048)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="default workload without its surrogate leg")
    ap.add_argument("--cpu-iters", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload == "hier":
        return bench_hier(args)
    if args.workload == "uneven":
        return bench_uneven(args)
    if args.workload == "surrogate":
        return bench_surrogate(args)
    if args.workload == "cnn":
        return bench_cnn(args)
    if args.workload == "surrogate_ood":
        return bench_surrogate_ood(args)
    if args.workload == "study":
        return bench_study(args)
    if args.workload == "contrast":
        return bench_contrast(args)
    if args.workload == "timing":
        return bench_timing(args)

    import torch
    from paper_2208_02320_amd import hh, synth

    n = args.size
    phases = synth.FOUR_PHASE["phases"]
    if n <= 512:
        lab = synth.four_phase(n, sigma=2.0, seed=1)
        dev = torch.from_numpy(lab).to("cuda:0")
    else:  # the same recipe on the device (a host filter of 1024^3 voxels takes minutes)
        dev = synth.four_phase_device(n, sigma=2.0, seed=1)
        lab = None
        args.no_cpu = True
    ctx = hh.Context(0)
    opts = dict(tol=1e-6, precision=0)
    if args.plan:  # a fixed tile plan (profiling runs), else the tuned one
        opts["plan"] = [int(x) for x in args.plan.split(",")]
    print("bench: %d^3 four-phase, warmup %d" % (n, args.warmup), file=sys.stderr, flush=True)
    setup = []
    for _ in range(args.warmup):  # the first call autotunes and captures graphs (one-time)
        setup.append(ctx.homogenize(dev, phases, **opts).report["setup_ms"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timed = []
    last = None
    for _ in range(args.steps):
        last = ctx.homogenize(dev, phases, **opts)
        timed.append(last.report)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if not setup:  # no warm-up: the one-time setup fell inside the timed steps
        setup = [timed[0]["setup_ms"]]
    vi = sum(r["voxel_iters"] for r in timed)
    iters = timed[-1]["iters"]
    print("bench: %d steps %.3f s, iters %s, plan %s, one-time setup %s ms" %
          (args.steps, dt, iters, timed[-1]["plan"], [round(x, 1) for x in setup]), file=sys.stderr, flush=True)
    # per-class kernel times: the same solves again with HIP events around every launch
    # (plain launches instead of graph replays), outside the timed region
    reps = [ctx.homogenize(dev, phases, profile=1, **opts).report for _ in range(args.steps)]

    # roofline of the dominant kernel class
    ab = algorithmic_bytes(n, n, n)
    sys_iters = sum(sum(r["iters"]) for r in reps)
    ms = {k: sum(r["kernel_ms"][k] for r in reps) for k in KCLS}
    launches = {k: sum(r["kernel_launches"][k] for r in reps) for k in KCLS}
    dom = max(KCLS, key=lambda k: ms[k])
    bytes_dom = ab[dom] * sys_iters
    achieved = bytes_dom / (ms[dom] * 1e-3) / 1e9
    per_class = {k: {"ms": round(ms[k], 3), "launches": launches[k],
                     "GBs": round(ab[k] * sys_iters / max(ms[k] * 1e-3, 1e-12) / 1e9, 1)}
                 for k in KCLS}
    print("bench: per-class %s" % json.dumps(per_class), file=sys.stderr, flush=True)

    # the surrogate pipeline on the 1024^3 workload (shipped networks, gate, FFT
    # fallback, level 2) against the plain FFT hierarchy of the same image
    sur = None
    if not args.no_surrogate:
        from paper_2208_02320_amd import surrogate
        paths = surrogate.default_weights(64, 8, args.weights_dir)
        if all(os.path.exists(pth) for pth in paths):
            ctx.release_workspace()
            nets = [surrogate.load(ctx, pth) for pth in paths]
            img = synth.four_phase_device(args.sur_size, sigma=2.0, seed=3, device="cuda:0")
            torch.cuda.synchronize()
            sur = surrogate_leg(ctx, img, phases, nets, steps=args.steps, warmup=1, spread_tol=args.spread_tol,
                                bound_tol=args.bound_tol)
            sur["workload"] = ("hierarchical %d^3 four-phase (seed 3), n = 64, pad 8, shipped network pair, "
                               "spread_tol %g, FFT fallback tol 1e-6" % (args.sur_size, args.spread_tol))
            print("bench: surrogate %d^3: %.0f subimages/s, fallback %.3f, C* error %.2e, %.0fx the plain hierarchy" %
                  (args.sur_size, sur["subimages_per_s"], sur["fallback_fraction"], sur["rel_error_vs_plain"],
                   sur["speedup_vs_plain"]), file=sys.stderr, flush=True)
            del img
            for net in nets:
                net.close()
    cpu = None if args.no_cpu else cpu_baseline(lab, phases, args.cpu_iters)
    err = error_vs_stored_oracle(n, last.C) if last is not None else None
    out = {
        "metric": "voxel-iters/s of FFT elasticity solve",
        "value": vi / dt,
        "unit": "voxel-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain FFT solve, %d^3 four-phase rock-like image, 6 unit loads, "
                               "FP32 fields / FP64 reductions, tol 1e-6" % n,
                   "voxels": n ** 3, "iters_per_load": iters,
                   "voxel_iters_per_step": vi / args.steps, "tile_plan": timed[-1]["plan"],
                   "graph_replay": True, "one_time_setup_ms": round(setup[0], 2)},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": profiled_traffic(dom, n, timed[-1]["plan"]),
                     "algorithmic_bytes_per_launch": round(bytes_dom / max(launches[dom], 1)),
                     "algorithmic_bytes_per_system_iter": ab[dom],
                     "mean_launch_ms": round(ms[dom] / max(launches[dom], 1), 4)},
        "cpu_baseline": cpu,
        "error_vs_oracle": err,
        "surrogate": sur,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
