"""Seeded synthetic rock-like label images and workload recipes.

This module produces inputs only: it holds none of the homogenization
arithmetic, and both the CPU oracle (through the tests) and the GPU path
consume exactly the arrays it returns.

The paper's five segmented micro-CT sandstones (Sec. 2, Table 1) are not
available, so images stand in for them: periodic Gaussian-smoothed white
noise thresholded at quantiles, which gives an exponentially decaying
two-point correlation like the one fitted in Sec. 2 (Fig. 1b).

Label conventions: ``labels`` is a C-contiguous ``uint8`` array indexed
``[z][y][x]`` (x fastest).  ``fracs[i]`` is the volume fraction of label ``i``;
``low_to_high`` lists the labels in the order in which they take the lowest
to highest smoothed-noise values (pores lowest).
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

# Phase table (bulk K, shear G in GPa).  The two-phase quartz/pore set of the
# benchmarks uses the quartz row; the paper's own quartz (K 36, G 45) and
# pore (1e-5 GPa) values of Sec. 2 are listed for completeness.
QUARTZ = (37.0, 44.0)
FELDSPAR = (76.0, 26.0)
CLAY = (21.0, 7.0)
PORE = (2.25, 1.0)
PHASE_TABLE = (QUARTZ, FELDSPAR, CLAY, PORE)

FOUR_PHASE = dict(phases=[QUARTZ, FELDSPAR, CLAY, PORE],
                  fracs=[0.55, 0.15, 0.10, 0.20], low_to_high=[3, 2, 1, 0])
TWO_PHASE = dict(phases=[QUARTZ, PORE], fracs=[0.80, 0.20], low_to_high=[1, 0])
# The paper's own two-phase moduli: quartz K 36 / G 45 GPa and pores of 1e-5
# GPa (Sec. 2), and the second set of Appendix B, a phase ten times stiffer
# than the other (its soft bulk modulus is printed garbled; read as 9.80,
# a tenth of 98.04).
PAPER_TWO_PHASE = [(36.0, 45.0), (1e-5, 1e-5)]
APPENDIX_B_TWO_PHASE = [(98.04, 37.59), (9.80, 3.76)]


def smoothed_noise(shape, sigma, seed, dtype=np.float32):
    """Periodic Gaussian-smoothed standard-normal noise (wrap boundary)."""
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape, dtype=dtype)
    if sigma > 0:
        w = ndimage.gaussian_filter(w, sigma=sigma, mode="wrap", output=dtype)
    return w


def threshold(values, fracs, low_to_high):
    """Label voxels by quantile thresholds of ``values``."""
    fracs = np.asarray(fracs, dtype=np.float64)
    if np.any(fracs < 0) or abs(fracs.sum() - 1.0) > 1e-9:
        raise ValueError("fractions must be non-negative and sum to 1")
    order = list(low_to_high)
    if sorted(order) != list(range(len(fracs))):
        raise ValueError("low_to_high must be a permutation of the labels")
    cum = np.cumsum([fracs[l] for l in order])[:-1]
    flat = values.reshape(-1)
    cuts = np.quantile(flat, cum) if len(cum) else np.zeros(0)
    bins = np.searchsorted(cuts, flat, side="right")
    lut = np.asarray(order, dtype=np.uint8)
    return lut[bins].reshape(values.shape)


def rocklike(shape, fracs, sigma=2.0, seed=0, low_to_high=None):
    """Rock-like periodic label image of ``shape`` (an int means a cube)."""
    if np.isscalar(shape):
        shape = (int(shape),) * 3
    if low_to_high is None:
        low_to_high = list(range(len(fracs)))[::-1]
    v = smoothed_noise(shape, sigma, seed)
    return np.ascontiguousarray(threshold(v, fracs, low_to_high))


def two_phase(n, porosity=0.20, sigma=2.0, seed=0):
    """Quartz (label 0) / pore (label 1) image: the 32^3 plain-solve case."""
    return rocklike(n, [1.0 - porosity, porosity], sigma, seed, [1, 0])


def four_phase(n, sigma=2.0, seed=1):
    """Quartz/feldspar/clay/pore (labels 0..3) image at 0.55/0.15/0.10/0.20."""
    return rocklike(n, FOUR_PHASE["fracs"], sigma, seed, FOUR_PHASE["low_to_high"])


def laminate(shape, thickness, axis=0, first=0, second=1):
    """Periodic two-phase laminate: layers of ``thickness`` voxels normal to
    array ``axis`` (0 = z, 1 = y, 2 = x), alternating labels."""
    if np.isscalar(shape):
        shape = (int(shape),) * 3
    idx = np.arange(shape[axis])
    layer = np.where((idx // thickness) % 2 == 0, first, second).astype(np.uint8)
    sl = [None, None, None]
    sl[axis] = slice(None)
    return np.ascontiguousarray(np.broadcast_to(layer[tuple(sl)], shape))


def compress_contrast(moduli, max_ratio=50.0):
    """Scale a set of (K, G) pairs in log space about their geometric mean so
    that max/min over all entries is at most ``max_ratio``."""
    m = np.asarray(moduli, dtype=np.float64)
    lg = np.log(m)
    span = lg.max() - lg.min()
    if span <= np.log(max_ratio):
        return [tuple(r) for r in m]
    centre = 0.5 * (lg.max() + lg.min())
    s = np.log(max_ratio) / span
    return [tuple(r) for r in np.exp(centre + (lg - centre) * s)]


def uneven_batch(count, sizes=(32, 48, 64, 96), seed=1234, max_ratio=50.0):
    """Recipe for a batch of independent items of mixed cube sizes.

    Each item draws a size, 2-4 phases from the phase table (moduli
    log-compressed so that max/min <= ``max_ratio``), Dirichlet fractions and
    a smoothing length; the image itself comes from :func:`item_image`.
    Returns a list of dicts (size, phases, fracs, sigma, seed).
    """
    rng = np.random.default_rng(seed)
    items = []
    for i in range(count):
        n = int(rng.choice(sizes))
        m = int(rng.integers(2, 5))
        pick = rng.choice(len(PHASE_TABLE), size=m, replace=False)
        phases = compress_contrast([PHASE_TABLE[j] for j in pick], max_ratio)
        fr = rng.dirichlet(np.full(m, 2.0))
        fr = np.maximum(fr, 0.05)
        fr = fr / fr.sum()
        sigma = float(rng.uniform(1.5, 3.0))
        items.append(dict(size=n, phases=phases, fracs=[float(f) for f in fr],
                          sigma=sigma, seed=int(seed * 100003 + i)))
    return items


def item_image(item):
    """Label image of one :func:`uneven_batch` item."""
    m = len(item["fracs"])
    return rocklike(item["size"], item["fracs"], item["sigma"], item["seed"],
                    list(range(m)))


def correlation_x(labels, solid_label=0, max_lag=10):
    """Two-point correlation along x of the indicator of ``solid_label``
    (Sec. 2, eq_correlation), for lags 0..max_lag (periodic)."""
    m = (labels == solid_label).astype(np.float64)
    mean = m.mean()
    var = (m * m).mean() - mean * mean
    out = []
    for l in range(max_lag + 1):
        out.append(((m * np.roll(m, -l, axis=2)).mean() - mean * mean) / var)
    return np.asarray(out)


# ---------------------------------------------------------------------------
# The same recipe on a torch device, for images too large to make quickly on
# the host (the 1024^3 surrogate workload and its training images).  Same
# steps - standard-normal noise, periodic Gaussian smoothing with the kernel
# sampled at integer offsets up to 4 sigma and normalised to sum 1, quantile
# thresholds with linear interpolation - but a different random stream, so the
# images are statistically, not bitwise, equal to the host generator's.
# ---------------------------------------------------------------------------
def smoothed_noise_device(shape, sigma, seed, device="cuda"):
    import torch
    shape = tuple(int(s) for s in shape)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    w = torch.randn(shape, generator=gen, device=device, dtype=torch.float32)
    if sigma > 0:
        r = int(4.0 * sigma + 0.5)
        x = np.arange(-r, r + 1, dtype=np.float64)
        k = np.exp(-0.5 * (x / sigma) ** 2)
        k /= k.sum()
        for axis in range(3):
            acc = torch.zeros_like(w)
            for j, kj in enumerate(k):
                acc.add_(torch.roll(w, shifts=r - j, dims=axis), alpha=float(kj))
            w = acc
    return w


def threshold_device(values, fracs, low_to_high):
    import torch
    fracs = np.asarray(fracs, dtype=np.float64)
    if np.any(fracs < 0) or abs(fracs.sum() - 1.0) > 1e-9:
        raise ValueError("fractions must be non-negative and sum to 1")
    order = list(low_to_high)
    if sorted(order) != list(range(len(fracs))):
        raise ValueError("low_to_high must be a permutation of the labels")
    cum = np.cumsum([fracs[l] for l in order])[:-1]
    flat = values.reshape(-1)
    srt = torch.sort(flat).values
    n = flat.numel()
    cuts = []
    for q in cum:
        pos = q * (n - 1)
        lo = int(np.floor(pos))
        hi = min(lo + 1, n - 1)
        a, b = float(srt[lo]), float(srt[hi])
        cuts.append(a + (pos - lo) * (b - a))
    del srt
    bins = torch.bucketize(flat, torch.tensor(cuts, dtype=flat.dtype, device=flat.device), right=True)
    lut = torch.tensor(order, dtype=torch.uint8, device=flat.device)
    return lut[bins].reshape(values.shape)


def rocklike_device(shape, fracs, sigma=2.0, seed=0, low_to_high=None, device="cuda"):
    """Rock-like periodic label image as a uint8 torch tensor on ``device``."""
    if np.isscalar(shape):
        shape = (int(shape),) * 3
    if low_to_high is None:
        low_to_high = list(range(len(fracs)))[::-1]
    v = smoothed_noise_device(shape, sigma, seed, device)
    return threshold_device(v, fracs, low_to_high).contiguous()


def four_phase_device(n, sigma=2.0, seed=1, device="cuda"):
    return rocklike_device(n, FOUR_PHASE["fracs"], sigma, seed, FOUR_PHASE["low_to_high"], device)
