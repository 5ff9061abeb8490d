"""Hierarchical homogenization, moduli and the n^-1 fit -- FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps in the paper's order (Sec. 3, Fig. 2; Sec. 4, Fig. 4; Sec. 5):

1. Partition the N^3 image into (N/n)^3 subimages of n^3 voxels (Sec. 3).
2. For each subimage take the box Omega_B = subimage plus p voxels of the
   surrounding material on every side (Sec. 4, Fig. 4); at the image edge the
   surround wraps periodically (reading: the paper does not say).
3. Homogenize the box under periodic boundary conditions and average over the
   central region Omega_R only: C_R = Sigma_R E_R^-1 (Sec. 4).
4. Assemble the intermediate (N/n)^3 image whose voxels carry C_R (Sec. 3);
   the symmetric part (C_R + C_R^T)/2 is used (reading: with padding C_R is
   not exactly symmetric and the second solve needs a self-adjoint operator).
5. Homogenize the intermediate image with the same periodic solver and an
   anisotropic law per voxel (Sec. 4, closing paragraph) -> C*.
   ``hierarchical_levels`` repeats steps 1-4 on the intermediate image
   before step 5 (more than two levels).
6. Bulk and shear moduli (reading: Voigt isotropic projection of C*) and the
   fit M(n) = M_inf + c n^-1 (Sec. 5, eq_fit_power_law) by unweighted least
   squares (reading: the fitting method is not stated).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import galerkin as g

UPPER = [(i, j) for i in range(6) for j in range(i, 6)]


def to21(C):
    """Upper triangle (row-major) of a 6x6 Voigt matrix."""
    return np.array([C[i, j] for (i, j) in UPPER])


def from21(c):
    C = np.zeros((6, 6))
    for v, (i, j) in zip(c, UPPER):
        C[i, j] = C[j, i] = v
    return C


def partition(labels, n):
    """Block origins (z, y, x) of the (N/n)^3 subimages, C order."""
    N = labels.shape
    if any(s % n for s in N):
        raise ValueError("the subimage size must divide the image size")
    return [(z, y, x) for z in range(0, N[0], n) for y in range(0, N[1], n)
            for x in range(0, N[2], n)]


def padded_box(labels, origin, n, p):
    """Omega_B: the n^3 block at ``origin`` plus p voxels of surround, wrapped."""
    z, y, x = origin
    iz = np.arange(z - p, z + n + p) % labels.shape[0]
    iy = np.arange(y - p, y + n + p) % labels.shape[1]
    ix = np.arange(x - p, x + n + p) % labels.shape[2]
    return labels[np.ix_(iz, iy, ix)]


@dataclass
class HierResult:
    C: np.ndarray              # final C* (6x6 Voigt)
    C_sub: np.ndarray          # (m, m, m, 6, 6) symmetric subimage stiffnesses
    C_sub_raw: np.ndarray      # raw Sigma E^-1 per subimage
    level2: g.Homogenized
    subs: list


def subimage_stiffness(labels, phases, n, p, **kw):
    """Steps 1-3 for every subimage; returns raw C_R per block in C order."""
    out = []
    for origin in partition(labels, n):
        box = padded_box(labels, origin, n, p)
        region = (p, p, p, p + n, p + n, p + n)
        out.append(g.homogenize(g.IsotropicMedium(box, phases), region=region, **kw))
    return out


def hierarchical(labels, phases, n, p=0, level2_kw=None, **kw):
    """Two-level hierarchical homogenization of Sec. 3 -> HierResult."""
    subs = subimage_stiffness(labels, phases, n, p, **kw)
    m = tuple(s // n for s in labels.shape)
    raw = np.stack([s.C for s in subs]).reshape(m + (6, 6))
    symm = 0.5 * (raw + np.swapaxes(raw, -1, -2))
    l2 = g.homogenize(g.AnisotropicMedium(symm), **(level2_kw or kw))
    return HierResult(C=l2.C_sym, C_sub=symm, C_sub_raw=raw, level2=l2, subs=subs)


def padded_field_box(field, origin, n, p):
    """Omega_B of an intermediate image (m_z, m_y, m_x, 6, 6), wrapped."""
    z, y, x = origin
    iz = np.arange(z - p, z + n + p) % field.shape[0]
    iy = np.arange(y - p, y + n + p) % field.shape[1]
    ix = np.arange(x - p, x + n + p) % field.shape[2]
    return field[np.ix_(iz, iy, ix)]


def hierarchical_levels(labels, phases, levels, **kw):
    """Repeated coarse-graining (reading: Sec. 3's scheme applied again to its
    own intermediate image, as in the renormalization it is modelled on).

    ``levels`` = [(n_1, p_1), (n_2, p_2), ...]: the label image is cut into
    n_1^3 subimages with p_1 voxels of surround (steps 1-4); each further
    level cuts the current intermediate image into n_l^3 blocks of voxels
    with p_l voxels of surround, homogenizes each with the anisotropic law
    over its central n_l^3 region, and assembles the symmetric parts into the
    next intermediate image.  The last image is homogenized whole (step 5).
    Returns (C*, list of the intermediate images)."""
    n1, p1 = levels[0]
    subs = subimage_stiffness(labels, phases, n1, p1, **kw)
    m = tuple(s // n1 for s in labels.shape)
    raw = np.stack([s.C for s in subs]).reshape(m + (6, 6))
    field = 0.5 * (raw + np.swapaxes(raw, -1, -2))
    images = [field]
    for n, p in levels[1:]:
        if any(s % n for s in field.shape[:3]):
            raise ValueError("the block size must divide the intermediate image")
        out = []
        for origin in partition(field[..., 0, 0], n):
            box = padded_field_box(field, origin, n, p)
            region = (p, p, p, p + n, p + n, p + n)
            out.append(g.homogenize(g.AnisotropicMedium(box), region=region, **kw).C)
        m = tuple(s // n for s in field.shape[:3])
        raw = np.stack(out).reshape(m + (6, 6))
        field = 0.5 * (raw + np.swapaxes(raw, -1, -2))
        images.append(field)
    if field.shape[:3] == (1, 1, 1):
        return field[0, 0, 0].copy(), images
    return g.homogenize(g.AnisotropicMedium(field), **kw).C_sym, images


def arithmetic_mean_moduli(C_sub):
    """Arithmetic mean of the subimages' (K, G) (the AM comparator of Sec. 5)."""
    KG = np.array([voigt_moduli(C) for C in C_sub.reshape(-1, 6, 6)])
    return KG.mean(axis=0)


def voigt_moduli(C):
    """Bulk and shear moduli of the Voigt isotropic projection of a 6x6 stiffness."""
    d = C[0, 0] + C[1, 1] + C[2, 2]
    o = C[0, 1] + C[0, 2] + C[1, 2]
    s = C[3, 3] + C[4, 4] + C[5, 5]
    return (d + 2.0 * o) / 9.0, (d - o + 3.0 * s) / 15.0


def richardson(ns, values):
    """Least-squares fit of M(n) = M_inf + c / n (Sec. 5, eq_fit_power_law).

    ``values`` has shape (m, ...) for the m subimage sizes in ``ns``; returns
    (M_inf, c) with the trailing shape."""
    ns = np.asarray(ns, dtype=np.float64)
    v = np.asarray(values, dtype=np.float64)
    if len(ns) < 2 or len(set(ns.tolist())) < 2:
        raise ValueError("need at least two distinct subimage sizes")
    A = np.stack([np.ones_like(ns), 1.0 / ns], axis=1)
    coef, *_ = np.linalg.lstsq(A, v.reshape(len(ns), -1), rcond=None)
    return coef[0].reshape(v.shape[1:]), coef[1].reshape(v.shape[1:])
