"""FP64 reference of the surrogate's acceptance gate.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The gate is not part of the paper: it decides when a network prediction of
a subimage stiffness may replace the FFT solve of Sec. 4.  Written out from
its definition, with eigenvalues (the kernel uses Cholesky pivots):

* the prediction is the mean of the two networks' outputs (or the one
  output);
* in Mandel form M(C) = D C D, D = diag(1, 1, 1, sqrt2, sqrt2, sqrt2), the
  prediction must be positive definite;
* with t = bound_tol * ||M(C_a)||_F, both M(C_V) - M(C) + t I and
  M(C) - M(C_R) + t I must be positive definite, where C_V and C_R are the
  Voigt and Reuss stiffnesses of the subimage's phase fractions (the
  bracket of Sec. 1's classical bounds);
* with two networks, ||M(C_a) - M(C_b)||_F <= spread_tol ||M(C_a)||_F;
* input-space test, per network: with f_c the fraction of label c in the
  network's input window and (mu_c, s_c) the mean and inverse standard
  deviation of that fraction over the training windows, |f_c - mu_c| s_c
  <= z_max for every label with s_c > 0, and f_c = mu_c (to within half a
  voxel) for a label with s_c = 0; z_max = 0 skips the test;
* texture test, per network with interface statistics (mean m, inverse
  standard deviation s > 0 of the training windows' interface density):
  |d - m| s <= z_max, where d is the fraction of the window's face-adjacent
  voxel pairs (along each axis, inside the window) whose labels differ.

Any failed condition flags the item for the FFT solver.
"""
from __future__ import annotations

import numpy as np

from . import bounds
from .hier import from21

_D = np.diag([1.0, 1.0, 1.0, np.sqrt(2.0), np.sqrt(2.0), np.sqrt(2.0)])


def mandel(C):
    return _D @ np.asarray(C, dtype=np.float64) @ _D


def _pd(A):
    return bool(np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0.0)


def gate(c21a, c21b, CV, CR, spread_tol, bound_tol):
    """True when the item goes to the FFT solver.  c21a/c21b: 21 upper-
    triangle components (c21b may be None); CV, CR: 6x6 Voigt matrices."""
    Ma = mandel(from21(c21a))
    Mb = Ma if c21b is None else mandel(from21(c21b))
    M = 0.5 * (Ma + Mb)
    nrm = np.linalg.norm(Ma)
    if not _pd(M):
        return True
    t = bound_tol * nrm
    if not _pd(mandel(CV) - M + t * np.eye(6)):
        return True
    if not _pd(M - mandel(CR) + t * np.eye(6)):
        return True
    if c21b is not None and np.linalg.norm(Ma - Mb) > spread_tol * nrm:
        return True
    return False


def fractions_outside(window_labels, mu, sc, z_max):
    """True when the input-space test fails for one network's window."""
    if not z_max > 0.0:
        return False
    w = np.asarray(window_labels)
    nv = w.size
    for c in range(8):
        f = np.count_nonzero(w == c) / nv
        d = abs(f - mu[c])
        if (d * sc[c] > z_max) if sc[c] > 0.0 else (d > 0.5 / nv):
            return True
    return False


def interface_density(window_labels):
    """Fraction of the face-adjacent voxel pairs of a window whose labels
    differ, counted pair by pair over the three axes."""
    w = np.asarray(window_labels)
    nz, ny, nx = w.shape
    diff = pairs = 0
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                for dz, dy, dx in ((0, 0, 1), (0, 1, 0), (1, 0, 0)):
                    z2, y2, x2 = z + dz, y + dy, x + dx
                    if z2 < nz and y2 < ny and x2 < nx:
                        pairs += 1
                        diff += int(w[z, y, x] != w[z2, y2, x2])
    return diff / pairs


def interface_outside(window_labels, mean, scale, z_max):
    """True when the texture test fails for one network's window."""
    if not (z_max > 0.0 and scale > 0.0):
        return False
    return abs(interface_density(window_labels) - mean) * scale > z_max


def gate_margin(c21a, c21b, CV, CR, bound_tol):
    """Smallest eigenvalue over the three definiteness tests, relative to
    ||M(C_a)||_F: items with a margin near zero may go either way."""
    Ma = mandel(from21(c21a))
    Mb = Ma if c21b is None else mandel(from21(c21b))
    M = 0.5 * (Ma + Mb)
    nrm = np.linalg.norm(Ma)
    t = bound_tol * nrm
    ev = [np.linalg.eigvalsh(M).min(),
          np.linalg.eigvalsh(mandel(CV) - M + t * np.eye(6)).min(),
          np.linalg.eigvalsh(M - mandel(CR) + t * np.eye(6)).min()]
    return min(abs(e) for e in ev) / nrm


def core_bounds(box_labels, pad, n, phases):
    """Voigt and Reuss stiffness of the n^3 core of a padded box."""
    core = np.asarray(box_labels)[pad:pad + n, pad:pad + n, pad:pad + n]
    return bounds.voigt_reuss(core, phases)
