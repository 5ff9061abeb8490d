"""Rigorous bounds and closed forms used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names the Voigt-Reuss and Hashin-Shtrikman bounds (Sec. 1) as the
classical but loose alternatives to computation; here they, and two textbook
closed forms, serve as independent checks of the computed stiffness:

* Voigt / Reuss: <C> and <C^-1>^-1 bracket the homogenized stiffness in the
  quadratic-form sense (constant-strain and constant-stress trial fields).
* Hashin-Shtrikman bounds for isotropic multiphase mixtures (Berryman's form).
* Backus average of a periodic laminate (exact transversely isotropic result).
* Hill's result for phases of equal shear modulus: K* = <1/(K + 4mu/3)>^-1 - 4mu/3.
"""
from __future__ import annotations

import numpy as np

from . import galerkin as g


def fractions(labels, nphase):
    return np.bincount(np.asarray(labels).ravel(), minlength=nphase) / labels.size


def iso_voigt_matrix(K, G):
    return g.tensor_to_voigt(g.iso_tensor(K, G))


def voigt_reuss(labels, phases):
    """(C_Voigt, C_Reuss) as 6x6 Voigt matrices."""
    f = fractions(labels, len(phases))
    Cs = [iso_voigt_matrix(K, G) for K, G in phases]
    CV = sum(fi * C for fi, C in zip(f, Cs))
    SR = sum(fi * np.linalg.inv(C) for fi, C in zip(f, Cs))
    return CV, np.linalg.inv(SR)


def hashin_shtrikman(f, K, G):
    """((K_lo, K_hi), (G_lo, G_hi)) for isotropic phases with fractions f."""
    f, K, G = (np.asarray(a, dtype=np.float64) for a in (f, K, G))

    def lam(z):
        return 1.0 / np.sum(f / (K + 4.0 * z / 3.0)) - 4.0 * z / 3.0

    def gam(z):
        return 1.0 / np.sum(f / (G + z)) - z

    def zeta(k, m):
        return m / 6.0 * (9.0 * k + 8.0 * m) / (k + 2.0 * m)

    return ((lam(G.min()), lam(G.max())),
            (gam(zeta(K.min(), G.min())), gam(zeta(K.max(), G.max()))))


def backus(f, phases):
    """Effective 6x6 stiffness of a laminate with layer normal along x3."""
    f = np.asarray(f, dtype=np.float64)
    lam = np.array([K - 2.0 * G / 3.0 for K, G in phases])
    mu = np.array([G for _, G in phases])
    M = lam + 2.0 * mu
    avg = lambda a: float(np.sum(f * a))
    C33 = 1.0 / avg(1.0 / M)
    C13 = avg(lam / M) * C33
    C44 = 1.0 / avg(1.0 / mu)
    C66 = avg(mu)
    C11 = avg(4.0 * mu * (lam + mu) / M) + avg(lam / M) ** 2 * C33
    C12 = C11 - 2.0 * C66
    C = np.zeros((6, 6))
    C[0, 0] = C[1, 1] = C11
    C[0, 1] = C[1, 0] = C12
    C[0, 2] = C[2, 0] = C[1, 2] = C[2, 1] = C13
    C[2, 2] = C33
    C[3, 3] = C[4, 4] = C44
    C[5, 5] = C66
    return C


def hill_equal_shear(f, K, mu):
    """Exact bulk modulus of any mixture whose phases share the shear modulus mu."""
    f, K = np.asarray(f, dtype=np.float64), np.asarray(K, dtype=np.float64)
    return 1.0 / np.sum(f / (K + 4.0 * mu / 3.0)) - 4.0 * mu / 3.0
