"""Dense brute-force solve of the discrete periodic problem -- FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Independent of the FFT/CG route in ``galerkin``: it never applies a
projection.  The discrete problem of Appendix A (trigonometric collocation,
trapezoidal quadrature) is: find the periodic displacement u whose nodal
strain eps* = sym(D u) minimises sum_x (E + eps*) : C(x) : (E + eps*), where
D is the spectral derivative on the grid, here assembled as explicit real
matrices from the DFT matrix and the wave numbers (with the same Nyquist
reading as the oracle: the Nyquist wavenumber component is zero).  The normal
equations B^T C B u = -B^T C E are solved by least squares (their null space
holds rigid translations and the Nyquist modes).  Tiny grids only.

Under the other even-grid reading (``nyquist='zero'``: the operator vanishes
at every frequency with a Nyquist component) the trial displacements are
restricted instead: u = Phi v, with Phi the real filter that removes every
Fourier mode having a Nyquist index on some axis, so the strains range over
exactly the compatible fields without support on those frequencies.
"""
from __future__ import annotations

import numpy as np

from . import galerkin as g


def derivative_matrix(n, nyquist="component"):
    """Real n x n matrix of the spectral derivative d/dx on a unit-spaced periodic grid."""
    j = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(j, j) / n)
    m = np.rint(np.fft.fftfreq(n) * n)
    k = m / n
    if nyquist == "component" and n % 2 == 0:
        k = np.where(np.abs(m) == n // 2, 0.0, k)
    D = (F.conj().T / n) @ np.diag(2j * np.pi * k) @ F
    if np.abs(D.imag).max() > 1e-10:
        raise ValueError("derivative not real under this Nyquist reading")
    return D.real


def nyquist_filter(n):
    """Real n x n projector onto the trigonometric modes of an n-point periodic
    grid other than the Nyquist mode (the identity for odd n)."""
    j = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(j, j) / n)
    m = np.rint(np.fft.fftfreq(n) * n)
    keep = ~((n % 2 == 0) & (np.abs(m) == n // 2))
    Phi = (F.conj().T / n) @ np.diag(keep.astype(float)) @ F
    if np.abs(Phi.imag).max() > 1e-10:
        raise ValueError("filter not real")
    return Phi.real


def gradient_matrices(shape, nyquist="component"):
    """(Dx, Dy, Dz) acting on fields flattened in C order [z][y][x].  With
    nyquist='zero' each derivative acts on the Nyquist-filtered field."""
    if nyquist == "zero":
        nz, ny, nx = shape
        Fz, Fy, Fx = (nyquist_filter(n) for n in (nz, ny, nx))
        dz, dy, dx = (derivative_matrix(n) @ f for n, f in ((nz, Fz), (ny, Fy), (nx, Fx)))
        return (np.kron(Fz, np.kron(Fy, dx)), np.kron(Fz, np.kron(dy, Fx)), np.kron(dz, np.kron(Fy, Fx)))
    nz, ny, nx = shape
    Iz, Iy, Ix = np.eye(nz), np.eye(ny), np.eye(nx)
    Dx = np.kron(Iz, np.kron(Iy, derivative_matrix(nx, nyquist)))
    Dy = np.kron(Iz, np.kron(derivative_matrix(ny, nyquist), Ix))
    Dz = np.kron(derivative_matrix(nz, nyquist), np.kron(Iy, Ix))
    return Dx, Dy, Dz


def strain_operator(shape, nyquist="component"):
    """B: u (3V) -> sym grad u as full 3x3 components (9V), component-major."""
    V = int(np.prod(shape))
    D = gradient_matrices(shape, nyquist)
    B = np.zeros((9 * V, 3 * V))
    for i in range(3):
        for j in range(3):
            row = (3 * i + j) * V
            # eps_ij = (d_j u_i + d_i u_j) / 2
            B[row:row + V, i * V:(i + 1) * V] += 0.5 * D[j]
            B[row:row + V, j * V:(j + 1) * V] += 0.5 * D[i]
    return B


def stiffness_matrix(medium):
    """Block operator of C(x) on 9V-vectors (component-major, voxel-minor)."""
    C = medium.tensor_field().reshape(3, 3, 3, 3, -1)
    V = C.shape[-1]
    M = np.zeros((9 * V, 9 * V))
    idx = np.arange(V)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    M[(3 * i + j) * V + idx, (3 * k + l) * V + idx] = C[i, j, k, l]
    return M


def solve_load(medium, E, nyquist="component"):
    """eps* (3,3,nz,ny,nx) minimising the discrete energy for strain E."""
    shape = tuple(medium.shape)
    V = int(np.prod(shape))
    B = strain_operator(shape, nyquist)
    M = stiffness_matrix(medium)
    e = np.repeat(E.reshape(9), V)
    K = B.T @ M @ B
    f = -B.T @ (M @ e)
    u, *_ = np.linalg.lstsq(K, f, rcond=1e-12)
    return (B @ u).reshape((3, 3) + shape)


def homogenize(medium, region=None, nyquist="component"):
    """C_R = Sigma_R E_R^-1 from the dense solves (same averaging as Sec. 4)."""
    sl = (slice(None), slice(None)) + g.region_slices(medium.shape, region)
    Sigma = np.zeros((6, 6))
    Eps = np.zeros((6, 6))
    for a in range(6):
        E = g.unit_strain(a)
        eps = E[:, :, None, None, None] + solve_load(medium, E, nyquist)
        sig = medium.stress(eps)
        Sigma[:, a] = g.stress_voigt(sig[sl].mean(axis=(-3, -2, -1)))
        Eps[:, a] = g.strain_voigt(eps[sl].mean(axis=(-3, -2, -1)))
    return np.linalg.solve(Eps.T, Sigma.T).T
