"""Periodic Fourier-Galerkin elasticity solve -- FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
baseline of bench.py; never by the product path.  Shares no code with it.

What it computes (paper, Sec. 4 and Appendix A):

* Constitutive law (Sec. 4, the isotropic law following Fig. 4):
  sigma_ij = K eps_kk delta_ij + 2 mu (eps_ij - eps_kk delta_ij / 3); for the
  intermediate image a general anisotropic stiffness per voxel (Sec. 4,
  closing paragraph).
* Strain split eps = E + eps*, eps* periodic with zero mean (Sec. 4).
* Projection (Appendix A): G^_ijlm(k) = delta_im k_j k_l / |k|^2, G^(0) = 0,
  applied as [G * zeta]_ij = F^-1[ G^_ijkl zeta^_lk ]; with either index
  ordering printed in Appendix A this is (zeta^ k)_i k_j / |k|^2, i.e. the
  orthogonal projection onto gradient fields.
* Discrete equations (Appendix A, trigonometric collocation):
  G * (C : eps*) = - G * (C : E), solved by conjugate gradients.
* Averages over the region Omega_R and C_R = Sigma_R E_R^-1 (Sec. 4).

Readings where the paper is silent or garbled:

* Grid/frequency: arrays are indexed [z][y][x]; tensor index 0/1/2 is x/y/z;
  k_d = m_d / N_d with integer m_d in FFT order (unit voxel; the projection
  is 0-homogeneous in k so the scale is immaterial).
* Even N (Appendix A only treats odd N): ``nyquist='component'`` (default)
  sets the Nyquist wavenumber component k_d to 0; ``'zero'`` zeroes the
  operator at every frequency that has a Nyquist component; ``'naive'``
  keeps k_d = -1/2 (not Hermitian-consistent; the real part is taken).
* CG: x0 = 0, Frobenius inner product summed over voxels, stop when
  ||r|| <= tol ||b||; no iterations when b = 0.
* Voigt order (11, 22, 33, 23, 13, 12); strain vectors carry engineering
  shear strains (2 eps_ij); unit load a sets the a-th entry of that vector to 1.
* ``form='sym6'`` uses the symmetric projection onto compatible symmetric
  strains (the Green operator of an isotropic reference medium with
  lambda0 = 0, mu0 = 1/2); it has the same solution as the paper's form.
* ``scheme='basic'`` is the Moulinec-Suquet fixed point cited in Appendix A,
  eps <- eps - Gamma0 * sigma(eps), with lambda0, mu0 the mid-range of the
  phases; it reaches the same solution.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft

VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
_WORKERS = max(1, os.cpu_count() or 1)


def set_workers(n):
    """Number of threads scipy.fft may use (the oracle is otherwise serial)."""
    global _WORKERS
    _WORKERS = max(1, int(n))


def workers():
    return _WORKERS


# --------------------------------------------------------------------------
# Tensors and Voigt notation (Sec. 4)
# --------------------------------------------------------------------------

def lame(K, G):
    """(lambda, mu) of the isotropic tensor written in Sec. 4."""
    return K - 2.0 * G / 3.0, G


def iso_tensor(K, G):
    """C_ijkl = (K - 2G/3) d_ij d_kl + G (d_ik d_jl + d_il d_jk)  (Sec. 4)."""
    d = np.eye(3)
    lam, mu = lame(K, G)
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def voigt_to_tensor(Cv):
    """6x6 Voigt stiffness (engineering strains) -> C_ijkl (with minor symmetries)."""
    Cv = np.asarray(Cv, dtype=np.float64)
    C = np.zeros(Cv.shape[:-2] + (3, 3, 3, 3))
    for a, (i, j) in enumerate(VOIGT):
        for b, (k, l) in enumerate(VOIGT):
            v = Cv[..., a, b]
            C[..., i, j, k, l] = v
            C[..., j, i, k, l] = v
            C[..., i, j, l, k] = v
            C[..., j, i, l, k] = v
    return C


def tensor_to_voigt(C):
    """C_ijkl -> 6x6 Voigt matrix."""
    Cv = np.zeros(C.shape[:-4] + (6, 6))
    for a, (i, j) in enumerate(VOIGT):
        for b, (k, l) in enumerate(VOIGT):
            Cv[..., a, b] = C[..., i, j, k, l]
    return Cv


def stress_voigt(t):
    """Symmetric tensor(s) (3, 3, ...) -> Voigt stress vector(s) (6, ...)."""
    return np.stack([t[i, j] for (i, j) in VOIGT])


def strain_voigt(t):
    """Symmetric tensor(s) (3, 3, ...) -> Voigt strain vector(s), engineering shears."""
    return np.stack([t[i, j] * (1.0 if i == j else 2.0) for (i, j) in VOIGT])


def strain_from_voigt(v):
    """Voigt engineering strain vector (6,) -> symmetric 3x3 tensor."""
    e = np.zeros((3, 3))
    for a, (i, j) in enumerate(VOIGT):
        s = 1.0 if i == j else 0.5
        e[i, j] = v[a] * s
        e[j, i] = v[a] * s
    return e


def unit_strain(a):
    """The a-th of the six independent macroscopic strains (Sec. 4)."""
    v = np.zeros(6)
    v[a] = 1.0
    return strain_from_voigt(v)


def mandel_scale():
    """Diagonal scaling taking a Voigt stiffness to its Mandel (tensor-norm) form."""
    return np.array([1.0, 1.0, 1.0, np.sqrt(2.0), np.sqrt(2.0), np.sqrt(2.0)])


def rel_error(C, C_ref):
    """||C - C_ref||_F / ||C_ref||_F on the Mandel-scaled 6x6 matrices."""
    s = mandel_scale()
    M = np.outer(s, s)
    return float(np.linalg.norm((C - C_ref) * M) / np.linalg.norm(C_ref * M))


# --------------------------------------------------------------------------
# Media: sigma = C(x) : eps
# --------------------------------------------------------------------------

class IsotropicMedium:
    """Per-voxel isotropic phases selected by a label image (Sec. 4)."""

    def __init__(self, labels, phases):
        labels = np.asarray(labels)
        ph = np.asarray(phases, dtype=np.float64)
        if labels.ndim != 3:
            raise ValueError("labels must be a 3-D array [z][y][x]")
        if labels.size and int(labels.max()) >= len(ph):
            raise ValueError("label outside the phase table")
        if np.any(ph <= 0):
            raise ValueError("moduli must be positive")
        self.shape = labels.shape
        self.labels = labels
        self.phases = ph
        self.K = ph[:, 0][labels]
        self.G = ph[:, 1][labels]

    def stress(self, eps):
        """sigma_ij = K eps_kk d_ij + 2 mu (eps_ij - eps_kk d_ij / 3)."""
        tr = eps[0, 0] + eps[1, 1] + eps[2, 2]
        sig = 2.0 * self.G * eps
        for i in range(3):
            sig[i, i] = sig[i, i] + self.K * tr - 2.0 * self.G * tr / 3.0
        return sig

    def tensor_field(self):
        """C_ijkl per voxel, shape (3,3,3,3,nz,ny,nx)."""
        Cs = np.stack([iso_tensor(K, G) for K, G in self.phases])
        return np.moveaxis(Cs[self.labels], (0, 1, 2), (4, 5, 6))

    def bounds_moduli(self):
        return self.phases[:, 0], self.phases[:, 1]


class AnisotropicMedium:
    """Per-voxel general stiffness given as 6x6 Voigt matrices (nz,ny,nx,6,6)."""

    def __init__(self, Cv_field):
        Cv = np.asarray(Cv_field, dtype=np.float64)
        if Cv.ndim != 5 or Cv.shape[-2:] != (6, 6):
            raise ValueError("expected a (nz, ny, nx, 6, 6) stiffness field")
        self.shape = Cv.shape[:3]
        self.Cv = Cv
        self.C = np.moveaxis(voigt_to_tensor(Cv), (0, 1, 2), (4, 5, 6))

    def stress(self, eps):
        return np.einsum("ijkl...,kl...->ij...", self.C, eps)

    def tensor_field(self):
        return self.C


# --------------------------------------------------------------------------
# Frequencies and projection operators (Appendix A)
# --------------------------------------------------------------------------

@dataclass
class Frequencies:
    k: np.ndarray          # (3, nz, ny, nx): (k_x, k_y, k_z)
    k2: np.ndarray         # |k|^2
    dead: np.ndarray       # bool: operator is zero here


def frequencies(shape, nyquist="component"):
    """Wave vectors on the FFT grid of an [z][y][x] image of ``shape``."""
    if nyquist not in ("component", "zero", "naive"):
        raise ValueError("unknown Nyquist convention")
    nz, ny, nx = shape
    comps = []
    any_nyq = np.zeros(shape, dtype=bool)
    for axis, n in ((2, nx), (1, ny), (0, nz)):
        m = np.rint(np.fft.fftfreq(n) * n)
        k = m / n
        nyq = (n % 2 == 0) & (np.abs(m) == n // 2)
        if nyquist == "component":
            k = np.where(nyq, 0.0, k)
        view = [1, 1, 1]
        view[axis] = n
        comps.append(np.broadcast_to(k.reshape(view), shape))
        any_nyq |= np.broadcast_to(nyq.reshape(view), shape)
    k = np.stack(comps).astype(np.float64)
    k2 = np.sum(k * k, axis=0)
    dead = k2 == 0.0
    if nyquist == "zero":
        dead = dead | any_nyq
    return Frequencies(k=k, k2=k2, dead=dead)


def _safe(fr):
    return np.where(fr.dead, 1.0, fr.k2)


def project_paper(zh, fr):
    """Appendix A: [G^ zeta^]_ij = G^_ijkl zeta^_lk with G^_ijlm = d_im k_j k_l/|k|^2,
    which contracts to (zeta^ k)_i k_j / |k|^2; zero where the operator is dead."""
    k = fr.k
    zk = np.einsum("ik...,k...->i...", zh, k)
    out = np.einsum("i...,j...->ij...", zk, k) / _safe(fr)
    return np.where(fr.dead, 0.0, out)


def project_sym(th, fr):
    """Orthogonal projection onto compatible symmetric strains:
    [k_i (tau k)_j + k_j (tau k)_i] / |k|^2 - k_i k_j (k.tau.k) / |k|^4."""
    k = fr.k
    s = _safe(fr)
    tk = np.einsum("ij...,j...->i...", th, k)
    ktk = np.einsum("i...,i...->...", tk, k)
    out = (np.einsum("i...,j...->ij...", k, tk) + np.einsum("i...,j...->ij...", tk, k)) / s \
        - np.einsum("i...,j...->ij...", k, k) * ktk / (s * s)
    return np.where(fr.dead, 0.0, out)


def gamma0(th, fr, lam0, mu0):
    """Green operator of the isotropic reference medium (lambda0, mu0), in the
    textbook form of Moulinec & Suquet (cited in Appendix A):
    Gamma_ijkh = (d_ki k_h k_j + d_hi k_k k_j + d_kj k_h k_i + d_hj k_k k_i) / (4 mu0 |k|^2)
                 - (lam0 + mu0) / (mu0 (lam0 + 2 mu0)) k_i k_j k_k k_h / |k|^4."""
    k = fr.k
    s = _safe(fr)
    d = np.eye(3)
    t1 = (np.einsum("ki,h...,j...->ijkh...", d, k, k)
          + np.einsum("hi,k...,j...->ijkh...", d, k, k)
          + np.einsum("kj,h...,i...->ijkh...", d, k, k)
          + np.einsum("hj,k...,i...->ijkh...", d, k, k)) / (4.0 * mu0 * s)
    t2 = (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0)) * np.einsum(
        "i...,j...,k...,h...->ijkh...", k, k, k, k) / (s * s)
    G = t1 - t2
    out = np.einsum("ijkh...,kh...->ij...", G, th)
    return np.where(fr.dead, 0.0, out)


def fft3(f):
    return sfft.fftn(f, axes=(-3, -2, -1), workers=_WORKERS)


def ifft3(f):
    return sfft.ifftn(f, axes=(-3, -2, -1), workers=_WORKERS)


def convolve(proj, field_, fr):
    """[G * f](x) = F^-1[ G^(k) : F[f](k) ](x)  (Appendix A, FFT convolution)."""
    return ifft3(proj(fft3(field_), fr)).real


# --------------------------------------------------------------------------
# Solvers
# --------------------------------------------------------------------------

def inner(a, b):
    """Frobenius inner product summed over the grid (trapezoidal rule)."""
    return float(np.sum(a * b))


def sym(t):
    return 0.5 * (t + np.swapaxes(t, 0, 1))


@dataclass
class SolveInfo:
    iters: int
    rel_resid: float
    history: list = field(default_factory=list)
    converged: bool = True


def cg(apply_A, b, tol, maxit):
    """Conjugate gradients for A x = b from x0 = 0 (Appendix A, closing part)."""
    x = np.zeros_like(b)
    r = b.copy()
    bb = inner(b, b)
    if bb == 0.0:
        return x, SolveInfo(0, 0.0, [0.0], True)
    p = r.copy()
    rr = bb
    hist = [1.0]
    for it in range(1, maxit + 1):
        q = apply_A(p)
        alpha = rr / inner(p, q)
        x += alpha * p
        r -= alpha * q
        rr_new = inner(r, r)
        hist.append(np.sqrt(rr_new / bb))
        if np.sqrt(rr_new) <= tol * np.sqrt(bb):
            return x, SolveInfo(it, hist[-1], hist, True)
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, SolveInfo(maxit, hist[-1], hist, False)


def solve_load(medium, E, tol=1e-10, maxit=5000, form="paper9", scheme="cg",
               nyquist="component", ref=None):
    """Fluctuation eps* for one macroscopic strain E (3x3).

    form='paper9': unknown is a gradient field H* (9 components) with
    G * (C : sym(E + H*)) = 0, eps* = sym(H*) -- Appendix A as printed.
    form='sym6'  : unknown is a compatible symmetric strain with the
    symmetric projection.  scheme='basic' runs the fixed point instead of CG.
    """
    fr = frequencies(medium.shape, nyquist)
    Eg = np.broadcast_to(E[:, :, None, None, None], (3, 3) + tuple(medium.shape)).copy()
    if scheme == "basic":
        return _basic_scheme(medium, Eg, fr, tol, maxit, ref)
    if form == "paper9":
        proj = project_paper
        A = lambda h: convolve(proj, medium.stress(sym(h)), fr)
        b = -convolve(proj, medium.stress(Eg), fr)
        h, info = cg(A, b, tol, maxit)
        return sym(h), info
    if form == "sym6":
        proj = project_sym
        A = lambda e: convolve(proj, medium.stress(e), fr)
        b = -convolve(proj, medium.stress(Eg), fr)
        return cg(A, b, tol, maxit)
    raise ValueError("unknown form")


def _basic_scheme(medium, Eg, fr, tol, maxit, ref):
    """eps^{i+1} = eps^i - Gamma0 * sigma(eps^i), eps^0 = E; residual is the
    equilibrium residual || G * sigma || / || G * (C:E) ||."""
    if ref is None:
        if isinstance(medium, IsotropicMedium):
            lam, mu = lame(medium.phases[:, 0], medium.phases[:, 1])
            ref = (0.5 * (lam.min() + lam.max()), 0.5 * (mu.min() + mu.max()))
        else:
            raise ValueError("reference medium required for an anisotropic medium")
    lam0, mu0 = ref
    eps = Eg.copy()
    hist = []
    nb = None
    for it in range(0, maxit + 1):
        sh = fft3(medium.stress(eps))
        gs = ifft3(project_sym(sh, fr)).real
        res = np.sqrt(inner(gs, gs))
        if nb is None:
            nb = res
            if nb == 0.0:
                return eps - Eg, SolveInfo(0, 0.0, [0.0], True)
        hist.append(res / nb)
        if res <= tol * nb:
            return eps - Eg, SolveInfo(it, hist[-1], hist, True)
        if it == maxit:
            break
        eps = eps - ifft3(gamma0(sh, fr, lam0, mu0)).real
    return eps - Eg, SolveInfo(maxit, hist[-1], hist, False)


# --------------------------------------------------------------------------
# Homogenized stiffness of a region (Sec. 4)
# --------------------------------------------------------------------------

@dataclass
class Homogenized:
    C: np.ndarray            # raw Sigma_R E_R^-1 (6x6 Voigt)
    C_sym: np.ndarray        # (C + C^T)/2
    Sigma: np.ndarray        # columns: Voigt <sigma>_R per load
    Eps: np.ndarray          # columns: Voigt (engineering) <eps>_R per load
    infos: list

    @property
    def iters(self):
        return [i.iters for i in self.infos]

    @property
    def asym(self):
        return float(np.abs(self.C - self.C.T).max() / np.abs(self.C).max())


def region_slices(shape, region):
    """region = (x0, y0, z0, x1, y1, z1), half-open, or None for the whole box."""
    if region is None:
        return (slice(None),) * 3
    x0, y0, z0, x1, y1, z1 = region
    nz, ny, nx = shape
    if not (0 <= x0 < x1 <= nx and 0 <= y0 < y1 <= ny and 0 <= z0 < z1 <= nz):
        raise ValueError("region outside the box")
    return (slice(z0, z1), slice(y0, y1), slice(x0, x1))


def homogenize(medium, region=None, tol=1e-10, maxit=5000, form="paper9",
               scheme="cg", nyquist="component", loads=None, ref=None):
    """C_R = Sigma_R E_R^-1 from six independent macroscopic strains (Sec. 4)."""
    sl = (slice(None), slice(None)) + region_slices(medium.shape, region)
    Sigma = np.zeros((6, 6))
    Eps = np.zeros((6, 6))
    infos = []
    for a in range(6):
        E = unit_strain(a) if loads is None else strain_from_voigt(np.asarray(loads)[:, a])
        eps_star, info = solve_load(medium, E, tol, maxit, form, scheme, nyquist, ref)
        eps = E[:, :, None, None, None] + eps_star
        sig = medium.stress(eps)
        s_avg = sig[sl].mean(axis=(-3, -2, -1))
        e_avg = eps[sl].mean(axis=(-3, -2, -1))
        Sigma[:, a] = stress_voigt(s_avg)
        Eps[:, a] = strain_voigt(e_avg)
        infos.append(info)
    C = np.linalg.solve(Eps.T, Sigma.T).T
    return Homogenized(C=C, C_sym=0.5 * (C + C.T), Sigma=Sigma, Eps=Eps, infos=infos)


def homogenize_labels(labels, phases, **kw):
    return homogenize(IsotropicMedium(labels, phases), **kw)
