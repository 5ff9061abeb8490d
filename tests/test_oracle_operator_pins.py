"""Pins of the oracle's reference-medium Green operator, its second even-grid
reading, the Hashin-Shtrikman bounds and the arithmetic-mean comparator.

Each check comes from outside the function it pins:

* Gamma0(lambda0, mu0) of the basic scheme (the Moulinec-Suquet operator
  cited in Appendix A) by the problem it solves, written with the dense
  real-space derivative matrices of ``oracle.brute``: Gamma0 tau is the
  compatible zero-mean strain e with div(C0 : e - tau) = 0, and Gamma0 fixes
  every compatible field after C0.
* nyquist='zero' (the even-grid reading that zeroes the operator at every
  frequency with a Nyquist component; Appendix A treats odd grids only) by a
  dense energy minimisation over displacements without Nyquist modes.
* Hashin-Shtrikman (the bounds named in Sec. 1) by the two-phase formulas of
  Hashin and Shtrikman (1963), by the collapse onto the phase moduli for
  identical phases, by the Reuss limit of a shear-free phase and by the
  Voigt-Reuss bracket.
* The arithmetic mean of subimage moduli (the AM comparator of Sec. 5) by a
  tiled cell and by isotropic subimages.
"""
import numpy as np
import pytest

from oracle import bounds, brute, galerkin as g, hier
from paper_2208_02320_amd import synth

QP = [synth.QUARTZ, synth.PORE]


def sym_field(rng, shape):
    return g.sym(rng.standard_normal((3, 3) + shape))


def compatible_field(shape, rng, nyquist="component"):
    """sym grad u of a random displacement, from the dense derivative matrices."""
    B = brute.strain_operator(shape, nyquist)
    u = rng.standard_normal(B.shape[1])
    return (B @ u).reshape((3, 3) + shape)


def divergence(s, shape, nyquist="component"):
    """(div s)_i = sum_j d_j s_ij with the dense spectral derivatives."""
    D = brute.gradient_matrices(shape, nyquist)
    V = int(np.prod(shape))
    return np.stack([sum(D[j] @ s[i, j].reshape(V) for j in range(3)) for i in range(3)])


def iso_apply(lam0, mu0, e):
    tr = e[0, 0] + e[1, 1] + e[2, 2]
    out = 2.0 * mu0 * e
    for i in range(3):
        out[i, i] = out[i, i] + lam0 * tr
    return out


MEDIA = [(0.0, 0.5), (30.0, 20.0), (-5.0, 12.0), (80.0, 3.0), (1.0, 1e-3)]


@pytest.mark.parametrize("shape", [(5, 4, 6), (3, 5, 5)])
@pytest.mark.parametrize("lam0,mu0", MEDIA)
def test_gamma0_solves_the_reference_medium_problem(shape, lam0, mu0):
    rng = np.random.default_rng(int(100 * mu0) + len(shape))
    fr = g.frequencies(shape)
    op = lambda th, f: g.gamma0(th, f, lam0, mu0)
    tau = sym_field(rng, shape)
    e = g.convolve(op, tau, fr)
    scale = np.abs(tau).max() / min(mu0, lam0 + 2 * mu0 / 3 if lam0 + 2 * mu0 / 3 > 0 else mu0)
    # compatible: in the range of sym grad (dense least squares, zero residual)
    B = brute.strain_operator(shape)
    u, *_ = np.linalg.lstsq(B, e.reshape(-1), rcond=1e-12)
    assert np.abs(B @ u - e.reshape(-1)).max() < 1e-10 * scale
    assert np.abs(e.mean(axis=(-3, -2, -1))).max() < 1e-12 * scale
    # equilibrium of C0 : e - tau
    assert np.abs(divergence(iso_apply(lam0, mu0, e) - tau, shape)).max() < 1e-10 * np.abs(tau).max()
    # Gamma0 (C0 : eps) = eps for every compatible eps
    eps = compatible_field(shape, rng)
    back = g.convolve(op, iso_apply(lam0, mu0, eps), fr)
    assert np.abs(back - eps).max() < 1e-11 * np.abs(eps).max()


def test_gamma0_plausible_mistakes_fail():
    """The check above rejects a wrong coefficient of the k^4 term and a
    dropped term of the first part (mistakes planted in copies, on the CPU)."""
    shape, lam0, mu0 = (5, 4, 6), 30.0, 20.0
    rng = np.random.default_rng(0)
    fr = g.frequencies(shape)
    k, s = fr.k, np.where(fr.dead, 1.0, fr.k2)
    d = np.eye(3)

    def gam(th, c2, drop):
        t1 = (np.einsum("ki,h...,j...->ijkh...", d, k, k) + np.einsum("hi,k...,j...->ijkh...", d, k, k)
              + np.einsum("kj,h...,i...->ijkh...", d, k, k)
              + (0 if drop else np.einsum("hj,k...,i...->ijkh...", d, k, k))) / (4.0 * mu0 * s)
        t2 = c2 * np.einsum("i...,j...,k...,h...->ijkh...", k, k, k, k) / (s * s)
        return np.where(fr.dead, 0.0, np.einsum("ijkh...,kh...->ij...", t1 - t2, th))

    eps = compatible_field(shape, rng)
    c_ok = (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0))
    ok = g.convolve(lambda th, f: gam(th, c_ok, False), iso_apply(lam0, mu0, eps), fr)
    assert np.abs(ok - eps).max() < 1e-11
    for c2, drop in ((lam0 / (mu0 * (lam0 + 2.0 * mu0)), False), (c_ok, True)):
        bad = g.convolve(lambda th, f: gam(th, c2, drop), iso_apply(lam0, mu0, eps), fr)
        assert np.abs(bad - eps).max() > 1e-3 * np.abs(eps).max()


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 5, 4), (6, 6, 6)])
def test_nyquist_zero_matches_restricted_brute_force(shape):
    """nyquist='zero' equals the energy minimiser over displacements with no
    Fourier mode that has a Nyquist index; it differs from the default."""
    lab = np.random.default_rng(sum(shape)).random(shape) < 0.35
    m = g.IsotropicMedium(lab.astype(np.uint8), QP)
    Cb = brute.homogenize(m, nyquist="zero")
    r = g.homogenize(m, tol=1e-12, form="sym6", nyquist="zero")
    assert g.rel_error(r.C, Cb) < 1e-10
    Cc = brute.homogenize(m)
    assert g.rel_error(Cb, Cc) > 1e-3


def test_nyquist_zero_brute_force_restricts_the_trial_space():
    """The restricted strains have no energy at frequencies with a Nyquist
    index, and on odd grids the restriction is empty."""
    shape = (4, 6, 4)
    e = compatible_field(shape, np.random.default_rng(5), nyquist="zero")
    eh = np.fft.fftn(e, axes=(-3, -2, -1))
    nz, ny, nx = shape
    assert np.abs(eh[..., nz // 2, :, :]).max() < 1e-10
    assert np.abs(eh[..., :, ny // 2, :]).max() < 1e-10
    assert np.abs(eh[..., :, :, nx // 2]).max() < 1e-10
    for n in (3, 5):
        assert np.allclose(brute.nyquist_filter(n), np.eye(n), atol=1e-13)


def hs_two_phase(f1, K1, G1, K2, G2):
    """Hashin-Shtrikman (1963) two-phase formulas with phase 1 as the
    comparison material: the upper bounds when phase 1 is the stiffer one in
    both moduli, the lower bounds when it is the softer one."""
    f2 = 1.0 - f1
    K = K1 + f2 / (1.0 / (K2 - K1) + f1 / (K1 + 4.0 * G1 / 3.0))
    G = G1 + f2 / (1.0 / (G2 - G1) + 2.0 * f1 * (K1 + 2.0 * G1) / (5.0 * G1 * (K1 + 4.0 * G1 / 3.0)))
    return K, G


@pytest.mark.parametrize("phases", [(synth.QUARTZ, synth.PORE), (synth.QUARTZ, synth.CLAY),
                                    ((76.0, 50.0), (21.0, 7.0))])
@pytest.mark.parametrize("f1", [0.1, 0.45, 0.8])
def test_hashin_shtrikman_two_phase_closed_form(phases, f1):
    (K1, G1), (K2, G2) = phases  # phase 1 stiffer in both moduli
    (klo, khi), (glo, ghi) = bounds.hashin_shtrikman([f1, 1 - f1], [K1, K2], [G1, G2])
    Ku, Gu = hs_two_phase(f1, K1, G1, K2, G2)
    Kl, Gl = hs_two_phase(1 - f1, K2, G2, K1, G1)
    assert np.isclose(khi, Ku, rtol=1e-13) and np.isclose(ghi, Gu, rtol=1e-13)
    assert np.isclose(klo, Kl, rtol=1e-13) and np.isclose(glo, Gl, rtol=1e-13)


def test_hashin_shtrikman_special_cases():
    K, G = np.array([37.0, 76.0, 21.0, 2.25]), np.array([44.0, 26.0, 7.0, 1.0])
    f = np.array(synth.FOUR_PHASE["fracs"])
    (klo, khi), (glo, ghi) = bounds.hashin_shtrikman(f, K, G)
    # inside Voigt-Reuss, lower below upper
    assert 1 / np.sum(f / K) <= klo <= khi <= np.sum(f * K)
    assert 1 / np.sum(f / G) <= glo <= ghi <= np.sum(f * G)
    # identical phases: both bounds are the phase moduli
    (a, b), (c, d) = bounds.hashin_shtrikman(f, np.full(4, 30.0), np.full(4, 12.0))
    assert np.allclose([a, b, c, d], [30.0, 30.0, 12.0, 12.0], rtol=1e-14)
    # a single phase present
    (a, b), (c, d) = bounds.hashin_shtrikman([0.0, 1.0, 0.0, 0.0], K, G)
    assert np.allclose([a, b, c, d], [76.0, 76.0, 26.0, 26.0], rtol=1e-13)
    # a phase without shear stiffness: the lower bulk bound is the Reuss average
    with np.errstate(divide="ignore"):
        (a, _), _ = bounds.hashin_shtrikman([0.3, 0.7], [2.25, 37.0], [0.0, 44.0])
    assert np.isclose(a, 1 / (0.3 / 2.25 + 0.7 / 37.0), rtol=1e-14)
    # equal shear moduli: the bulk bounds coincide with Hill's exact result
    (a, b), _ = bounds.hashin_shtrikman([0.4, 0.6], [10.0, 50.0], [7.0, 7.0])
    assert np.isclose(a, b, rtol=1e-14)
    # invariant under a relabelling of the phases
    p = [2, 0, 3, 1]
    assert np.allclose(bounds.hashin_shtrikman(f[p], K[p], G[p]), ((klo, khi), (glo, ghi)), rtol=1e-14)


def test_hashin_shtrikman_benchmark_intervals():
    """The intervals of the two benchmark phase sets: two-phase quartz/pore at
    porosity 0.2, and the four-phase fractions 0.55/0.15/0.10/0.20."""
    (klo, khi), (glo, ghi) = bounds.hashin_shtrikman([0.8, 0.2], [37.0, 2.25], [44.0, 1.0])
    assert np.allclose([klo, khi, glo, ghi], [11.707, 27.203, 7.772, 29.458], atol=6e-4)
    (klo, khi), (glo, ghi) = bounds.hashin_shtrikman([0.55, 0.15, 0.10, 0.20], [37.0, 76.0, 21.0, 2.25],
                                                     [44.0, 26.0, 7.0, 1.0])
    assert np.allclose([klo, khi, glo, ghi], [11.725, 29.042, 6.896, 23.779], atol=6e-4)


def test_arithmetic_mean_moduli():
    """The AM comparator of Sec. 5: a periodic tiling of one cell gives that
    cell's Voigt moduli; isotropic subimages give the means of their K and G."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((6, 6))
    cell = A @ A.T + 6 * np.eye(6)
    C_sub = np.broadcast_to(cell, (2, 3, 2, 6, 6)).copy()
    assert np.allclose(hier.arithmetic_mean_moduli(C_sub), hier.voigt_moduli(cell), rtol=1e-14)
    KG = np.array([(37.0, 44.0), (76.0, 26.0), (21.0, 7.0)])
    C_iso = np.stack([bounds.iso_voigt_matrix(K, G) for K, G in KG])
    assert np.allclose(hier.arithmetic_mean_moduli(C_iso), KG.mean(axis=0), rtol=1e-14)
    # the mean over a tiled image of two different cells weighs both equally
    C2 = np.stack([C_iso[0], C_iso[1]] * 4)
    assert np.allclose(hier.arithmetic_mean_moduli(C2), KG[:2].mean(axis=0), rtol=1e-14)
