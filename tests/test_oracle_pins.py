"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: dense
brute force, closed forms (Backus laminate, Hill's equal-shear mixture,
homogeneous media), rigorous bounds, exact symmetries, and the algebraic
properties of the projection of Appendix A.
"""
import numpy as np
import pytest

from oracle import bounds, brute, galerkin as g, hier
from paper_2208_02320_amd import synth

QP = [synth.QUARTZ, synth.PORE]


def rand_labels(shape, frac=0.3, seed=0, nphase=2):
    rng = np.random.default_rng(seed)
    if nphase == 2:
        return (rng.random(shape) < frac).astype(np.uint8)
    return rng.integers(0, nphase, size=shape).astype(np.uint8)


# ---------------------------------------------------------------- Sec. 4 law

def test_constitutive_law_physical_meaning():
    """Hydrostatic strain gives 3K eps0 I; a pure shear gives 2 mu eps (Sec. 4)."""
    lab = np.zeros((2, 2, 2), np.uint8)
    m = g.IsotropicMedium(lab, [(37.0, 44.0)])
    e = np.zeros((3, 3, 2, 2, 2))
    for i in range(3):
        e[i, i] = 0.01
    s = m.stress(e)
    assert np.allclose(s[0, 0], 3 * 37.0 * 0.01) and np.allclose(s[0, 1], 0.0)
    e = np.zeros((3, 3, 2, 2, 2))
    e[0, 1] = e[1, 0] = 0.02
    s = m.stress(e)
    assert np.allclose(s[0, 1], 2 * 44.0 * 0.02) and np.allclose(s[0, 0], 0.0)


def test_constitutive_law_both_printed_forms_agree():
    """The tensor C_ijkl of Sec. 4 contracted with eps equals the explicit law."""
    lab = rand_labels((3, 4, 5), nphase=2)
    m = g.IsotropicMedium(lab, QP)
    eps = np.random.default_rng(1).standard_normal((3, 3, 3, 4, 5))
    eps = 0.5 * (eps + eps.transpose(1, 0, 2, 3, 4))
    s1 = m.stress(eps)
    s2 = np.einsum("ijkl...,kl...->ij...", m.tensor_field(), eps)
    assert np.abs(s1 - s2).max() < 1e-12


def test_isotropic_voigt_matrix_entries():
    C = bounds.iso_voigt_matrix(37.0, 44.0)
    assert np.isclose(C[0, 0], 37 + 4 * 44 / 3) and np.isclose(C[0, 1], 37 - 2 * 44 / 3)
    assert np.isclose(C[3, 3], 44.0)


def test_voigt_moduli_of_isotropic_tensor():
    K, G = hier.voigt_moduli(bounds.iso_voigt_matrix(21.0, 7.0))
    assert np.isclose(K, 21.0) and np.isclose(G, 7.0)


# ---------------------------------------------------------- Appendix A operator

@pytest.mark.parametrize("shape", [(5, 6, 7), (4, 4, 4)])
def test_projection_algebra(shape):
    """Both projections are idempotent and self-adjoint; gradients are fixed
    points of the paper's operator and symmetric gradients of the symmetric one."""
    rng = np.random.default_rng(2)
    fr = g.frequencies(shape)
    for proj in (g.project_paper, g.project_sym):
        a = rng.standard_normal((3, 3) + shape)
        b = rng.standard_normal((3, 3) + shape)
        if proj is g.project_sym:
            a, b = g.sym(a), g.sym(b)
        Pa = g.convolve(proj, a, fr)
        assert np.abs(g.convolve(proj, Pa, fr) - Pa).max() < 1e-12
        assert abs(g.inner(Pa, b) - g.inner(a, g.convolve(proj, b, fr))) < 1e-10
    # a gradient field: H_ij = d_j u_i built with the dense spectral derivative
    Dx, Dy, Dz = brute.gradient_matrices(shape)
    u = rng.standard_normal((3, int(np.prod(shape))))
    H = np.stack([np.stack([D @ u[i] for D in (Dx, Dy, Dz)]) for i in range(3)])
    H = H.reshape((3, 3) + shape)
    assert np.abs(g.convolve(g.project_paper, H, fr) - H).max() < 1e-11
    assert np.abs(g.convolve(g.project_sym, g.sym(H), fr) - g.sym(H)).max() < 1e-11


def test_gamma0_reference_half_is_symmetric_projection():
    """Gamma0(lambda0 = 0, mu0 = 1/2) is exactly the symmetric projection."""
    shape = (5, 4, 6)
    fr = g.frequencies(shape)
    t = g.sym(np.random.default_rng(3).standard_normal((3, 3) + shape)).astype(complex)
    assert np.abs(g.gamma0(t, fr, 0.0, 0.5) - g.project_sym(t, fr)).max() < 1e-13


def test_projection_zero_mean():
    fr = g.frequencies((4, 6, 5))
    t = np.random.default_rng(4).standard_normal((3, 3, 4, 6, 5))
    assert np.abs(g.convolve(g.project_paper, t, fr).mean(axis=(-3, -2, -1))).max() < 1e-14


# ----------------------------------------------------------- discrete solution

@pytest.mark.parametrize("shape", [(4, 4, 4), (5, 5, 5), (4, 5, 6)])
def test_fft_cg_matches_dense_brute_force(shape):
    m = g.IsotropicMedium(rand_labels(shape, seed=sum(shape)), QP)
    Cb = brute.homogenize(m)
    for form in ("paper9", "sym6"):
        r = g.homogenize(m, tol=1e-12, form=form)
        assert g.rel_error(r.C, Cb) < 1e-11, form


def test_dense_brute_force_with_region():
    m = g.IsotropicMedium(rand_labels((5, 6, 5), seed=7), QP)
    region = (1, 1, 1, 4, 5, 4)
    Cb = brute.homogenize(m, region=region)
    r = g.homogenize(m, region=region, tol=1e-12, form="sym6")
    assert g.rel_error(r.C, Cb) < 1e-10


def test_homogeneous_medium_exact():
    """C* = C_phase; the right-hand side is zero up to FFT rounding, so CG
    stops after at most one step."""
    lab = np.zeros((6, 5, 4), np.uint8)
    r = g.homogenize(g.IsotropicMedium(lab, [(37.0, 44.0)]), tol=1e-6)
    assert max(r.iters) <= 1
    C = r.C
    assert np.allclose(C, bounds.iso_voigt_matrix(37.0, 44.0), atol=1e-12)
    assert np.isclose(C[0, 0], 95.0 + 2.0 / 3.0) and np.isclose(C[0, 1], 7.0 + 2.0 / 3.0)


@pytest.mark.parametrize("n,t", [(8, 2), (9, 3), (7, 1)])
def test_laminate_equals_backus(n, t):
    """Layers normal to x3: exact on odd grids or with even layer thickness."""
    lab = synth.laminate(n, t, axis=0)
    f = bounds.fractions(lab, 2)
    r = g.homogenize(g.IsotropicMedium(lab, QP), tol=1e-12, form="sym6")
    assert g.rel_error(r.C, bounds.backus(f, QP)) < 1e-10


def test_backus_closed_form_values():
    """50/50 quartz(37,44)/pore(2.25,1) laminate: transversely isotropic values."""
    C = bounds.backus([0.5, 0.5], QP)
    assert np.allclose([C[0, 0], C[0, 1], C[0, 2], C[2, 2], C[3, 3], C[5, 5]],
                       [49.43857, 4.43857, 1.80297, 6.90792, 1.95556, 22.5], atol=1e-5)


@pytest.mark.parametrize("n", [5, 7])
def test_hill_equal_shear_modulus_odd_grid(n):
    """Phases sharing mu: C* is isotropic with Hill's exact bulk modulus."""
    ph = [(40.0, 10.0), (5.0, 10.0), (15.0, 10.0)]
    lab = rand_labels((n, n, n), seed=n, nphase=3)
    r = g.homogenize(g.IsotropicMedium(lab, ph), tol=1e-12, form="sym6")
    f = bounds.fractions(lab, 3)
    Kh = bounds.hill_equal_shear(f, [p[0] for p in ph], 10.0)
    assert g.rel_error(r.C, bounds.iso_voigt_matrix(Kh, 10.0)) < 1e-10


@pytest.mark.parametrize("shape,seed", [((8, 8, 8), 0), ((7, 9, 6), 1)])
def test_voigt_reuss_bounds(shape, seed):
    lab = rand_labels(shape, seed=seed, nphase=3)
    ph = [synth.QUARTZ, synth.CLAY, synth.PORE]
    r = g.homogenize(g.IsotropicMedium(lab, ph), tol=1e-10, form="sym6")
    CV, CR = bounds.voigt_reuss(lab, ph)
    s = np.outer(g.mandel_scale(), g.mandel_scale())
    assert np.linalg.eigvalsh((CV - r.C_sym) * s).min() > 0
    assert np.linalg.eigvalsh((r.C_sym - CR) * s).min() > 0


def test_symmetric_positive_definite():
    lab = rand_labels((6, 7, 8), seed=5, nphase=3)
    r = g.homogenize(g.IsotropicMedium(lab, [synth.QUARTZ, synth.FELDSPAR, synth.PORE]),
                     tol=1e-12, form="sym6")
    assert np.abs(r.C - r.C.T).max() < 1e-9 * np.abs(r.C).max()
    assert np.linalg.eigvalsh(r.C_sym).min() > 0


def test_axis_permutation_covariance():
    """Swapping image axes x<->z permutes the stiffness indices 1<->3."""
    lab = rand_labels((4, 5, 6), seed=9)
    r = g.homogenize(g.IsotropicMedium(lab, QP), tol=1e-12, form="sym6")
    rt = g.homogenize(g.IsotropicMedium(np.ascontiguousarray(lab.transpose(2, 1, 0)), QP),
                      tol=1e-12, form="sym6")
    Q = np.zeros((3, 3))
    Q[0, 2] = Q[1, 1] = Q[2, 0] = 1.0
    Ct = g.tensor_to_voigt(np.einsum("ia,jb,kc,ld,abcd->ijkl", Q, Q, Q, Q,
                                     g.voigt_to_tensor(r.C)))
    assert g.rel_error(rt.C, Ct) < 1e-11


def test_mirror_flips_odd_couplings():
    lab = rand_labels((5, 6, 7), seed=11)
    r = g.homogenize(g.IsotropicMedium(lab, QP), tol=1e-12, form="sym6")
    rm = g.homogenize(g.IsotropicMedium(np.ascontiguousarray(lab[:, :, ::-1]), QP),
                      tol=1e-12, form="sym6")
    nx = np.array([sum(1 for q in ij if q == 0) for ij in g.VOIGT])
    sign = (-1.0) ** (nx[:, None] + nx[None, :])
    assert g.rel_error(rm.C, sign * r.C) < 1e-11


def test_translation_invariance():
    lab = rand_labels((6, 5, 4), seed=13)
    r = g.homogenize(g.IsotropicMedium(lab, QP), tol=1e-12, form="sym6")
    rs = g.homogenize(g.IsotropicMedium(np.roll(lab, (2, 1, 3), axis=(0, 1, 2)), QP),
                      tol=1e-12, form="sym6")
    assert g.rel_error(rs.C, r.C) < 1e-11


def test_variants_reach_the_same_solution():
    """Paper's 9-component form, symmetric form and basic fixed point agree."""
    m = g.IsotropicMedium(rand_labels((6, 7, 8), seed=3), QP)
    r9 = g.homogenize(m, tol=1e-11, form="paper9")
    r6 = g.homogenize(m, tol=1e-11, form="sym6")
    rb = g.homogenize(m, tol=1e-11, scheme="basic")
    assert g.rel_error(r6.C, r9.C) < 1e-10
    assert g.rel_error(rb.C, r9.C) < 1e-9
    assert max(r6.iters) < max(r9.iters) < max(rb.iters)


def test_nyquist_readings():
    """No Nyquist frequency on odd grids: readings agree; on even grids they differ."""
    m = g.IsotropicMedium(rand_labels((5, 5, 5), seed=2), QP)
    a = g.homogenize(m, tol=1e-12, nyquist="component", form="sym6").C
    b = g.homogenize(m, tol=1e-12, nyquist="zero", form="sym6").C
    assert g.rel_error(a, b) < 1e-12
    m = g.IsotropicMedium(rand_labels((6, 6, 6), seed=2), QP)
    a = g.homogenize(m, tol=1e-12, nyquist="component", form="sym6").C
    b = g.homogenize(m, tol=1e-12, nyquist="zero", form="sym6").C
    assert g.rel_error(a, b) > 1e-3


def test_anisotropic_medium_matches_isotropic_medium():
    lab = rand_labels((4, 5, 6), seed=4)
    iso = g.IsotropicMedium(lab, QP)
    Cs = np.stack([bounds.iso_voigt_matrix(K, G) for K, G in QP])[lab]
    r1 = g.homogenize(iso, tol=1e-12, form="sym6")
    r2 = g.homogenize(g.AnisotropicMedium(Cs), tol=1e-12, form="sym6")
    assert g.rel_error(r2.C, r1.C) < 1e-12


def test_anisotropic_brute_force():
    rng = np.random.default_rng(8)
    A = rng.standard_normal((4, 4, 5, 6, 6))
    Cv = np.einsum("...ij,...kj->...ik", A, A) + 5 * np.eye(6)
    m = g.AnisotropicMedium(Cv)
    r = g.homogenize(m, tol=1e-12, form="sym6")
    assert g.rel_error(r.C, brute.homogenize(m)) < 1e-10


# ------------------------------------------------------------------ hierarchy

def test_partition_and_wrapped_padding():
    lab = np.arange(6 * 6 * 6, dtype=np.int64).reshape(6, 6, 6) % 251
    assert len(hier.partition(lab, 3)) == 8
    box = hier.padded_box(lab, (3, 0, 3), 3, 1)
    assert box.shape == (5, 5, 5)
    assert box[0, 0, 0] == lab[2, 5, 2] and box[4, 4, 4] == lab[0, 3, 0]
    with pytest.raises(ValueError):
        hier.partition(lab, 4)


def test_hierarchy_exact_for_tiled_cell():
    """A period-n tiling: brute force, HH(n, p=0) and HH(n, 2p = n) all equal C_cell."""
    cell = rand_labels((6, 6, 6), seed=21)
    big = np.tile(cell, (2, 2, 2))
    kw = dict(tol=1e-12, form="sym6")
    Cc = g.homogenize(g.IsotropicMedium(cell, QP), **kw).C
    Cb = g.homogenize(g.IsotropicMedium(big, QP), **kw).C
    assert g.rel_error(Cb, Cc) < 1e-11
    assert g.rel_error(hier.hierarchical(big, QP, 6, 0, **kw).C, Cc) < 1e-10
    assert g.rel_error(hier.hierarchical(big, QP, 6, 3, **kw).C, Cc) < 1e-10


def test_padding_reduces_hierarchy_error():
    """Sec. 5 observation on a synthetic image: padding lowers the HH error."""
    lab = synth.rocklike(16, [0.75, 0.25], sigma=1.5, seed=3, low_to_high=[1, 0])
    kw = dict(tol=1e-9, form="sym6")
    Cref = g.homogenize(g.IsotropicMedium(lab, QP), **kw).C
    e0 = g.rel_error(hier.hierarchical(lab, QP, 8, 0, **kw).C, Cref)
    e2 = g.rel_error(hier.hierarchical(lab, QP, 8, 2, **kw).C, Cref)
    assert e2 < e0


def test_richardson_recovers_exact_power_law():
    ns = [16, 32, 64, 128]
    Minf = np.array([[21.3, 1.0], [23.5, 2.0]])
    c = np.array([[58.9, -3.0], [74.9, 0.5]])
    vals = [Minf + c / n for n in ns]
    m, cc = hier.richardson(ns, vals)
    assert np.allclose(m, Minf, rtol=1e-13) and np.allclose(cc, c, rtol=1e-12)
    m2, _ = hier.richardson([32, 64], [vals[1], vals[2]])
    assert np.allclose(m2, (64 * vals[2] - 32 * vals[1]) / 32)


def test_upper_triangle_roundtrip():
    A = np.random.default_rng(0).standard_normal((6, 6))
    S = A + A.T
    assert np.array_equal(hier.from21(hier.to21(S)), S)


# ----------------------------------------------------------- synthetic inputs

def test_generator_fractions_and_correlation():
    lab = synth.four_phase(32, seed=1)
    f = bounds.fractions(lab, 4)
    assert np.allclose(f, synth.FOUR_PHASE["fracs"], atol=2e-4)
    c = synth.correlation_x(synth.two_phase(32, seed=0), 0, 6)
    assert c[0] == 1.0 and np.all(np.diff(c) < 0) and 0.0 < c[5] < 0.3


def test_generator_deterministic():
    a = synth.four_phase(24, seed=5)
    b = synth.four_phase(24, seed=5)
    assert np.array_equal(a, b) and a.dtype == np.uint8 and a.flags.c_contiguous


def test_two_phase_32_within_hashin_shtrikman():
    """The 32^3 two-phase benchmark image: Voigt-projected moduli of C* lie in
    the Hashin-Shtrikman interval of its phase fractions."""
    lab = synth.two_phase(32, 0.2, 2.0, 0)
    r = g.homogenize(g.IsotropicMedium(lab, QP), tol=1e-6, form="sym6")
    K, G = hier.voigt_moduli(r.C_sym)
    f = bounds.fractions(lab, 2)
    (kl, kh), (gl, gh) = bounds.hashin_shtrikman(f, [37.0, 2.25], [44.0, 1.0])
    assert kl < K < kh and gl < G < gh
    assert max(r.iters) < 60
