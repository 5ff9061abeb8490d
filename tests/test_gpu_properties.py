"""Properties of the GPU result that hold for any microstructure, checked on
the HIP path directly (the oracle meets the same ones in the CPU pins):
symmetry and positive definiteness of C, the Voigt-Reuss bracket, covariance
under axis permutations, invariance under periodic translation, and
exactness of the two-level scheme on periodic tilings (Sec. 3: a tiling of
one block makes every subimage, and the intermediate image, that block).
"""
import numpy as np
import pytest

from oracle import bounds
from oracle import galerkin as g
from oracle import hier
from paper_2208_02320_amd import synth

pytestmark = pytest.mark.gpu

PH3 = [synth.QUARTZ, synth.FELDSPAR, synth.PORE]
TOL32 = 1e-5
MANDEL = np.array([1.0, 1.0, 1.0, np.sqrt(2.0), np.sqrt(2.0), np.sqrt(2.0)])
PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]  # Voigt order 11 22 33 23 13 12


@pytest.fixture(scope="module")
def ctx():
    from paper_2208_02320_amd import hh
    c = hh.Context(0)
    yield c
    c.close()


def image(shape, seed):
    return synth.rocklike(shape, [0.6, 0.25, 0.15], sigma=1.5, seed=seed, low_to_high=[2, 1, 0])


def mandel(C):
    return C * np.outer(MANDEL, MANDEL)


def voigt_map(perm):
    """Index map of the Voigt components when a [z][y][x] label array is
    transposed by `perm` (new array axis k = old array axis perm[k]): new
    physical axis p is old physical axis 2 - perm[2 - p]."""
    pi = [2 - perm[2 - p] for p in range(3)]
    return [PAIRS.index(tuple(sorted((pi[i], pi[j])))) for i, j in PAIRS]


def test_symmetric_positive_definite_and_bracketed(ctx):
    lab = image((24, 20, 16), seed=5)
    r = ctx.homogenize(lab, PH3, tol=1e-6)
    assert np.abs(r.C_raw - r.C_raw.T).max() < 1e-5 * np.abs(r.C_raw).max()
    M = mandel(r.C)
    assert np.linalg.eigvalsh(M).min() > 0.0
    CV, CR = bounds.voigt_reuss(lab, PH3)
    scale = np.abs(M).max()
    assert np.linalg.eigvalsh(mandel(CV) - M).min() > -1e-5 * scale
    assert np.linalg.eigvalsh(M - mandel(CR)).min() > -1e-5 * scale


@pytest.mark.parametrize("perm", [(2, 1, 0), (1, 2, 0), (0, 2, 1)])
def test_axis_permutation_covariance(ctx, perm):
    lab = image((16, 20, 24), seed=6)
    C = ctx.homogenize(lab, PH3, tol=1e-6).C
    Cp = ctx.homogenize(np.ascontiguousarray(np.transpose(lab, perm)), PH3, tol=1e-6).C
    m = voigt_map(perm)
    want = C[np.ix_(m, m)]
    assert g.rel_error(Cp, want) < TOL32


def test_periodic_translation_invariance(ctx):
    lab = image((20, 24, 16), seed=7)
    C = ctx.homogenize(lab, PH3, tol=1e-6).C
    Cs = ctx.homogenize(np.ascontiguousarray(np.roll(lab, (3, -5, 7), axis=(0, 1, 2))), PH3, tol=1e-6).C
    assert g.rel_error(Cs, C) < TOL32


@pytest.mark.parametrize("pad", [0, 8])
def test_hierarchy_exact_on_a_periodic_tiling(ctx, pad):
    """A 48^3 image that tiles one 16^3 block: the plain solve, the block's
    own solve and the two-level scheme agree.  With pad = n/2 each padded box
    is 2^3 copies of the block and its core average is the block's."""
    block = image((16, 16, 16), seed=8)
    tiled = np.tile(block, (3, 3, 3))
    Cb = ctx.homogenize(block, PH3, tol=1e-6).C
    Ct = ctx.homogenize(tiled, PH3, tol=1e-6).C
    C2, Cs, _ = ctx.hierarchical(tiled, PH3, 16, pad, tol=1e-6)
    assert g.rel_error(Ct, Cb) < TOL32
    assert g.rel_error(C2, Cb) < TOL32
    for c in Cs:
        assert g.rel_error(hier.from21(c), Cb) < TOL32
