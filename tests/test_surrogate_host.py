"""Host logic of the surrogate pipeline: the cube-symmetry augmentation
(boxes and stiffness transformed together) against oracle solves, the
error measure, and the device image generator's smoothing against the
textbook periodic Gaussian filter."""
import numpy as np
import pytest

from oracle import galerkin as g
from oracle import hier
from paper_2208_02320_amd import surrogate as sur
from paper_2208_02320_amd import synth

QP = [synth.QUARTZ, synth.PORE]


def test_48_distinct_orthogonal_symmetries():
    syms = sur.cube_symmetries()
    Qs = [sur.sym_matrix(p, s) for p, s in syms]
    assert len({Q.tobytes() for Q in Qs}) == 48
    for Q in Qs:
        assert np.allclose(Q @ Q.T, np.eye(3))


@pytest.mark.parametrize("k", [0, 5, 13, 22, 37, 47])
def test_symmetry_maps_stiffness_of_mapped_image(k):
    """Homogenizing the mapped image gives the mapped stiffness."""
    lab = synth.rocklike((8, 8, 8), [0.7, 0.3], sigma=1.2, seed=4, low_to_high=[1, 0])
    p, s = sur.cube_symmetries()[k]
    C = g.homogenize(g.IsotropicMedium(lab, QP), tol=1e-11, form="sym6").C_sym
    C2 = g.homogenize(g.IsotropicMedium(sur.transform_boxes(lab, p, s), QP), tol=1e-11, form="sym6").C_sym
    want = sur.c21_transform(p, s) @ hier.to21(C)
    assert np.abs(hier.to21(C2) - want).max() < 1e-7 * np.abs(want).max()


def test_symmetry_transform_is_a_representation():
    syms = sur.cube_symmetries()
    rng = np.random.default_rng(0)
    for _ in range(10):
        a, b = rng.integers(48, size=2)
        Qa, Qb = sur.sym_matrix(*syms[a]), sur.sym_matrix(*syms[b])
        Qab = Qa @ Qb
        c = [i for i, (p, s) in enumerate(syms) if np.allclose(sur.sym_matrix(p, s), Qab)][0]
        Ta, Tb, Tc = (sur.c21_transform(*syms[i]) for i in (a, b, c))
        assert np.allclose(Ta @ Tb, Tc)


def test_box_transform_torch_matches_numpy():
    import torch
    rng = np.random.default_rng(1)
    b = rng.integers(0, 4, size=(3, 6, 6, 6)).astype(np.uint8)
    for p, s in sur.cube_symmetries()[::7]:
        a = sur.transform_boxes(b, p, s)
        t = sur.transform_boxes(torch.from_numpy(b), p, s).numpy()
        assert np.array_equal(a, t)


def test_rel_error21_is_mandel_frobenius():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((6, 6)); A = A + A.T
    B = A + 0.01 * rng.standard_normal((6, 6)); B = B + B.T - A
    e = sur.rel_error21(hier.to21(B), hier.to21(A))[0]
    assert abs(e - g.rel_error(B, A)) < 1e-12


def test_device_generator_smoothing_is_periodic_gaussian():
    import torch
    from scipy import ndimage
    gen = torch.Generator()
    gen.manual_seed(5)
    w = torch.randn((16, 20, 24), generator=gen).numpy().astype(np.float64)
    s = synth.smoothed_noise_device((16, 20, 24), 2.0, 5, device="cpu").numpy()
    assert np.abs(s - ndimage.gaussian_filter(w, 2.0, mode="wrap")).max() < 1e-6


def test_device_generator_fractions():
    lab = synth.four_phase_device(32, seed=3, device="cpu").numpy()
    f = np.bincount(lab.ravel(), minlength=4) / lab.size
    assert np.abs(f - synth.FOUR_PHASE["fracs"]).max() < 1.0 / lab.size


def test_float_reciprocal_division_is_exact():
    """The network kernels split voxel indices with q = int(a * (1/d)) plus one
    integer correction step, in float32; exact for 0 <= a < 2^23, d >= 1."""
    rng = np.random.default_rng(0)
    ds = set([1, 2, 3, 7, 8, 15, 16, 17, 31, 32, 33, 64, 100, 127, 128, 129, 4095, 4096, 4097, 32767, 32768,
              32769, 2 ** 21 - 1, 2 ** 21])
    ds |= set(int(x) for x in rng.integers(1, 2 ** 21, size=300))
    for d in sorted(ds):
        inv = np.float32(1.0) / np.float32(d)
        ks = np.unique(np.concatenate([np.arange(0, 5), (2 ** 23 - 1) // d - np.arange(0, 3),
                                       rng.integers(0, (2 ** 23 - 1) // d + 1, size=40)]))
        a = np.concatenate([ks * d - 1, ks * d, ks * d + 1, rng.integers(0, 2 ** 23, size=200)])
        a = a[(a >= 0) & (a < 2 ** 23)].astype(np.int64)
        q = (a.astype(np.float32) * inv).astype(np.int64)  # truncation, as the float-to-int conversion
        r = a - q * d
        q = q + (r >= d) - (r < 0)
        assert np.array_equal(q, a // d), d


def test_interface_densities_match_oracle():
    """The training pipeline's interface densities (torch, vectorized) of
    the core and of the whole box against the oracle's pair-by-pair count."""
    import torch
    from oracle import surrogate as sg
    rng = np.random.default_rng(3)
    boxes = rng.integers(0, 4, size=(5, 10, 10, 10)).astype(np.uint8)
    boxes[1] = 2  # constant box
    t = torch.from_numpy(boxes)
    for off, edge in ((2, 6), (0, 10)):
        got = sur.interface_densities(t, off, edge, chunk=2)
        want = [sg.interface_density(b[off:off + edge, off:off + edge, off:off + edge]) for b in boxes]
        assert np.array_equal(got, np.array(want))
