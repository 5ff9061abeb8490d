"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances: FP32 fields with FP64 reductions at residual tol 1e-6 must
match the oracle (tol 1e-10) to a relative Frobenius error of 1e-5 on the
Mandel-scaled stiffness; the FP64 path at tol 1e-10 to 1e-8.
"""
import numpy as np
import pytest

from oracle import bounds, galerkin as g, hier
from paper_2208_02320_amd import synth

pytestmark = pytest.mark.gpu

QP = [synth.QUARTZ, synth.PORE]
FOUR = synth.FOUR_PHASE["phases"]
TOL32 = 1e-5
TOL64 = 1e-8


@pytest.fixture(scope="module")
def ctx():
    from paper_2208_02320_amd import hh
    c = hh.Context(0)
    yield c
    c.close()


def oracle(lab, phases, **kw):
    kw.setdefault("tol", 1e-10)
    kw.setdefault("form", "sym6")
    return g.homogenize(g.IsotropicMedium(lab, phases), **kw)


def rand_labels(shape, nphase=2, seed=0, frac=0.3):
    rng = np.random.default_rng(seed)
    if nphase == 2:
        return (rng.random(shape) < frac).astype(np.uint8)
    return rng.integers(0, nphase, size=shape).astype(np.uint8)


def test_homogeneous_medium_exact(ctx):
    lab = np.zeros((16, 16, 16), np.uint8)
    r = ctx.homogenize(lab, [(37.0, 44.0)])
    assert g.rel_error(r.C, bounds.iso_voigt_matrix(37.0, 44.0)) < 1e-6
    assert max(r.report["iters"]) <= 1


def test_two_phase_32_fp32(ctx):
    """The 32^3 two-phase benchmark image (pore 20 %, sigma 2, seed 0)."""
    lab = synth.two_phase(32, 0.2, 2.0, 0)
    r = ctx.homogenize(lab, QP, tol=1e-6)
    ref = oracle(lab, QP)
    err = g.rel_error(r.C, ref.C_sym)
    print("32^3 fp32 err %.3e iters %s oracle iters %s" % (err, r.report["iters"], ref.iters))
    assert err < TOL32
    ref6 = oracle(lab, QP, tol=1e-6)
    for a, b in zip(r.report["iters"], ref6.iters):
        assert abs(a - b) <= 3


def test_two_phase_32_fp64(ctx):
    lab = synth.two_phase(32, 0.2, 2.0, 0)
    r = ctx.homogenize(lab, QP, tol=1e-10, precision=1)
    ref = oracle(lab, QP)
    assert g.rel_error(r.C, ref.C_sym) < TOL64


@pytest.mark.parametrize("shape", [(5, 6, 8), (9, 4, 10), (15, 12, 16)])
def test_non_cubic_odd_even_fp64(ctx, shape):
    lab = rand_labels(shape, nphase=3, seed=sum(shape))
    ph = [synth.QUARTZ, synth.CLAY, synth.PORE]
    r = ctx.homogenize(lab, ph, tol=1e-11, precision=1)
    ref = oracle(lab, ph, tol=1e-12)
    assert g.rel_error(r.C, ref.C_sym) < TOL64


@pytest.mark.parametrize("n", [4, 8, 16, 20, 24, 27, 48])
def test_sizes_fp32(ctx, n):
    lab = synth.rocklike(n, [0.6, 0.25, 0.15], sigma=1.0, seed=n, low_to_high=[2, 1, 0])
    ph = [synth.QUARTZ, synth.FELDSPAR, synth.PORE]
    r = ctx.homogenize(lab, ph, tol=1e-6)
    ref = oracle(lab, ph)
    assert g.rel_error(r.C, ref.C_sym) < TOL32


# Lengths with prime factors above 5 (padded boxes of the paper's subimage
# sizes 75, 90, 150, 180, 225, 300 with 5 or 10 voxels of padding) and the
# longest FP32 axes (1024 runs 2-column y/z tiles), each on every axis in
# turn of a thin image.
LONG32 = [85, 95, 110, 115, 130, 140, 170, 190, 220, 225, 235, 245, 265, 272, 288, 300, 310, 320, 340, 512, 900, 1024]


def thin(n, axis, seed):
    shape = [6, 4, 5]
    shape[axis] = n
    return synth.rocklike(tuple(shape), [0.6, 0.25, 0.15], sigma=1.0, seed=seed, low_to_high=[2, 1, 0])


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("n", LONG32)
def test_long_and_prime_axes_fp32(ctx, n, axis):
    lab = thin(n, axis, seed=n + axis)
    ph = [synth.QUARTZ, synth.FELDSPAR, synth.PORE]
    r = ctx.homogenize(lab, ph, tol=1e-6, tune=0)
    ref = oracle(lab, ph)
    err = g.rel_error(r.C, ref.C_sym)
    print("n=%d axis %d err %.2e" % (n, axis, err))
    assert err < TOL32


def compiled_lengths(precision):
    from paper_2208_02320_amd import hh
    return [n for n in range(2, 1025) if hh.size_supported(n, precision)]


@pytest.mark.parametrize("precision", [0, 1])
def test_every_compiled_length(ctx, precision):
    """Each compiled axis length has its own register-DFT plan (factors and
    prime kernels); every one runs on a thin image with the long axis taking
    x, y and z in turn, against the oracle."""
    tol, rtol = (1e-6, TOL32) if precision == 0 else (1e-11, TOL64)
    ph = [synth.QUARTZ, synth.FELDSPAR, synth.PORE]
    worst = 0.0
    for n in compiled_lengths(precision):
        axis = n % 3
        lab = thin(n, axis, seed=3 * n + precision)
        r = ctx.homogenize(lab, ph, tol=tol, precision=precision, tune=0)
        ref = oracle(lab, ph, tol=1e-12 if precision else 1e-10)
        err = g.rel_error(r.C, ref.C_sym)
        worst = max(worst, err)
        assert err < rtol, (n, axis, err)
    print("precision %d: %d lengths, worst error %.2e" % (precision, len(compiled_lengths(precision)), worst))


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("n", [85, 95, 110])
def test_prime_axes_fp64(ctx, n, axis):
    lab = thin(n, axis, seed=2 * n + axis)
    ph = [synth.QUARTZ, synth.FELDSPAR, synth.PORE]
    r = ctx.homogenize(lab, ph, tol=1e-11, precision=1)
    ref = oracle(lab, ph, tol=1e-12)
    assert g.rel_error(r.C, ref.C_sym) < TOL64


def test_laminate_backus_fp32(ctx):
    lab = synth.laminate(16, 4, axis=0)
    r = ctx.homogenize(lab, QP, tol=1e-7)
    f = bounds.fractions(lab, 2)
    assert g.rel_error(r.C, bounds.backus(f, QP)) < TOL32


def test_region_average_fp64(ctx):
    lab = rand_labels((12, 12, 12), seed=3)
    region = (2, 3, 1, 10, 9, 11)
    r = ctx.homogenize(lab, QP, region=region, tol=1e-11, precision=1)
    ref = oracle(lab, QP, region=region, tol=1e-12)
    assert g.rel_error(r.C_raw, ref.C) < TOL64
    assert g.rel_error(r.C, ref.C_sym) < TOL64


def test_nyquist_zero_convention(ctx):
    lab = rand_labels((8, 8, 8), seed=4)
    r = ctx.homogenize(lab, QP, tol=1e-11, precision=1, nyquist=1)
    ref = oracle(lab, QP, tol=1e-12, nyquist="zero")
    assert g.rel_error(r.C, ref.C_sym) < TOL64


def test_custom_loads(ctx):
    lab = rand_labels((8, 10, 6), seed=5)
    rng = np.random.default_rng(0)
    loads = rng.standard_normal((6, 6)) + 3 * np.eye(6)
    r = ctx.homogenize(lab, QP, loads=loads, tol=1e-11, precision=1)
    ref = oracle(lab, QP, tol=1e-12)
    assert g.rel_error(r.C, ref.C_sym) < 1e-7


def test_basic_scheme(ctx):
    lab = rand_labels((8, 8, 8), seed=6)
    r = ctx.homogenize(lab, QP, tol=1e-9, precision=1, scheme=1, max_iter=5000)
    ref = oracle(lab, QP)
    assert g.rel_error(r.C, ref.C_sym) < 1e-7
    rb = oracle(lab, QP, tol=1e-9, scheme="basic")
    assert abs(max(r.report["iters"]) - max(rb.iters)) <= 2


def test_anisotropic_voxels(ctx):
    rng = np.random.default_rng(8)
    A = rng.standard_normal((6, 5, 4, 6, 6))
    Cv = np.einsum("...ij,...kj->...ik", A, A) + 5 * np.eye(6)
    C21 = np.stack([Cv[..., i, j] for i in range(6) for j in range(i, 6)], axis=-1)
    r = ctx.homogenize_aniso(C21, tol=1e-11, precision=1)
    ref = g.homogenize(g.AnisotropicMedium(Cv), tol=1e-12, form="sym6")
    assert g.rel_error(r.C, ref.C_sym) < TOL64
    r32 = ctx.homogenize_aniso(C21, tol=1e-6)
    assert g.rel_error(r32.C, ref.C_sym) < TOL32


def test_hierarchical_small_fp64(ctx):
    lab = synth.rocklike(24, [0.75, 0.25], sigma=1.5, seed=3, low_to_high=[1, 0])
    C, Cs, rep = ctx.hierarchical(lab, QP, 8, 2, tol=1e-11, precision=1)
    ref = hier.hierarchical(lab, QP, 8, 2, tol=1e-12, form="sym6")
    assert g.rel_error(C, ref.C) < TOL64
    sub = np.stack([hier.to21(c) for c in ref.C_sub.reshape(-1, 6, 6)])
    assert np.abs(Cs - sub).max() < 1e-7 * np.abs(sub).max()


def test_hierarchical_fp32(ctx):
    lab = synth.four_phase(32, seed=2)
    C, Cs, rep = ctx.hierarchical(lab, FOUR, 16, 4, tol=1e-6)
    ref = hier.hierarchical(lab, FOUR, 16, 4, tol=1e-10, form="sym6")
    assert g.rel_error(C, ref.C) < TOL32


def test_hierarchical_single_subimage(ctx):
    """n = N: one padded subimage; the intermediate image is a single voxel,
    so C* is that subimage's symmetrized stiffness."""
    lab = synth.rocklike(24, [0.7, 0.3], sigma=1.5, seed=5, low_to_high=[1, 0])
    C, Cs, rep = ctx.hierarchical(lab, QP, 24, 4, tol=1e-11, precision=1)
    ref = hier.hierarchical(lab, QP, 24, 4, tol=1e-12, form="sym6")
    assert Cs.shape == (1, 21)
    assert g.rel_error(C, ref.C) < TOL64
    assert np.array_equal(hier.to21(C), Cs[0])
    from paper_2208_02320_amd import hh
    with pytest.raises(hh.HHError):  # 1 x 1 x 2 intermediate image
        ctx.hierarchical(np.zeros((48, 24, 24), np.uint8), QP, 24, 0)


def test_hierarchical_levels_fp64(ctx):
    """Three levels: 4^3 subimages with 1 voxel of surround, then 2^3 blocks of
    the 4^3 intermediate image with 1 voxel of surround, then the 2^3 image."""
    lab = synth.four_phase(16, sigma=1.0, seed=6)
    levels = [(4, 1), (2, 1)]
    C, rep = ctx.hierarchical_levels(lab, FOUR, levels, tol=1e-11, precision=1)
    ref, _ = hier.hierarchical_levels(lab, FOUR, levels, tol=1e-12, form="sym6")
    assert g.rel_error(C, ref) < TOL64
    assert rep["items"] == 64
    C32, _ = ctx.hierarchical_levels(lab, FOUR, levels, tol=1e-6)
    assert g.rel_error(C32, ref) < TOL32


def test_hierarchical_levels_reduce_to_two_levels(ctx):
    lab = synth.four_phase(16, sigma=1.0, seed=7)
    C2, _, _ = ctx.hierarchical(lab, FOUR, 4, 1, tol=1e-6)
    C1, _ = ctx.hierarchical_levels(lab, FOUR, [(4, 1)], tol=1e-6)
    assert np.array_equal(C1, C2)
    # a single block at level two is the two-level solve
    Cb, _ = ctx.hierarchical_levels(lab, FOUR, [(4, 1), (4, 0)], tol=1e-6)
    assert g.rel_error(Cb, C2) < 1e-12


def test_hierarchical_levels_errors(ctx):
    from paper_2208_02320_amd import hh
    lab = np.zeros((16, 16, 16), np.uint8)
    with pytest.raises(hh.HHError) as e:
        ctx.hierarchical_levels(lab, FOUR, [(4, 1), (3, 0)])  # 3 does not divide 4
    assert e.value.code == -1
    with pytest.raises(hh.HHError) as e:
        ctx.hierarchical_levels(lab, FOUR, [(4, 1), (2, 1)] * 5)  # more than 8 levels
    assert e.value.code == -1


@pytest.mark.parametrize("lpw", [1, 2, 4, 5])
def test_loads_split_over_waves_give_the_same_result(ctx, lpw):
    """An image's six load cases solved a few at a time (the path taken when
    six systems do not fit in device memory) give bit-identical stiffness:
    every system's arithmetic is the same, only the launches group them
    differently.  Single image, a batch of three, and the two-level scheme."""
    lab = synth.rocklike((24, 20, 16), [0.6, 0.25, 0.15], sigma=1.5, seed=41, low_to_high=[2, 1, 0])
    ph = [synth.QUARTZ, synth.FELDSPAR, synth.PORE]
    r6 = ctx.homogenize(lab, ph, tol=1e-6, tune=0)
    r = ctx.homogenize(lab, ph, tol=1e-6, tune=0, loads_per_wave=lpw)
    assert np.array_equal(r.C_raw, r6.C_raw)
    assert r.report["iters"] == r6.report["iters"]
    imgs = [lab, lab[::-1].copy(), np.ascontiguousarray(np.roll(lab, 5, axis=2))]
    C6 = ctx.homogenize_batch(imgs, [ph] * 3, tol=1e-6, tune=0)[1]
    C = ctx.homogenize_batch(imgs, [ph] * 3, tol=1e-6, tune=0, loads_per_wave=lpw)[1]
    assert np.array_equal(C, C6)
    big = synth.rocklike(32, [0.6, 0.25, 0.15], sigma=1.5, seed=42, low_to_high=[2, 1, 0])
    H6 = ctx.hierarchical(big, ph, 16, 2, tol=1e-6, tune=0)[0]
    H = ctx.hierarchical(big, ph, 16, 2, tol=1e-6, tune=0, loads_per_wave=lpw)[0]
    assert np.array_equal(H, H6)


def test_batch_mixed_sizes(ctx):
    recipe = synth.uneven_batch(6, sizes=(8, 12, 16), seed=77)
    imgs = [synth.item_image(it) for it in recipe]
    phs = [it["phases"] for it in recipe]
    C, Craw, st, iters, rep = ctx.homogenize_batch(imgs, phs, tol=1e-6)
    assert (st == 0).all()
    for i in range(len(imgs)):
        ref = oracle(imgs[i], phs[i])
        assert g.rel_error(C[i], ref.C_sym) < TOL32, i


def test_device_tensor_inputs(ctx):
    import torch
    lab = synth.two_phase(16, 0.3, 1.5, 1)
    d = torch.from_numpy(lab).cuda()
    r1 = ctx.homogenize(d, QP, tol=1e-6)
    r2 = ctx.homogenize(lab, QP, tol=1e-6)
    assert np.array_equal(r1.C, r2.C)


@pytest.mark.parametrize("start", [0, 1, 8])
def test_device_label_check(ctx, start):
    """Labels on the device are checked against nphase there: an image whose
    first byte sits at any alignment, with one bad label among the bytes
    before its first 16-byte boundary, in the body, or in its last bytes."""
    import torch
    from paper_2208_02320_amd import hh
    lab = synth.two_phase(16, 0.3, 1.5, 1)
    base = torch.zeros(start + lab.size, dtype=torch.uint8, device="cuda")
    d = base[start:].view(16, 16, 16)
    d.copy_(torch.from_numpy(lab))
    want = ctx.homogenize(lab, QP, tol=1e-6).C
    assert np.array_equal(ctx.homogenize(d, QP, tol=1e-6).C, want)
    for pos in (0, 3, 100, 2049, lab.size - 1):
        flat = d.view(-1)
        keep = int(flat[pos])
        flat[pos] = 2 + pos % 200
        with pytest.raises(hh.HHError) as e:
            ctx.homogenize(d, QP, tol=1e-6)
        assert e.value.code == -1 and "label %d" % (2 + pos % 200) in str(e.value), pos
        flat[pos] = keep


def test_errors(ctx):
    from paper_2208_02320_amd import hh
    lab = np.full((8, 8, 8), 2, np.uint8)
    with pytest.raises(hh.HHError) as e:
        ctx.homogenize(lab, QP)
    assert e.value.code == -1
    with pytest.raises(hh.HHError) as e:
        ctx.homogenize(np.zeros((7, 8, 8), np.uint8), QP)
    assert e.value.code == -2
    with pytest.raises(hh.HHError) as e:
        ctx.hierarchical(np.zeros((24, 24, 24), np.uint8), QP, 10, 0)
    assert e.value.code == -1
    with pytest.raises(hh.HHError) as e:
        ctx.homogenize(np.zeros((8, 8, 8), np.uint8), [(1.0, -1.0)])
    assert e.value.code == -1
    with pytest.raises(hh.HHError) as e:
        ctx.homogenize(np.zeros((8, 8, 8), np.uint8), [(float("nan"), 1.0)])
    assert e.value.code == -1
    with pytest.raises(hh.HHError) as e:
        ctx.homogenize(np.zeros((8, 8, 8), np.uint8), QP[:1], loads_per_wave=7)
    assert e.value.code == -1
    loads = np.eye(6)
    loads[:, 5] = loads[:, 4]  # two equal columns: the loads are not independent
    with pytest.raises(hh.HHError) as e:
        ctx.homogenize(np.zeros((8, 8, 8), np.uint8), QP[:1], loads=loads)
    assert e.value.code == -1


def test_fp32_tolerance_floor_reports_status(ctx):
    lab = synth.two_phase(32, 0.2, 2.0, 0)
    r = ctx.homogenize(lab, QP, tol=1e-9, max_iter=400, stall_limit=40, check=False)
    assert r.report["status"] in (0, -6, -7)
    ref = oracle(lab, QP)
    assert g.rel_error(r.C, ref.C_sym) < TOL32


def test_max_iter_one(ctx):
    lab = synth.two_phase(16, 0.2, 2.0, 0)
    r = ctx.homogenize(lab, QP, tol=1e-6, max_iter=1, check=False)
    assert r.report["status"] == -6 and max(r.report["iters"]) == 1
