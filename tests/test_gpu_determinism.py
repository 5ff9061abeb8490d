"""Bitwise reproducibility: every FP64 reduction of the solve follows a fixed
tree defined on the grid (line groups, row and column sums, fixed chunks),
never on the tile a workgroup holds, so every tile variant, the tuned plan
and the default plan return identical bits."""
import numpy as np
import pytest

from oracle import galerkin as g
from paper_2208_02320_amd import synth

pytestmark = pytest.mark.gpu

FOUR = synth.FOUR_PHASE["phases"]
PLANS = [(0, 0, 0), (1, 1, 1), (2, 2, 2), (3, 3, 3), (4, 4, 4), (2, 0, 1), (1, 2, 4)]


@pytest.fixture(scope="module")
def ctx():
    from paper_2208_02320_amd import hh
    c = hh.Context(0)
    yield c
    c.close()


def image(shape, seed):
    return synth.rocklike(shape, synth.FOUR_PHASE["fracs"], sigma=1.5, seed=seed,
                          low_to_high=synth.FOUR_PHASE["low_to_high"])


@pytest.mark.parametrize("shape,region", [((48, 48, 48), None), ((6, 85, 95), None),
                                          ((80, 80, 80), (8, 8, 8, 72, 72, 72)),
                                          ((30, 40, 36), (3, 5, 2, 27, 33, 30))])
def test_all_tile_plans_give_identical_bits(ctx, shape, region):
    lab = image(shape, seed=sum(shape))
    out = []
    for plan in PLANS:
        r = ctx.homogenize(lab, FOUR, region=region, tol=1e-6, plan=plan, tune=0)
        assert r.report["plan"] == list(plan)
        out.append((plan, r.C_raw, r.report["iters"]))
    plan0, C0, it0 = out[0]
    for plan, C, it in out[1:]:
        print("shape %s plan %s max |dC| %.3e" % (shape, plan, np.abs(C - C0).max()))
        assert it == it0, plan
        assert np.array_equal(C, C0), plan
    if lab.size <= 60000:  # the larger images are covered by the parity tests
        ref = g.homogenize(g.IsotropicMedium(lab, FOUR), region=region, tol=1e-10, form="sym6")
        assert g.rel_error(0.5 * (C0 + C0.T), ref.C_sym) < 1e-5


def test_tuned_and_default_plans_give_identical_bits():
    from paper_2208_02320_amd import hh
    lab = image((64, 64, 64), seed=11)
    a = hh.Context(0)
    b = hh.Context(0)
    try:
        rt = a.homogenize(lab, FOUR, tol=1e-6, tune=1)
        rd = b.homogenize(lab, FOUR, tol=1e-6, tune=0)
        print("tuned plan %s, default plan %s" % (rt.report["plan"], rd.report["plan"]))
        assert np.array_equal(rt.C_raw, rd.C_raw)
        ht = a.hierarchical(image((96, 96, 96), seed=12), FOUR, 32, 8, tol=1e-6, tune=1)
        hd = b.hierarchical(image((96, 96, 96), seed=12), FOUR, 32, 8, tol=1e-6, tune=0)
        assert np.array_equal(ht[0], hd[0]) and np.array_equal(ht[1], hd[1])
    finally:
        a.close()
        b.close()


def test_batch_plans_give_identical_bits(ctx):
    recipe = synth.uneven_batch(12, sizes=(16, 24, 32), seed=5)
    imgs = [synth.item_image(it) for it in recipe]
    phs = [it["phases"] for it in recipe]
    ref = ctx.homogenize_batch(imgs, phs, tol=1e-6, tune=0)
    for plan in ((1, 1, 1), (2, 2, 2), (1, 0, 4)):
        r = ctx.homogenize_batch(imgs, phs, tol=1e-6, tune=0, plan=plan)
        assert np.array_equal(r[0], ref[0]) and np.array_equal(r[3], ref[3]), plan


def test_concurrent_shape_groups_equal_sequential_groups(ctx):
    """hh_homogenize_batch runs its shape groups concurrently on up to four
    lanes; every item gets the bits it gets when the groups run one after
    another."""
    recipe = synth.uneven_batch(40, sizes=(16, 24, 32, 48), seed=9)
    imgs = [synth.item_image(it) for it in recipe]
    phs = [it["phases"] for it in recipe]
    seq = ctx.homogenize_batch(imgs, phs, tol=1e-6, lanes=1)
    for lanes in (0, 2, 4):
        par = ctx.homogenize_batch(imgs, phs, tol=1e-6, lanes=lanes)
        assert np.array_equal(par[0], seq[0]) and np.array_equal(par[1], seq[1]), lanes
        assert np.array_equal(par[2], seq[2]) and np.array_equal(par[3], seq[3]), lanes
        assert par[4]["voxel_iters"] == seq[4]["voxel_iters"]
