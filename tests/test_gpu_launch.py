"""GPU tests of the launch machinery: every compiled tile variant against
the oracle, hipGraph replay of iteration chunks against plain launches, and
the autotuner's cached plan."""
import numpy as np
import pytest

from oracle import galerkin as g
from paper_2208_02320_amd import synth

pytestmark = pytest.mark.gpu

FOUR = synth.FOUR_PHASE["phases"]
TOL32 = 1e-5


@pytest.fixture(scope="module")
def ctx():
    from paper_2208_02320_amd import hh
    c = hh.Context(0)
    yield c
    c.close()


def oracle(lab, phases):
    return g.homogenize(g.IsotropicMedium(lab, phases), tol=1e-10, form="sym6")


_cache = {}


def image_and_oracle(shape):
    if shape not in _cache:
        lab = synth.rocklike(shape, synth.FOUR_PHASE["fracs"], sigma=1.5, seed=sum(shape),
                             low_to_high=synth.FOUR_PHASE["low_to_high"])
        _cache[shape] = (lab, oracle(lab, FOUR).C_sym)
    return _cache[shape]


@pytest.mark.parametrize("shape", [(16, 16, 16), (20, 24, 30), (48, 48, 48), (64, 64, 64), (6, 85, 95)])
@pytest.mark.parametrize("plan", [(0, 0, 0), (1, 1, 1), (2, 2, 2), (1, 2, 0), (2, 0, 1), (0, 0, 3), (3, 4, 4)])
def test_every_tile_variant_matches_oracle(ctx, shape, plan):
    lab, ref = image_and_oracle(shape)
    r = ctx.homogenize(lab, FOUR, tol=1e-6, plan=plan, tune=0)
    assert r.report["plan"] == list(plan)
    err = g.rel_error(r.C, ref)
    print("shape %s plan %s err %.2e iters %s" % (shape, plan, err, r.report["iters"]))
    assert err < TOL32


@pytest.mark.parametrize("n", [300, 320])
def test_region_sums_agree_across_x_variants(ctx, n):
    """Sub-box averages through the x-pass tile variants: at these lengths
    variant 1 runs 64-thread workgroups, fewer than the 3 R x 16 line-group
    tasks of the region sums, and variants 0 and 2 hold more rows.  Four
    iterations of each; the sums follow the same fixed tree in every
    variant, so the results are identical."""
    from paper_2208_02320_amd import synth as sy
    lab = sy.four_phase_device(n, sigma=2.0, seed=7)
    region = (10, 12, 14, n - 10, n - 12, n - 14)
    out = {}
    for xv in (0, 1, 2):
        r = ctx.homogenize(lab, FOUR, region=region, tol=1e-6, plan=(0, 0, xv), tune=0, max_iter=4, check=False)
        assert r.report["plan"] == [0, 0, xv]
        out[xv] = r.C_raw
    for xv in (1, 2):
        assert np.array_equal(out[xv], out[0]), xv


def test_graph_replay_equals_plain_launches(ctx):
    """Chunks of 3 iterations captured once and replayed many times, with the
    eager convergence poll and a synchronization between replays; three
    calls in a row (the later ones reuse the cached graphs)."""
    lab = synth.four_phase(32, seed=8)
    eager = ctx.homogenize(lab, FOUR, tol=1e-6, graph=0, tune=0, chunk=3)
    for k in range(3):
        r = ctx.homogenize(lab, FOUR, tol=1e-6, graph=1, tune=0, chunk=3)
        assert np.array_equal(r.C, eager.C), k
        assert r.report["iters"] == eager.report["iters"], k
    assert min(eager.report["iters"]) > 9  # several replays per load


def test_graph_replay_in_a_batch_and_hierarchy(ctx):
    recipe = synth.uneven_batch(5, sizes=(16, 24), seed=3)
    imgs = [synth.item_image(it) for it in recipe]
    phs = [it["phases"] for it in recipe]
    a = ctx.homogenize_batch(imgs, phs, tol=1e-6, graph=0, tune=0)
    b = ctx.homogenize_batch(imgs, phs, tol=1e-6, graph=1, tune=0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[3], b[3])
    lab = synth.four_phase(48, seed=9)
    h0 = ctx.hierarchical(lab, FOUR, 16, 4, tol=1e-6, graph=0, tune=0)
    h1 = ctx.hierarchical(lab, FOUR, 16, 4, tol=1e-6, graph=1, tune=0)
    assert np.array_equal(h0[0], h1[0]) and np.array_equal(h0[1], h1[1])


def test_autotuner_plan_is_cached_and_correct(ctx):
    from paper_2208_02320_amd import hh
    c = hh.Context(0)  # a fresh context has no plans
    lab = synth.four_phase(48, seed=10)
    r1 = c.homogenize(lab, FOUR, tol=1e-6)
    r2 = c.homogenize(lab, FOUR, tol=1e-6)
    print("plan %s, setup %.1f ms then %.1f ms" % (r1.report["plan"], r1.report["setup_ms"], r2.report["setup_ms"]))
    assert r1.report["plan"] == r2.report["plan"]
    assert all(0 <= v < 5 for v in r1.report["plan"])
    assert r1.report["setup_ms"] > 0.0
    assert r2.report["setup_ms"] < r1.report["setup_ms"]
    assert np.array_equal(r1.C, r2.C)
    ref = oracle(lab, FOUR)
    assert g.rel_error(r1.C, ref.C_sym) < TOL32
    c.close()


def test_unavailable_variant_is_rejected(ctx):
    from paper_2208_02320_amd import hh
    lab = synth.four_phase(16, seed=1)
    with pytest.raises(hh.HHError):
        ctx.homogenize(lab, FOUR, precision=1, plan=(1, 0, 0))
    with pytest.raises(hh.HHError):
        ctx.homogenize(lab, FOUR, plan=(5, 0, 0))


def test_plan_cache_file_is_written_and_reused(tmp_path):
    """A context with a plan file appends the plans it tunes; a later context
    reading the file uses them without tuning, with the same result."""
    from paper_2208_02320_amd import hh
    path = tmp_path / "plans.txt"
    lab = synth.four_phase(40, seed=14)
    with hh.Context(0) as a:
        a.plan_cache(path)
        r1 = a.homogenize(lab, FOUR, tol=1e-6)
    lines = [l.split() for l in open(path)]
    assert len(lines) == 1 and lines[0][0] == "hh-plan" and lines[0][1].startswith("gfx950")
    assert [int(v) for v in lines[0][3:6]] == [40, 40, 40]
    assert [int(v) for v in lines[0][9:12]] == r1.report["plan"]
    with hh.Context(0) as b:
        b.plan_cache(path)
        r2 = b.homogenize(lab, FOUR, tol=1e-6)
    assert r2.report["plan"] == r1.report["plan"]
    assert r2.report["setup_ms"] < r1.report["setup_ms"]
    assert np.array_equal(r2.C, r1.C)
    assert len(open(path).readlines()) == 1  # nothing new was tuned
