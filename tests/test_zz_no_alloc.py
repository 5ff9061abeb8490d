"""The allocation-free entry point hh_homogenize_noalloc, through the C ABI,
against hh_homogenize on the same inputs: two calls in a row, the second on
a smaller image, then an image beyond the static scratch (rejected before
any device work).  No device memory is allocated: the context's workspace
and torch's allocator stay as they were."""
import numpy as np
import pytest

from paper_2208_02320_amd import synth

pytestmark = pytest.mark.gpu

FOUR = synth.FOUR_PHASE["phases"]


def test_noalloc_matches_the_allocating_entry_point():
    import torch
    from paper_2208_02320_amd import hh
    big = torch.from_numpy(synth.four_phase(48, sigma=1.5, seed=41)).cuda()
    small = torch.from_numpy(synth.rocklike((24, 32, 20), synth.FOUR_PHASE["fracs"], sigma=1.5, seed=42,
                                            low_to_high=synth.FOUR_PHASE["low_to_high"])).cuda()
    with hh.Context(0) as ref_ctx:
        ref_big = ref_ctx.homogenize(big, FOUR, tol=1e-6, tune=0, graph=0)
        ref_small = ref_ctx.homogenize(small, FOUR, tol=1e-6, tune=0, graph=0)
    torch.cuda.synchronize()
    with hh.Context(0) as ctx:
        ws0 = ctx.workspace_bytes()
        alloc0 = torch.cuda.memory_allocated()
        a = ctx.homogenize_noalloc(big, FOUR, tol=1e-6, tune=0)
        b = ctx.homogenize_noalloc(small, FOUR, tol=1e-6, tune=0)
        torch.cuda.synchronize()
        assert ctx.workspace_bytes() == ws0 == 0  # nothing went through the context's allocator
        assert torch.cuda.memory_allocated() == alloc0
        for got, want in ((a, ref_big), (b, ref_small)):
            assert got.report["status"] == 0
            assert got.report["iters"] == want.report["iters"]
            # the same kernels on the same inputs: identical bits
            assert np.array_equal(got.C, want.C)
        # beyond the 128 MiB scratch: a clear error, no device work
        huge = torch.zeros((96, 96, 96), dtype=torch.uint8, device="cuda:0")
        with pytest.raises(hh.HHError) as e:
            ctx.homogenize_noalloc(huge, FOUR, tol=1e-6)
        assert e.value.code == -1 and "scratch" in str(e.value)
        # the entry point still works after the rejection
        c = ctx.homogenize_noalloc(small, FOUR, tol=1e-6, tune=0)
        assert np.array_equal(c.C, ref_small.C)
