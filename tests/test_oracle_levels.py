"""Pins of the oracle's repeated coarse-graining (more than two levels).

The recursion is checked against what it must reduce to: a single block at
the second level is the two-level scheme, a periodic shift by whole blocks
of every level leaves C* unchanged, and a periodic tiling of one cell gives
the cell's own stiffness at every level."""
import numpy as np

from oracle import galerkin as g
from oracle import hier
from paper_2208_02320_amd import synth

FOUR = synth.FOUR_PHASE["phases"]
KW = dict(tol=1e-9, form="sym6")


def test_one_block_at_level_two_is_the_two_level_scheme():
    lab = synth.four_phase(8, sigma=1.0, seed=3)
    C, images = hier.hierarchical_levels(lab, FOUR, [(2, 1), (4, 0)], **KW)
    assert [im.shape[:3] for im in images] == [(4, 4, 4), (1, 1, 1)]
    ref = hier.hierarchical(lab, FOUR, 2, 1, **KW)
    assert g.rel_error(C, ref.C) < 1e-12


def test_shift_by_whole_blocks_of_every_level():
    lab = synth.four_phase(8, sigma=1.0, seed=4)
    C, _ = hier.hierarchical_levels(lab, FOUR, [(2, 1), (2, 1)], **KW)
    shifted = np.roll(np.roll(lab, 4, axis=0), -4, axis=2)
    Cs, _ = hier.hierarchical_levels(shifted, FOUR, [(2, 1), (2, 1)], **KW)
    assert g.rel_error(Cs, C) < 1e-10


def test_tiled_cell_gives_the_cell_stiffness():
    rng = np.random.default_rng(5)
    cell = rng.integers(0, 4, size=(2, 2, 2)).astype(np.uint8)
    lab = np.tile(cell, (4, 4, 4))
    C, images = hier.hierarchical_levels(lab, FOUR, [(2, 0), (2, 1)], **KW)
    ref = g.homogenize(g.IsotropicMedium(cell, FOUR), **KW)
    assert g.rel_error(C, ref.C_sym) < 1e-9
    # every intermediate image is uniform
    for im in images:
        assert np.abs(im - im.reshape(-1, 6, 6)[0]).max() < 1e-9 * np.abs(im).max()
