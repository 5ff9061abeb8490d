"""Pins of the FP64 CNN reference: the convolution against its definition,
the hand-written backward against central finite differences, and the
bfloat16 rounding against exactly representable values."""
import numpy as np

from oracle import cnn


def test_conv_matches_definition():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 6, 6, 6, 8))
    W = rng.standard_normal((27, 5, 8))
    b = rng.standard_normal(5)
    assert np.abs(cnn.conv(x, W, b) - cnn.conv_direct(x, W, b)).max() < 1e-12


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    labels = rng.integers(0, 3, size=(2, 16, 16, 16))
    flat = cnn.init_params(3, seed=2)
    target = rng.standard_normal((2, 21))
    fst = (rng.random(8) * 0.5, 1.0 + rng.random(8) * 20.0)
    loss, g = cnn.loss_and_grad(flat, labels, target, fstats=fst)
    lay, n = cnn.layout()
    idx = []
    for name, off, shp in lay:
        size = int(np.prod(shp))
        cand = rng.integers(0, size, size=6) + off
        if name == "W1":  # real input channels only (padded ones never see data)
            w = flat[off:off + size].reshape(shp)
            real = np.flatnonzero(np.broadcast_to(np.arange(8) < 3, shp).ravel())
            cand = off + rng.choice(real, size=6)
        idx.extend(cand.tolist())
    h = 1e-6
    for i in idx:
        e = np.zeros(n)
        e[i] = h
        lp, _ = cnn.loss_and_grad(flat + e, labels, target, fstats=fst)
        lm, _ = cnn.loss_and_grad(flat - e, labels, target, fstats=fst)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_fraction_features_are_phase_fractions():
    rng = np.random.default_rng(3)
    labels = rng.integers(0, 9, size=(3, 8, 8, 8))  # label 8 lies outside the 8 channels
    f = cnn.fraction_features(labels)
    for b in range(3):
        cnt = np.bincount(labels[b].ravel(), minlength=9)[:8]
        assert np.array_equal(f[b], cnt / 512.0)
    mu, sc = np.full(8, 0.1), np.arange(8.0)
    assert np.allclose(cnn.fraction_features(labels, (mu, sc)), (f - 0.1) * sc)


def test_bf16_rounding():
    v = np.array([1.0, -2.5, 3.140625, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 65280.0])
    r = cnn.bf16(v)
    # representable values stay, halfway cases go to even
    assert r[0] == 1.0 and r[1] == -2.5 and r[2] == 3.140625 and r[5] == 65280.0
    assert r[3] == 1.0 and r[4] == 1.0 + 2 ** -6


def test_layout_size():
    _, n = cnn.layout()
    assert n == 27 * 32 * 8 + 32 + 27 * 32 * 32 + 32 + 27 * 64 * 32 + 64 + 27 * 64 * 64 + 64 + 21 * 72 + 21


# ---------------------------------------------------------------------------
# acceptance gate of the surrogate
# ---------------------------------------------------------------------------
def _bracket():
    from oracle import bounds
    from paper_2208_02320_amd import synth
    lab = synth.four_phase(16, seed=5)
    return bounds.voigt_reuss(lab, synth.FOUR_PHASE["phases"])


def test_gate_accepts_inside_the_bracket():
    from oracle import surrogate as sg
    from oracle.hier import to21
    CV, CR = _bracket()
    mid = to21(0.5 * (CV + CR))
    assert not sg.gate(mid, None, CV, CR, 0.05, 0.0)
    # the bracket ends pass with a small tolerance (exact ends are singular)
    assert not sg.gate(to21(CV), None, CV, CR, 0.05, 1e-9)
    assert not sg.gate(to21(CR), None, CV, CR, 0.05, 1e-9)
    assert sg.gate(to21(CV), None, CV, CR, 0.05, 0.0)


def test_gate_rejects_outside_and_indefinite():
    from oracle import surrogate as sg
    from oracle.hier import to21
    CV, CR = _bracket()
    assert sg.gate(to21(1.2 * CV), None, CV, CR, 0.05, 0.02)       # above Voigt
    assert sg.gate(to21(0.8 * CR), None, CV, CR, 0.05, 0.02)       # below Reuss
    assert sg.gate(to21(-0.5 * (CV + CR)), None, CV, CR, 0.05, 10.0)  # not positive definite
    # a shear entry pushed past Voigt is caught by one direction only
    C = 0.5 * (CV + CR)
    C[3, 3] = CV[3, 3] * 1.5
    assert sg.gate(to21(C), None, CV, CR, 0.05, 0.01)


def test_gate_spread_between_networks():
    from oracle import surrogate as sg
    from oracle.hier import to21
    CV, CR = _bracket()
    a = to21(0.5 * (CV + CR))
    assert not sg.gate(a, a * 1.01, CV, CR, 0.05, 0.0)
    assert sg.gate(a, a * 1.10, CV, CR, 0.05, 0.0)
    # the norm is taken in Mandel form, where C44 (component 15) carries a
    # factor 2: a change of 3 % of the norm there is a 6 % spread
    b = a.copy()
    b[15] += 0.06 * np.linalg.norm(sg.mandel(0.5 * (CV + CR))) / 2.0
    assert sg.gate(a, b, CV, CR, 0.05, 0.0)


def test_gate_fraction_range():
    """The input-space test on a 4^3 window with 16 voxels of label 0 and
    48 of label 1 (fractions 1/4 and 3/4), against means 0.2 and 0.8 with
    scale 10: both features are 0.5 from the mean."""
    from oracle import surrogate as sg
    w = np.ones((4, 4, 4), np.uint8)
    w[:1] = 0
    mu = np.array([0.2, 0.8, 0, 0, 0, 0, 0, 0])
    sc = np.array([10.0, 10.0, 0, 0, 0, 0, 0, 0])
    assert sg.fractions_outside(w, mu, sc, 0.4)
    assert not sg.fractions_outside(w, mu, sc, 0.6)
    assert not sg.fractions_outside(w, mu, sc, 0.0)  # test off
    # a label that never varied in training (scale 0) must keep its mean:
    # one voxel of label 2 fails at any positive limit (it replaces a voxel
    # of label 0, whose feature moves to 0.34)
    w[0, 0, 0] = 2
    assert sg.fractions_outside(w, mu, sc, 100.0)
    assert not sg.fractions_outside(w, mu, sc, 0.0)
    mu2 = mu.copy()
    mu2[2] = 1.0 / 64
    assert not sg.fractions_outside(w, mu2, sc, 0.6)


def test_interface_density_closed_forms():
    """Interface density on windows whose differing pairs can be counted by
    hand: none (constant), all (checkerboard), one plane of pairs."""
    from oracle import surrogate as sg
    assert sg.interface_density(np.zeros((4, 4, 4), np.uint8)) == 0.0
    z, y, x = np.indices((3, 3, 3))
    assert sg.interface_density(((x + y + z) % 2).astype(np.uint8)) == 1.0
    # 3^3 split at x = 1: the 9 rows each have one differing x pair, of 54 pairs
    assert sg.interface_density((x >= 1).astype(np.uint8)) == 9 / 54
    # 4^3 split at z = 2: 16 differing z pairs of 3 * 16 * 3 = 144
    z4 = np.indices((4, 4, 4))[0]
    assert sg.interface_density((z4 >= 2).astype(np.uint8)) == 16 / 144
    w = (x >= 1).astype(np.uint8)
    assert sg.interface_outside(w, 0.0, 10.0, 1.6)       # |1/6 - 0| * 10 = 1.67
    assert not sg.interface_outside(w, 0.0, 10.0, 1.7)
    assert not sg.interface_outside(w, 0.0, 0.0, 1.0)    # no statistics: no test
    assert not sg.interface_outside(w, 0.0, 10.0, 0.0)   # test off
