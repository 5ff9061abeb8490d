"""GPU parity of the CNN surrogate and its gate, through the C ABI.

Network tolerances: the oracle rounds to bfloat16 at the same points as the
kernels (weights, activations, masked output gradients), so the remaining
differences come from FP32 against FP64 accumulation, which moves a value
across a bfloat16 rounding boundary only rarely (a relative 2^-9 step).
Outputs must agree to 2e-3 of their scale, gradients to 2e-2 (relative L2
norm per parameter block; the bias gradients of the kernels sum FP32 values
before their bfloat16 rounding), and the loss to 1e-3.
"""
import numpy as np
import pytest

from oracle import cnn as ref
from oracle import galerkin as g
from oracle import hier
from oracle import surrogate as sg
from paper_2208_02320_amd import synth

pytestmark = pytest.mark.gpu

FOUR = synth.FOUR_PHASE["phases"]


@pytest.fixture(scope="module")
def ctx():
    from paper_2208_02320_amd import hh
    c = hh.Context(0)
    yield c
    c.close()


def boxes(batch, box, nphase, seed):
    """Label boxes cut from a rock-like image (so that windows hold
    realistic structure), back to back."""
    lab = synth.rocklike(max(2 * box, 32), [1.0 / nphase] * nphase, sigma=1.5, seed=seed)
    out = np.empty((batch, box, box, box), np.uint8)
    rng = np.random.default_rng(seed)
    for b in range(batch):
        z, y, x = rng.integers(0, lab.shape[0], size=3)
        out[b] = hier.padded_box(lab, (z, y, x), box, 0)
    return out


FSTATS = (np.linspace(0.05, 0.4, 8), np.linspace(3.0, 25.0, 8))


def net_with(ctx, nphase, n, params, fstats=FSTATS):
    from paper_2208_02320_amd import hh
    net = hh.Net(ctx, nphase, n)
    net.set_params(params)
    if fstats is not None:
        net.set_fraction_scaling(*fstats)
    return net


# pad 2: byte-wise label counts; pad 4 and 8: 4- and 8-byte chunks.  Inner
# layers on outputs of 16, 8, 4, 2 voxels per row: the x-shift path of every
# row width (n = 64 has the network's own sizes).  Up to four phases the first
# layer takes two labels per load where window rows start on even addresses
# (even pad), else one (odd pad: (32, 2, 4, 3)); at n = 32 and 64 it stages
# the workgroup's labels in LDS, in 8-byte units where box and offset are
# multiples of 8 ((64, 1, 4, 8), (32, 2, 4, 8)), else 2-byte ones
@pytest.mark.parametrize("n,batch,nphase,pad", [(16, 3, 3, 2), (32, 2, 4, 2), (16, 5, 8, 2), (16, 3, 4, 4),
                                                (16, 2, 5, 8), (64, 1, 4, 8), (32, 2, 4, 3), (32, 2, 4, 8),
                                                (64, 1, 4, 2)])
def test_forward_matches_oracle(ctx, n, batch, nphase, pad):
    lab = boxes(batch, n + 2 * pad, nphase, seed=n + batch)
    p = ref.init_params(nphase, seed=7).astype(np.float32)
    net = net_with(ctx, nphase, n, p)
    y = net.forward(lab, offset=pad)
    core = lab[:, pad:pad + n, pad:pad + n, pad:pad + n]
    yr, _ = ref.forward(p.astype(np.float64), core, bf=True, fstats=FSTATS)
    scale = max(1.0, np.abs(yr).max())
    err = np.abs(y - yr).max() / scale
    print("forward n=%d batch=%d err %.2e" % (n, batch, err))
    assert err < 2e-3
    net.close()


def test_forward_ignores_labels_outside_the_channels(ctx):
    """Labels 8..255 have no one-hot channel and no phase fraction."""
    n, batch, pad = 16, 2, 8
    lab = boxes(batch, n + 2 * pad, 8, seed=21)
    rng = np.random.default_rng(22)
    high = rng.random(lab.shape) < 0.3
    lab[high] = rng.integers(8, 256, size=int(high.sum()))
    p = ref.init_params(8, seed=9).astype(np.float32)
    net = net_with(ctx, 8, n, p)
    y = net.forward(lab, offset=pad)
    core = lab[:, pad:pad + n, pad:pad + n, pad:pad + n]
    yr, _ = ref.forward(p.astype(np.float64), core, bf=True, fstats=FSTATS)
    assert np.abs(y - yr).max() / max(1.0, np.abs(yr).max()) < 2e-3
    net.close()


@pytest.mark.parametrize("pad", [2, 1])
def test_four_phase_forward_ignores_labels_past_its_channels(ctx, pad):
    """A network of four phases has no one-hot channel for labels 4..255, on
    both first-layer paths (even and odd window offsets); the oracle's
    channels 4..7 carry zero weights."""
    n, batch = 16, 3
    lab = boxes(batch, n + 2 * pad, 4, seed=23 + pad)
    rng = np.random.default_rng(24)
    high = rng.random(lab.shape) < 0.3
    lab[high] = rng.integers(4, 256, size=int(high.sum()))
    p = ref.init_params(4, seed=13).astype(np.float32)
    net = net_with(ctx, 4, n, p)
    y = net.forward(lab, offset=pad)
    core = lab[:, pad:pad + n, pad:pad + n, pad:pad + n]
    yr, _ = ref.forward(p.astype(np.float64), core, bf=True, fstats=FSTATS)
    assert np.abs(y - yr).max() / max(1.0, np.abs(yr).max()) < 2e-3
    net.close()


def test_gradient_matches_oracle(ctx):
    n, batch, nphase, pad = 16, 3, 4, 1
    lab = boxes(batch, n + 2 * pad, nphase, seed=11)
    p = ref.init_params(nphase, seed=3).astype(np.float32)
    tgt = np.random.default_rng(4).standard_normal((batch, 21)).astype(np.float32)
    net = net_with(ctx, nphase, n, p)
    loss, grad = net.gradient(lab, tgt, offset=pad)
    core = lab[:, pad:pad + n, pad:pad + n, pad:pad + n]
    lr, gr = ref.loss_and_grad(p.astype(np.float64), core, tgt.astype(np.float64), bf=True, fstats=FSTATS)
    assert abs(loss - lr) <= 1e-3 * lr
    lay, _ = ref.layout()
    for name, off, shp in lay:
        sz = int(np.prod(shp))
        a, b = grad[off:off + sz].astype(np.float64), gr[off:off + sz]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print("grad %-4s rel %.2e |g| %.3e" % (name, rel, np.linalg.norm(b)))
        assert rel < 2e-2, name
    # padded input channels of the first layer see no data
    W1 = grad[:27 * 32 * 8].reshape(27, 32, 8)
    assert np.all(W1[:, :, nphase:] == 0.0)
    net.close()


def test_adam_first_step(ctx):
    """Adam's first step is lr * g / (|g| + eps) for every parameter."""
    n, batch, nphase = 16, 2, 3
    lab = boxes(batch, n, nphase, seed=21)
    p0 = ref.init_params(nphase, seed=5).astype(np.float32)
    tgt = np.random.default_rng(6).standard_normal((batch, 21)).astype(np.float32)
    net = net_with(ctx, nphase, n, p0)
    loss_g, gr = net.gradient(lab, tgt)
    lr = 1e-3
    loss_t = net.train_step(lab, tgt, lr)
    assert loss_t == loss_g  # same kernels, same order: identical
    p1 = net.get_params()
    step = (p0.astype(np.float64) - p1) / lr
    want = gr / (np.abs(gr) + 1e-8)
    mask = np.abs(gr) > 1e-5
    assert np.abs(step - want)[mask].max() < 2e-3
    assert np.all(p1.reshape(-1)[:27 * 32 * 8].reshape(27, 32, 8)[:, :, nphase:] == 0.0)
    net.close()


def test_training_reduces_loss(ctx):
    n, batch, nphase = 16, 8, 4
    lab = boxes(batch, n, nphase, seed=31)
    # targets depend on the phase fractions, plus an offset to learn
    fr = np.stack([np.bincount(b.ravel(), minlength=nphase) / b.size for b in lab])
    A = np.random.default_rng(8).standard_normal((nphase, 21))
    tgt = (1.5 + 4.0 * (fr - fr.mean(axis=0)) @ A).astype(np.float32)
    from paper_2208_02320_amd import hh
    net = hh.Net(ctx, nphase, n, seed=1)
    losses = [net.train_step(lab, tgt, 3e-3) for _ in range(80)]
    print("loss %.4f -> %.4f" % (losses[0], losses[-1]))
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.3 * losses[0]
    net.close()


def test_predict_applies_scaling(ctx):
    n, batch, nphase = 16, 3, 2
    lab = boxes(batch, n, nphase, seed=41)
    from paper_2208_02320_amd import hh
    net = hh.Net(ctx, nphase, n, seed=2)
    mean = np.linspace(1.0, 40.0, 21)
    scale = np.linspace(0.5, 3.0, 21)
    net.set_scaling(mean, scale)
    m2, s2 = net.get_scaling()
    assert np.array_equal(m2, mean) and np.array_equal(s2, scale)
    net.set_fraction_scaling(*FSTATS)
    f2, g2 = net.get_fraction_scaling()
    assert np.array_equal(f2, FSTATS[0]) and np.array_equal(g2, FSTATS[1])
    y = net.forward(lab).astype(np.float64)
    c = net.predict(lab)
    assert np.abs(c - (y * scale + mean)).max() < 1e-12 * np.abs(c).max()
    net.close()


# the copy moves 1-, 4- or 8-byte chunks, as the sizes and addresses allow
@pytest.mark.parametrize("shape,n,pad,shift", [((16, 48, 32), 16, 3, 0), ((32, 48, 64), 16, 4, 0),
                                               ((32, 48, 64), 16, 8, 0), ((16, 48, 32), 8, 0, 0),
                                               ((32, 48, 64), 16, 8, 1)])
def test_gather_subimages_matches_padded_boxes(ctx, shape, n, pad, shift):
    import torch
    lab = np.ascontiguousarray(synth.rocklike(shape, [0.5, 0.3, 0.2], sigma=1.5, seed=9))
    origins = hier.partition(lab, n)
    b = n + 2 * pad
    out = None
    if shift:  # an output address that is not 4-byte aligned
        out = torch.full((len(origins) * b ** 3 + shift,), 255, dtype=torch.uint8, device="cuda")[shift:]
    pack = ctx.gather_subimages(lab, n, pad, out=out).cpu().numpy().reshape(len(origins), b, b, b)
    for i, o in enumerate(origins):
        assert np.array_equal(pack[i], hier.padded_box(lab, o, n, pad)), i


def constant_net(ctx, nphase, n, c21):
    """A network whose every prediction is c21 (all weights zero)."""
    from paper_2208_02320_amd import hh
    net = hh.Net(ctx, nphase, n)
    net.set_params(np.zeros(net.num_params, np.float32))
    net.set_scaling(c21, np.ones(21))
    return net


def test_total_fallback_equals_plain_hierarchy(ctx):
    """A prediction outside every item's Voigt-Reuss bracket (twice the
    stiffest phase's Voigt bound) sends all items to the FFT solver; the
    result is then the plain two-level scheme's."""
    lab = synth.four_phase(48, seed=9)
    n, pad = 16, 2
    CV, _ = sg.core_bounds(lab, 0, 48, FOUR)
    net = constant_net(ctx, 4, n, hier.to21(2.0 * CV))
    C, Cs, fb, _ = ctx.hierarchical_surrogate(lab, FOUR, n, pad, net, None, spread_tol=0.05, bound_tol=0.0, tol=1e-6)
    Cp, Csp, _ = ctx.hierarchical(lab, FOUR, n, pad, tol=1e-6)
    assert fb.all()
    assert g.rel_error(C, Cp) < 1e-6
    for i in range(len(fb)):
        assert g.rel_error(hier.from21(Cs[i]), hier.from21(Csp[i])) < 1e-6, i


def test_total_fallback_from_image_windows(ctx):
    """Networks of 32^3 cores read them straight from the image; the padded
    boxes are gathered only for the FFT fallback, here of every item."""
    lab = synth.four_phase(64, seed=10)
    n, pad = 32, 8
    CV, _ = sg.core_bounds(lab, 0, 64, FOUR)
    net = constant_net(ctx, 4, n, hier.to21(2.0 * CV))
    C, Cs, fb, _ = ctx.hierarchical_surrogate(lab, FOUR, n, pad, net, None, spread_tol=0.05, bound_tol=0.0, tol=1e-6)
    Cp, Csp, _ = ctx.hierarchical(lab, FOUR, n, pad, tol=1e-6)
    assert fb.all()
    assert g.rel_error(C, Cp) < 1e-6
    for i in range(len(fb)):
        assert g.rel_error(hier.from21(Cs[i]), hier.from21(Csp[i])) < 1e-6, i


@pytest.mark.parametrize("start", [0, 1])
def test_surrogate_device_label_check(ctx, start):
    """Device labels of the two-level entry point are checked from the cores'
    label counts (the cores tile the image): a label in 4..7 is named, one of
    8 or more is reported as such, on image windows (start 0) and on gathered
    boxes (start 1)."""
    import torch
    from paper_2208_02320_amd import hh
    lab = synth.four_phase(64, seed=12)
    n, pad = 32, 8
    CV, CR = sg.core_bounds(lab, 0, 64, FOUR)
    net = constant_net(ctx, 4, n, hier.to21(0.5 * (CV + CR)))
    base = torch.zeros(start + lab.size, dtype=torch.uint8, device="cuda")
    d = base[start:].view(lab.shape)
    d.copy_(torch.from_numpy(lab))
    want = ctx.hierarchical_surrogate(lab, FOUR, n, pad, net, None, spread_tol=0.05, bound_tol=1.0, tol=1e-6)[0]
    got = ctx.hierarchical_surrogate(d, FOUR, n, pad, net, None, spread_tol=0.05, bound_tol=1.0, tol=1e-6)[0]
    assert np.array_equal(got, want)
    for (z, y, x), bad, text in (((40, 3, 50), 5, "label 5 >= nphase in subimage 5"),
                                 ((1, 60, 2), 200, "8 or more")):
        d[z, y, x] = bad
        with pytest.raises(hh.HHError) as e:
            ctx.hierarchical_surrogate(d, FOUR, n, pad, net, None, spread_tol=0.05, bound_tol=1.0, tol=1e-6)
        assert e.value.code == -1 and text in str(e.value), str(e.value)
        d[z, y, x] = int(lab[z, y, x])
    net.close()


def test_networks_read_the_image_or_the_gathered_boxes_alike(ctx):
    """The same image on the device twice: rows on even addresses (the
    networks, label and interface counts read the cores from the image) and
    one byte off (they read the gathered padded boxes).  Flags, subimage
    stiffness and C* are identical."""
    import os
    import torch
    from paper_2208_02320_amd import hh, surrogate as sur
    paths = sur.default_weights(64, 8)
    if not all(os.path.exists(p) for p in paths):
        pytest.skip("shipped weights missing")
    na, nb = hh.Net.load(ctx, paths[0]), hh.Net.load(ctx, paths[1])
    lab = synth.four_phase(128, seed=6)
    even = torch.from_numpy(lab).cuda()
    base = torch.zeros(lab.size + 1, dtype=torch.uint8, device="cuda")
    odd = base[1:].view(lab.shape)
    odd.copy_(even)
    for tol in (0.05, 0.003):  # the second sends every item to the FFT solver
        C1, Cs1, fb1, _ = ctx.hierarchical_surrogate(even, FOUR, 64, 8, na, nb, spread_tol=tol, bound_tol=0.0, tol=1e-6)
        C2, Cs2, fb2, _ = ctx.hierarchical_surrogate(odd, FOUR, 64, 8, na, nb, spread_tol=tol, bound_tol=0.0, tol=1e-6)
        assert np.array_equal(fb1, fb2) and np.array_equal(Cs1, Cs2) and np.array_equal(C1, C2), tol
    na.close()
    nb.close()


def test_gate_and_fallback_match_oracle(ctx):
    lab = synth.four_phase(64, seed=4)
    n, pad = 16, 4
    CV, CR = sg.core_bounds(lab, 0, 64, FOUR)
    # near the Voigt end of the whole image's bracket: items with less stiff
    # phase than average fall outside their own bracket (17 of 64 here)
    c = hier.to21(0.9 * CV + 0.1 * CR)
    net = constant_net(ctx, 4, n, c)
    C, Cs, fb, rep = ctx.hierarchical_surrogate(lab, FOUR, n, pad, net, None, spread_tol=0.05, bound_tol=0.0,
                                                tol=1e-6)
    origins = hier.partition(lab, n)
    want = np.zeros(len(origins), bool)
    tight = np.zeros(len(origins), bool)
    for i, o in enumerate(origins):
        box = hier.padded_box(lab, o, n, pad)
        cv, cr = sg.core_bounds(box, pad, n, FOUR)
        want[i] = sg.gate(c, None, cv, cr, 0.05, 0.0)
        tight[i] = sg.gate_margin(c, None, cv, cr, 0.0) < 1e-9
    print("fallback %d of %d (oracle %d)" % (fb.sum(), len(fb), want.sum()))
    assert 0 < want.sum() < len(want)  # the case exercises both branches
    assert np.array_equal(fb[~tight], want[~tight])
    # accepted items carry the prediction, gated items the FFT solve
    assert np.array_equal(Cs[~fb], np.broadcast_to(c, Cs[~fb].shape))
    _, Cs_fft, _ = ctx.hierarchical(lab, FOUR, n, pad, tol=1e-6)
    assert np.abs(Cs[fb] - Cs_fft[fb]).max() < 1e-5 * np.abs(Cs_fft).max()
    # level 2 on the assembled field against the oracle
    m = tuple(s // n for s in lab.shape)
    field = np.stack([hier.from21(r) for r in Cs]).reshape(m + (6, 6))
    l2 = g.homogenize(g.AnisotropicMedium(field), tol=1e-10, form="sym6")
    assert g.rel_error(C, l2.C_sym) < 1e-5
    assert rep["items"] == len(origins)
    net.close()


def test_fraction_gate_matches_oracle(ctx):
    """Input-space test: items whose core phase fractions lie more than
    z_max feature scales from the network's training mean go to the FFT
    solver, the same items as the oracle's test picks; z_max = 0 accepts
    all (the prediction sits inside every item's bracket)."""
    lab = synth.four_phase(64, seed=4)
    n, pad = 16, 4
    CV, CR = sg.core_bounds(lab, 0, 64, FOUR)
    c = hier.to21(0.5 * (CV + CR))
    net = constant_net(ctx, 4, n, c)
    mu = np.array([0.55, 0.15, 0.10, 0.20, 0, 0, 0, 0])
    sc = np.array([20.0, 60.0, 60.0, 30.0, 0, 0, 0, 0])
    net.set_fraction_scaling(mu, sc)
    origins = hier.partition(lab, n)
    z = 1.5
    want = np.array([sg.fractions_outside(hier.padded_box(lab, o, n, 0), mu, sc, z) for o in origins])
    net.set_fraction_gate(z)
    C, Cs, fb, _ = ctx.hierarchical_surrogate(lab, FOUR, n, pad, net, None, spread_tol=0.05, bound_tol=1.0, tol=1e-6)
    print("fraction gate: %d of %d items to the FFT solver (oracle %d)" % (fb.sum(), len(fb), want.sum()))
    assert 0 < want.sum() < len(want)
    assert np.array_equal(fb, want)
    assert np.array_equal(Cs[~fb], np.broadcast_to(c, Cs[~fb].shape))
    _, Cs_fft, _ = ctx.hierarchical(lab, FOUR, n, pad, tol=1e-6)
    assert np.abs(Cs[fb] - Cs_fft[fb]).max() < 1e-5 * np.abs(Cs_fft).max()
    net.set_fraction_gate(0.0)
    _, _, fb0, _ = ctx.hierarchical_surrogate(lab, FOUR, n, pad, net, None, spread_tol=0.05, bound_tol=1.0, tol=1e-6)
    assert not fb0.any()
    with pytest.raises(RuntimeError):
        net.set_fraction_gate(-1.0)
    net.close()


def test_interface_gate_matches_oracle(ctx):
    """Texture test: items whose core interface density lies more than
    z_max training standard deviations from the training mean go to the FFT
    solver, the same items as the oracle's test picks (identity fraction
    scaling: the fraction test never triggers here); a network reading the
    whole box counts the interfaces of the box."""
    n = 16
    # core windows at offset 4 (4-byte chunks), whole 32^3 boxes (8-byte
    # chunks), core windows at offset 1 (single bytes; 18^3 boxes)
    for size, pad, whole_box in ((64, 4, False), (48, 8, True), (48, 1, False)):
        lab = synth.four_phase(size, seed=4)
        CV, CR = sg.core_bounds(lab, 0, size, FOUR)
        c = hier.to21(0.5 * (CV + CR))
        origins = hier.partition(lab, n)
        edge, off = (n + 2 * pad, 0) if whole_box else (n, pad)
        net = constant_net(ctx, 4, edge, c)
        wins = [hier.padded_box(lab, o, n, pad)[off:off + edge, off:off + edge, off:off + edge] for o in origins]
        d = np.array([sg.interface_density(w) for w in wins])
        m, scale, z = float(np.median(d)), 1.0 / max(float(d.std()), 1e-6), 1.0
        want = np.array([sg.interface_outside(w, m, scale, z) for w in wins])
        tight = np.abs(np.abs(d - m) * scale - z) < 1e-9
        net.set_interface_stats(m, scale)
        assert net.get_interface_stats() == (m, scale)
        net.set_fraction_gate(z)
        C, Cs, fb, _ = ctx.hierarchical_surrogate(lab, FOUR, n, pad, net, None, spread_tol=0.05, bound_tol=1.0,
                                                  tol=1e-6)
        print("window %d: interface gate sends %d of %d (oracle %d)" % (edge, fb.sum(), len(fb), want.sum()))
        assert 0 < want.sum() < len(want)
        assert np.array_equal(fb[~tight], want[~tight])
        net.set_interface_stats(m, 0.0)  # no statistics: no texture test
        _, _, fb0, _ = ctx.hierarchical_surrogate(lab, FOUR, n, pad, net, None, spread_tol=0.05, bound_tol=1.0,
                                                  tol=1e-6)
        assert not fb0.any()
        with pytest.raises(RuntimeError):
            net.set_interface_stats(1.5, 1.0)
        net.close()


def test_spread_between_networks_sends_all_to_fft(ctx):
    lab = synth.four_phase(32, seed=6)
    n, pad = 16, 2
    CV, CR = sg.core_bounds(lab, 0, 32, FOUR)
    c = hier.to21(0.5 * (CV + CR))
    na = constant_net(ctx, 4, n, c)
    nb = constant_net(ctx, 4, n, 1.2 * c)
    C, Cs, fb, _ = ctx.hierarchical_surrogate(lab, FOUR, n, pad, na, nb, spread_tol=0.05, bound_tol=1.0, tol=1e-6)
    assert fb.all()
    C2, Cs2, _ = ctx.hierarchical(lab, FOUR, n, pad, tol=1e-6)
    assert np.abs(Cs - Cs2).max() < 1e-5 * np.abs(Cs2).max()
    assert g.rel_error(C, C2) < 1e-6
    # a loose spread tolerance accepts the mean of the two
    C3, Cs3, fb3, _ = ctx.hierarchical_surrogate(lab, FOUR, n, pad, na, nb, spread_tol=0.5, bound_tol=1.0,
                                                 tol=1e-6)
    assert not fb3.any()
    assert np.allclose(Cs3, np.broadcast_to(1.1 * c, Cs3.shape), rtol=1e-12)
    na.close()
    nb.close()


def test_network_reading_the_whole_padded_box(ctx):
    """A network whose input edge is n + 2 pad reads each whole box: with a
    constant prediction the gate and level 2 behave as for a core network."""
    lab = synth.four_phase(48, seed=12)
    n, pad = 16, 8  # boxes of 32^3
    CV, CR = sg.core_bounds(lab, 0, 48, FOUR)
    c = hier.to21(0.5 * (CV + CR))
    box_net = constant_net(ctx, 4, n + 2 * pad, c)
    core_net = constant_net(ctx, 4, n, c)
    Cb, Csb, fbb, _ = ctx.hierarchical_surrogate(lab, FOUR, n, pad, box_net, None, spread_tol=0.05, bound_tol=0.5,
                                                 tol=1e-6)
    Cc, Csc, fbc, _ = ctx.hierarchical_surrogate(lab, FOUR, n, pad, core_net, None, spread_tol=0.05, bound_tol=0.5,
                                                 tol=1e-6)
    assert np.array_equal(fbb, fbc) and np.array_equal(Csb, Csc) and np.array_equal(Cb, Cc)
    # and a trained-style forward on the box matches the oracle on the box
    from paper_2208_02320_amd import hh
    p = ref.init_params(4, seed=9).astype(np.float32)
    net = net_with(ctx, 4, 32, p)
    boxes_ = ctx.gather_subimages(lab, n, pad)[:3].contiguous()
    y = net.forward(boxes_, offset=0)
    yr, _ = ref.forward(p.astype(np.float64), boxes_.cpu().numpy(), bf=True, fstats=FSTATS)
    assert np.abs(y - yr).max() < 2e-3 * max(1.0, np.abs(yr).max())
    for x in (box_net, core_net, net):
        x.close()


def test_surrogate_single_subimage(ctx):
    lab = synth.four_phase(32, seed=13)
    n, pad = 32, 4
    CV, CR = sg.core_bounds(lab, 0, 32, FOUR)
    c = hier.to21(0.5 * (CV + CR))
    net = constant_net(ctx, 4, n, c)
    C, Cs, fb, _ = ctx.hierarchical_surrogate(lab, FOUR, n, pad, net, None, spread_tol=0.05, bound_tol=0.5, tol=1e-6)
    assert not fb.any()
    assert np.array_equal(Cs[0], c) and np.array_equal(hier.to21(C), c)
    net.close()


def test_surrogate_argument_errors(ctx):
    from paper_2208_02320_amd import hh
    lab = synth.four_phase(32, seed=6)
    net = hh.Net(ctx, 4, 16)
    with pytest.raises(hh.HHError):
        ctx.hierarchical_surrogate(lab, FOUR, 32, 0, net)  # input edge fits neither core nor box
    with pytest.raises(hh.HHError):
        net.forward(np.zeros((2, 16, 16, 16), np.uint8), offset=1)  # window outside the box
    with pytest.raises(hh.HHError):
        hh.Net(ctx, 4, 24)  # not a multiple of 16
    with pytest.raises(hh.HHError):
        net.set_params(np.zeros(5, np.float32))
    net.close()


def test_trained_network_gains_over_the_method_without_it(ctx):
    """Train on FFT-labelled subimages, then compare on held-out subimages:
    the trained network must beat the best constant stiffness and the Hill
    average of each subimage's phase fractions, and the surrogate hierarchy
    must replace most FFT work while staying close to the plain hierarchy."""
    from paper_2208_02320_amd import surrogate as sur
    n, pad = 16, 4
    data = sur.label_images(ctx, [10000, 10001, 10002, 10003], 64, n, pad, tol=1e-5, log=None)
    val = sur.label_images(ctx, [20000], 64, n, pad, tol=1e-5, log=None)
    nets = [sur.train(ctx, data, 4, epochs=60, batch=16, lr=2e-3, seed=s, log=None)[0] for s in (1, 2)]
    e_net = sur.rel_error21(sur.predict(nets[0], val), val.c21)
    e_const = sur.rel_error21(np.broadcast_to(data.c21.mean(axis=0), val.c21.shape), val.c21)
    boxes_h = val.boxes.cpu().numpy()
    hill = []
    for b in boxes_h:
        cv, cr = sg.core_bounds(b, pad, n, FOUR)
        hill.append(hier.to21(0.5 * (cv + cr)))
    e_hill = sur.rel_error21(np.array(hill), val.c21)
    print("held-out error: network %.4f, constant %.4f, Hill %.4f" % (e_net.mean(), e_const.mean(), e_hill.mean()))
    assert e_net.mean() < 0.75 * min(e_const.mean(), e_hill.mean())
    img = synth.four_phase_device(64, seed=20000, device="cuda:0")
    Cp, Csp, rp = ctx.hierarchical(img, FOUR, n, pad, tol=1e-5)
    C, Cs, fb, rs = ctx.hierarchical_surrogate(img, FOUR, n, pad, nets[0], nets[1], spread_tol=0.1,
                                               bound_tol=0.0, tol=1e-5)
    err = g.rel_error(C, Cp)
    print("surrogate hierarchy: fallback %d/%d, FFT voxel-iters %.3g vs %.3g, C* error %.2e" %
          (fb.sum(), fb.size, rs["voxel_iters"], rp["voxel_iters"], err))
    assert rs["voxel_iters"] < 0.8 * rp["voxel_iters"]
    # The level-2 image's voxels carry the accepted predictions.  When every
    # voxel stiffness lies within a factor (1 +- e) of the exact one in the
    # quadratic-form sense, so does the homogenized stiffness, so C* is off
    # by about the largest subimage error at most.  (The whole pipeline is
    # bitwise reproducible: labels, training and predictions do not depend
    # on the tile plan.)
    sub_err = sur.rel_error21(Cs, Csp)
    print("largest subimage error %.3e" % sub_err.max())
    assert err <= sub_err.max()
    for net in nets:
        net.close()


def test_two_networks_on_two_streams_match_one_at_a_time(ctx):
    """The two-level entry point runs the second network on a lane stream,
    concurrently with the first: an accepted subimage's stiffness is exactly
    the mean of the two networks' predictions made one at a time.  One
    network given twice stays on one stream and gives its own prediction."""
    import os
    from paper_2208_02320_amd import hh, surrogate as sur
    paths = sur.default_weights(64, 8)
    if not all(os.path.exists(p) for p in paths):
        pytest.skip("shipped weights missing")
    na, nb = hh.Net.load(ctx, paths[0]), hh.Net.load(ctx, paths[1])
    lab = synth.four_phase(128, seed=4)
    boxes_ = ctx.gather_subimages(lab, 64, 8)
    pa, pb = na.predict(boxes_, offset=8), nb.predict(boxes_, offset=8)
    for a, b, want in ((na, nb, 0.5 * (pa + pb)), (na, na, pa)):
        _, Cs, fb, _ = ctx.hierarchical_surrogate(lab, FOUR, 64, 8, a, b, spread_tol=0.05, bound_tol=0.0, tol=1e-6)
        assert (~fb).sum() >= 6
        assert np.array_equal(Cs[~fb], want[~fb])
    na.close()
    nb.close()


def test_network_file_loaded_by_the_library(ctx):
    """hh_net_load reads the shipped .npz (deflated zip of .npy arrays) into
    the same network the numpy reader builds, and hh_hierarchical with
    use_surrogate = 1 takes the attached networks' path."""
    import os
    from paper_2208_02320_amd import hh, surrogate as sur
    paths = sur.default_weights(64, 8)
    if not all(os.path.exists(p) for p in paths):
        pytest.skip("shipped weights missing")
    na = hh.Net.load(ctx, paths[0])
    nb = hh.Net.load(ctx, paths[1])
    with np.load(paths[0], allow_pickle=False) as z:
        assert np.array_equal(na.get_params(), z["params"])
        m, s_ = na.get_scaling()
        assert np.array_equal(m, z["mean"]) and np.array_equal(s_, z["scale"])
        fm, fs = na.get_fraction_scaling()
        assert np.array_equal(fm, z["fmu"]) and np.array_equal(fs, z["fsc"])
        assert (na.n, na.nphase) == (int(z["n"]), int(z["nphase"]))
        if "imu" in z.files:
            assert na.get_interface_stats() == (float(z["imu"]), float(z["isc"]))
    img = synth.four_phase_device(128, sigma=2.0, seed=31, device="cuda:0")
    C1, Cs1, fb1, r1 = ctx.hierarchical_surrogate(img, FOUR, 64, 8, na, nb, spread_tol=0.02, bound_tol=0.0)
    with pytest.raises(hh.HHError):
        ctx.hierarchical(img, FOUR, 64, 8, use_surrogate=True)
    ctx.set_surrogate(na, nb, spread_tol=0.02, bound_tol=0.0)
    C2, Cs2, r2 = ctx.hierarchical(img, FOUR, 64, 8, use_surrogate=True)
    ctx.set_surrogate(None)
    assert np.array_equal(C1, C2) and np.array_equal(Cs1, Cs2)
    with pytest.raises(hh.HHError):
        hh.Net.load(ctx, os.path.join(os.path.dirname(paths[0]), "missing.npz"))
    na.close()
    nb.close()
