"""FP64 reference of the CNN surrogate (forward, loss, hand-written backward).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The surrogate is not part of the paper: it is the learned stand-in for the
subimage solve of Sec. 4.  This module defines what its kernels compute:

* input: one-hot phase labels of an n^3 window, channels padded to 8;
* four convolutions, 3x3x3 taps (tz, ty, tx) in row-major order, stride 2,
  zero padding 1, bias, ReLU: 8 -> 32 -> 32 -> 64 -> 64 channels;
* global mean over the last 4-D activation (64 features), followed by the
  window's 8 phase fractions f_c (the mean of the one-hot input),
  standardized as (f_c - mu_c) s_c; linear map 72 -> 21;
* loss: mean over batch and outputs of the squared error.

Parameters use the flat layout of the library: per layer W[tap][cout][cin]
then bias[cout]; then W_fc[21][72], b_fc[21].

With ``bf16=True`` values are rounded to bfloat16 (round to nearest even)
where the kernels store or feed them in bfloat16: weights, every layer's
activation, the masked output gradients and the inputs that enter the
weight and data gradients.  Everything else is FP64.
"""
from __future__ import annotations

import numpy as np

CIN = (8, 32, 32, 64)
COUT = (32, 32, 64, 64)
CONV_FEAT, NFRAC, OUT = 64, 8, 21
FEAT = CONV_FEAT + NFRAC


def layout():
    """[(name, offset, shape)] of the flat parameter vector."""
    out, off = [], 0
    for l in range(4):
        shp = (27, COUT[l], CIN[l])
        out.append(("W%d" % (l + 1), off, shp))
        off += int(np.prod(shp))
        out.append(("b%d" % (l + 1), off, (COUT[l],)))
        off += COUT[l]
    out.append(("Wfc", off, (OUT, FEAT)))
    off += OUT * FEAT
    out.append(("bfc", off, (OUT,)))
    off += OUT
    return out, off


def unpack(flat):
    lay, n = layout()
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == n, "parameter count"
    return {name: flat[o:o + int(np.prod(s))].reshape(s) for name, o, s in lay}


def pack(params):
    lay, n = layout()
    out = np.zeros(n)
    for name, o, s in lay:
        out[o:o + int(np.prod(s))] = np.asarray(params[name]).ravel()
    return out


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def onehot(labels, nch=8):
    """labels (B, n, n, n) -> (B, n, n, n, nch)."""
    lab = np.asarray(labels)
    return (lab[..., None] == np.arange(nch)).astype(np.float64)


def conv(x, W, b):
    """3x3x3, stride 2, zero padding 1: x (B, D, D, D, Cin) -> (B, D/2, ...)."""
    B, D = x.shape[0], x.shape[1]
    Do = D // 2
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((B, Do, Do, Do, W.shape[1]))
    for t in range(27):
        tz, ty, tx = t // 9, (t // 3) % 3, t % 3
        # padded index of input 2 o + t - 1 is 2 o + t
        patch = xp[:, tz:tz + 2 * Do:2, ty:ty + 2 * Do:2, tx:tx + 2 * Do:2, :]
        out += patch @ W[t].T
    return out + b


def conv_direct(x, W, b):
    """The same convolution by its definition, one output value at a time."""
    B, D = x.shape[0], x.shape[1]
    Do = D // 2
    out = np.zeros((B, Do, Do, Do, W.shape[1]))
    for bb in range(B):
        for oz in range(Do):
            for oy in range(Do):
                for ox in range(Do):
                    acc = b.copy()
                    for t in range(27):
                        iz, iy, ix = 2 * oz + t // 9 - 1, 2 * oy + (t // 3) % 3 - 1, 2 * ox + t % 3 - 1
                        if 0 <= iz < D and 0 <= iy < D and 0 <= ix < D:
                            acc = acc + W[t] @ x[bb, iz, iy, ix]
                    out[bb, oz, oy, ox] = acc
    return out


def fraction_features(labels, fstats=None):
    """(B, 8) standardized phase fractions; fstats = (mu[8], s[8])."""
    f = onehot(labels).mean(axis=(1, 2, 3))
    if fstats is None:
        return f
    mu, sc = (np.asarray(a, dtype=np.float64) for a in fstats)
    return (f - mu) * sc


def forward(flat, labels, bf=False, fstats=None):
    """Outputs (B, 21) and the activations needed by backward()."""
    P = unpack(flat)
    r = bf16 if bf else (lambda a: a)
    x = onehot(labels)
    acts = [x]
    for l in range(4):
        z = conv(acts[-1], r(P["W%d" % (l + 1)]), P["b%d" % (l + 1)])
        acts.append(r(np.maximum(z, 0.0)))
    h = np.concatenate([acts[-1].mean(axis=(1, 2, 3)), fraction_features(labels, fstats)], axis=1)
    y = h @ P["Wfc"].T + P["bfc"]
    return y, dict(acts=acts, h=h)


def loss_and_grad(flat, labels, target, bf=False, fstats=None):
    """(loss, flat gradient) of the mean squared error."""
    P = unpack(flat)
    r = bf16 if bf else (lambda a: a)
    y, c = forward(flat, labels, bf, fstats)
    target = np.asarray(target, dtype=np.float64)
    B = y.shape[0]
    d = y - target
    loss = float((d * d).sum() / (B * OUT))
    dy = 2.0 * d / (B * OUT)
    G = {"Wfc": dy.T @ c["h"], "bfc": dy.sum(axis=0)}
    dh = dy @ P["Wfc"][:, :CONV_FEAT]  # the fraction features take no gradient
    A = c["acts"]
    V = np.prod(A[4].shape[1:4])
    dA = np.broadcast_to(dh[:, None, None, None, :] / V, A[4].shape).copy()
    for l in range(3, -1, -1):
        X, Y = A[l], A[l + 1]
        W = r(P["W%d" % (l + 1)])
        dZ = r(np.where(Y > 0.0, dA, 0.0))
        Xr = r(X)
        B_, D = X.shape[0], X.shape[1]
        Do = D // 2
        xp = np.pad(Xr, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
        dW = np.zeros_like(W)
        dxp = np.zeros_like(xp)
        dZf = dZ.reshape(-1, W.shape[1])
        for t in range(27):
            tz, ty, tx = t // 9, (t // 3) % 3, t % 3
            sl = (slice(None), slice(tz, tz + 2 * Do, 2), slice(ty, ty + 2 * Do, 2),
                  slice(tx, tx + 2 * Do, 2), slice(None))
            dW[t] = dZf.T @ xp[sl].reshape(-1, W.shape[2])
            dxp[sl] += dZ @ W[t]
        G["W%d" % (l + 1)] = dW
        G["b%d" % (l + 1)] = dZ.sum(axis=(0, 1, 2, 3))
        dA = dxp[:, 1:-1, 1:-1, 1:-1, :]
    return loss, pack(G)


def init_params(nphase, seed=0):
    """He-normal initialisation with zero weights on padded input channels."""
    rng = np.random.default_rng(seed)
    P = {}
    for l in range(4):
        cin_real = nphase if l == 0 else CIN[l]
        W = rng.normal(0.0, np.sqrt(2.0 / (27 * cin_real)), size=(27, COUT[l], CIN[l]))
        if l == 0:
            W[:, :, nphase:] = 0.0
        P["W%d" % (l + 1)] = W
        P["b%d" % (l + 1)] = rng.normal(0.0, 0.1, size=COUT[l])
    P["Wfc"] = rng.normal(0.0, np.sqrt(1.0 / FEAT), size=(OUT, FEAT))
    P["bfc"] = rng.normal(0.0, 0.1, size=OUT)
    return pack(P)
