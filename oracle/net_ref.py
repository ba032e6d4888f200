"""FP64 reference of the learned warm-start network (a method extension; not in the paper).

TEST INFRASTRUCTURE (same rules as the rest of ``oracle/``). Plain numpy: 3x3 cross-correlation
with zero padding, bias-free, LeakyReLU(0.1) after layers 1-5, input normalised by its RMS;
backward by the chain rule written out layer by layer; the masked scale-invariant loss.
Weights: one flat float array, per layer [c_out][c_in][3][3] (tap = 3 * row offset + column
offset), layers 3->32, 32->32 (x4), 32->3. Activations (C, n_v, n_u).

Parity unpinned beyond its own pins (torch conv2d in FP64 and finite differences): the paper
has no learned component to compare against.
"""
from __future__ import annotations

import numpy as np

CIN = [3, 32, 32, 32, 32, 32]
COUT = [32, 32, 32, 32, 32, 3]
SLOPE = 0.1
N_PARAMS = sum(ci * co * 9 for ci, co in zip(CIN, COUT))


def split(weights):
    w = np.asarray(weights, dtype=np.float64)
    out, o = [], 0
    for ci, co in zip(CIN, COUT):
        out.append(w[o:o + ci * co * 9].reshape(co, ci, 3, 3))
        o += ci * co * 9
    return out


def conv3x3(a, W):
    """out[o, y, x] = sum_i sum_{ky,kx} W[o, i, ky, kx] a[i, y + ky - 1, x + kx - 1] (zero outside)."""
    C, H, Wd = a.shape
    pad = np.zeros((C, H + 2, Wd + 2))
    pad[:, 1:-1, 1:-1] = a
    out = np.zeros((W.shape[0], H, Wd))
    for ky in range(3):
        for kx in range(3):
            patch = pad[:, ky:ky + H, kx:kx + Wd]                    # (C, H, W)
            out += np.tensordot(W[:, :, ky, kx], patch, axes=([1], [0]))
    return out


def leaky(z):
    return np.where(z > 0, z, SLOPE * z)


def forward(weights, x):
    """x: (3, n_v, n_u). Returns (output, list of the 5 hidden activations, input scale)."""
    Ws = split(weights)
    x = np.asarray(x, dtype=np.float64)
    rms = np.sqrt(np.mean(x * x))
    s = 1.0 / rms if rms > 0 else 0.0
    a = x * s
    acts = []
    for l in range(6):
        z = conv3x3(a, Ws[l])
        if l < 5:
            a = leaky(z)
            acts.append(a)
        else:
            return z, acts, s


def backward(weights, x, dout):
    """dLoss/dweights (flat) for dLoss/dout given; chain rule layer by layer."""
    Ws = split(weights)
    out, acts, s = forward(weights, x)
    xin = np.asarray(x, dtype=np.float64) * s
    inputs = [xin] + acts                                   # input of layer l
    grads = [None] * 6
    dz = np.asarray(dout, dtype=np.float64)
    for l in range(5, -1, -1):
        X = inputs[l]
        C, H, Wd = X.shape
        pad = np.zeros((C, H + 2, Wd + 2))
        pad[:, 1:-1, 1:-1] = X
        g = np.zeros_like(Ws[l])
        for ky in range(3):
            for kx in range(3):
                g[:, :, ky, kx] = np.tensordot(dz, pad[:, ky:ky + H, kx:kx + Wd], axes=([1, 2], [1, 2]))
        grads[l] = g
        if l > 0:
            # d input = correlation of dz with the flipped, transposed kernel
            Wt = np.transpose(Ws[l][:, :, ::-1, ::-1], (1, 0, 2, 3))
            da = conv3x3(dz, Wt)
            dz = da * np.where(inputs[l] > 0, 1.0, SLOPE)
    return np.concatenate([g.reshape(-1) for g in grads])


def loss(x, pred, target):
    """Mean over the batch of 1 - (p.t)^2 / (|p|^2 |t|^2) on CPs where x is not all zero, and
    its gradient with respect to pred. x, pred, target: (B, 3, n)."""
    x = np.asarray(x, dtype=np.float64)
    p = np.asarray(pred, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    B = p.shape[0]
    L = 0.0
    d = np.zeros_like(p)
    for b in range(B):
        m = (np.abs(x[b]).sum(axis=0) != 0).astype(np.float64)[None, :]
        pm, tm = p[b] * m, t[b] * m
        pt, pp, tt = (pm * tm).sum(), (pm * pm).sum(), (tm * tm).sum()
        L += 1.0 - pt * pt / (pp * tt)
        d[b] = (-2.0 * pt / (pp * tt) * tm + 2.0 * pt * pt / (pp * pp * tt) * pm) * m / B
    return L / B, d
