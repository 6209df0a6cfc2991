"""FP64 reference of the learned emission proposal (test infrastructure only).

Network: input (x_e, theta) normalised to [-1, 1] plus a 32-dimensional
random Fourier encoding [sin(2 pi B v), cos(2 pi B v)] with B in R^{16x2};
three hidden layers of width 64 with ReLU; 1024 outputs, a softmax over the
32x32 equal-area emission-direction cells.  One row per (transmit, element).

Loss: L = -sum_{r,c} H[r,c] log q[r,c] / sum H, where H[r,c] is the summed
magnitude of the recorded contributions of paths emitted from row r in cell
c.  It is the importance-sampling objective for the emission pdf p_t of
Eq. 4: minimising it fits q to the contribution-weighted direction density.

Precision: the network is defined with BF16 operands in every matrix product
(weights and activations rounded to nearest-even BF16) and wide
accumulation; with bf16=True this reference rounds the same operands and
accumulates in FP64.  With bf16=False it is the exact FP64 network (used to
pin the gradient formulas by finite differences).

Parameter vector layout (77,120 floats): W1[34][64], b1[64], W2[64][64],
b2[64], W3[64][64], b3[64], W4[64][1024], b4[1024]; W is (inputs, outputs).
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT, N_RFF = 34, 64, 1024, 16
SHAPES = [("W1", (N_IN, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_HID)), ("b3", (N_HID,)), ("W4", (N_HID, N_OUT)), ("b4", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round float32 values to the nearest bfloat16 (ties to even), as float64."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def features(xe_norm, th_norm, B):
    """Rows of [x, theta, sin(2 pi B v), cos(2 pi B v)] for v = (x, theta)."""
    v = np.stack([xe_norm, th_norm], 1)
    proj = 2.0 * np.pi * v @ np.asarray(B, np.float64).T          # (R, 16)
    return np.concatenate([v, np.sin(proj), np.cos(proj)], 1)


def row_inputs(n_tx, n_el, pitch, angles):
    """Normalised element position and steering angle for row r = tx * E + e:
    x_e divided by the half aperture, theta divided by the largest |theta|
    (or 1 if every angle is zero)."""
    xe = (np.arange(n_el) - 0.5 * (n_el - 1)) * pitch
    half = 0.5 * n_el * pitch
    amax = float(np.max(np.abs(angles))) if np.max(np.abs(angles)) > 0 else 1.0
    xn = np.tile(xe / half, n_tx)
    tn = np.repeat(np.asarray(angles, np.float64) / amax, n_el)
    return xn, tn


def _mm(a, b, q):
    return (bf16(a) @ bf16(b)) if q else (a @ b)


def forward(theta, X, q_bf16=True):
    p = unpack(theta)
    h1 = np.maximum(_mm(X, p["W1"], q_bf16) + p["b1"], 0.0)
    h2 = np.maximum(_mm(h1, p["W2"], q_bf16) + p["b2"], 0.0)
    h3 = np.maximum(_mm(h2, p["W3"], q_bf16) + p["b3"], 0.0)
    z = _mm(h3, p["W4"], q_bf16) + p["b4"]
    zm = z - z.max(1, keepdims=True)
    e = np.exp(zm)
    q = e / e.sum(1, keepdims=True)
    return dict(h1=h1, h2=h2, h3=h3, z=z, q=q, logq=zm - np.log(e.sum(1, keepdims=True)))


def loss_and_grad(theta, X, H, q_bf16=True):
    """Weighted cross-entropy and its gradient with respect to theta."""
    p = unpack(theta)
    f = forward(theta, X, q_bf16)
    tot = H.sum()
    loss = -(H * f["logq"]).sum() / tot
    dz = (f["q"] * H.sum(1, keepdims=True) - H) / tot
    g = {}
    g["W4"] = _mm(f["h3"].T, dz, q_bf16)
    g["b4"] = dz.sum(0)
    d3 = _mm(dz, p["W4"].T, q_bf16) * (f["h3"] > 0)
    g["W3"] = _mm(f["h2"].T, d3, q_bf16)
    g["b3"] = d3.sum(0)
    d2 = _mm(d3, p["W3"].T, q_bf16) * (f["h2"] > 0)
    g["W2"] = _mm(f["h1"].T, d2, q_bf16)
    g["b2"] = d2.sum(0)
    d1 = _mm(d2, p["W2"].T, q_bf16) * (f["h1"] > 0)
    g["W1"] = _mm(X.T, d1, q_bf16)
    g["b1"] = d1.sum(0)
    return loss, pack(g)


def adam(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; step counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def proposal_tables(q, eps):
    """Mixture q' = (1 - eps) q + eps / 1024 and its inclusive CDF."""
    qm = (1.0 - eps) * q + eps / N_OUT
    return qm, np.cumsum(qm, 1)
