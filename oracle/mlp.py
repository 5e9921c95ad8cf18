"""FP64 NumPy reference of the learned-impedance MLP (13 -> 64 -> 64 -> 1, ReLU).

TEST INFRASTRUCTURE ONLY.  Forward pass and the gradient of the mean squared
error written out layer by layer.  With ``bf16=True`` the values that the GPU
kernels feed to the matrix cores are rounded to BF16 (round to nearest even)
at the same points: standardised inputs, W1, W2, the post-ReLU first hidden
layer, and the back-propagated dH2 and dH1.  Everything else is FP64.

Parameter layout (float32 blob of 5147): mu[13], sigma[13], W1[64][13],
b1[64], W2[64][64], b2[64], w3[64], b3.
"""
from __future__ import annotations

import numpy as np

NF, NH = 13, 64
NTRAIN = NH * NF + NH + NH * NH + NH + NH + 1
NPARAMS = 2 * NF + NTRAIN


def bf16(x):
    """Round float32 values to the nearest BF16 (ties to even); returns float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def unpack(P):
    """Split the blob; float32 blobs stay float32 (as the kernels hold them), float64 stays float64."""
    P = np.asarray(P)
    if P.dtype != np.float64:
        P = P.astype(np.float32)
    o = 0
    mu = P[o:o + NF]; o += NF
    sd = P[o:o + NF]; o += NF
    W1 = P[o:o + NH * NF].reshape(NH, NF); o += NH * NF
    b1 = P[o:o + NH]; o += NH
    W2 = P[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = P[o:o + NH]; o += NH
    w3 = P[o:o + NH]; o += NH
    b3 = P[o]
    return mu, sd, W1, b1, W2, b2, w3, b3


def standardise(X, mu, sd):
    """(x - mu) * (1 / sigma); in float32 for float32 parameters, as the kernel computes it."""
    if mu.dtype == np.float64:
        return (np.asarray(X, dtype=np.float64) - mu) * (1.0 / sd)
    X = np.asarray(X, dtype=np.float32)
    isd = (np.float32(1.0) / sd).astype(np.float32)
    return ((X - mu).astype(np.float32) * isd).astype(np.float32)


def forward(P, X, bf=True):
    mu, sd, W1, b1, W2, b2, w3, b3 = unpack(P)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    xh = r(standardise(X, mu, sd))
    W1r, W2r = r(W1), r(W2)
    z1 = xh @ W1r.T + b1.astype(np.float64)
    h1 = r(np.maximum(z1, 0.0).astype(np.float32)) if bf else np.maximum(z1, 0.0)
    z2 = h1 @ W2r.T + b2.astype(np.float64)
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3.astype(np.float64) + float(b3)
    return dict(xh=xh, W1r=W1r, W2r=W2r, h1=h1, h2=h2, y=y, w3=w3.astype(np.float64))


def grad(P, X, t, bf=True):
    """Gradient of (1/n) sum (y - t)^2 in the training layout, and the loss."""
    f = forward(P, X, bf)
    n = X.shape[0]
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    e = f["y"] - np.asarray(t, dtype=np.float64)
    dy = 2.0 * e / n
    gw3 = f["h2"].T @ dy
    gb3 = dy.sum()
    g2 = np.outer(dy, f["w3"]) * (f["h2"] > 0)
    gb2 = g2.sum(0)
    g2r = r(g2.astype(np.float32)) if bf else g2
    gW2 = g2r.T @ f["h1"]
    g1 = (g2r @ f["W2r"]) * (f["h1"] > 0)
    gb1 = g1.sum(0)
    g1r = r(g1.astype(np.float32)) if bf else g1
    gW1 = g1r.T @ f["xh"]
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return g, float((e * e).mean())


def init_params(X, seed=0):
    """He-initialised weights, input standardisation from the data."""
    rng = np.random.default_rng(seed)
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(0)
    sd = np.maximum(X.std(0), 1e-3)
    W1 = rng.standard_normal((NH, NF)) * np.sqrt(2.0 / NF)
    W2 = rng.standard_normal((NH, NH)) * np.sqrt(2.0 / NH)
    w3 = rng.standard_normal(NH) * np.sqrt(1.0 / NH)
    P = np.concatenate([mu, sd, W1.ravel(), np.zeros(NH), W2.ravel(), np.zeros(NH), w3, [0.0]])
    return P.astype(np.float32)
