"""Pins of the MLP reference (CPU): back-propagation checked by finite differences."""
import numpy as np

from oracle import mlp as M


def _data(n=40, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, M.NF)).astype(np.float32) * 2 + 1
    t = rng.standard_normal(n)
    return X, t


def test_gradient_matches_finite_differences():
    """Without rounding the gradient equals central differences of the loss (FP64)."""
    X, t = _data()
    P = M.init_params(X, seed=1).astype(np.float64)
    P[2 * M.NF:] += np.random.default_rng(2).standard_normal(M.NTRAIN) * 0.05  # non-zero biases
    g, _ = M.grad(P, X, t, bf=False)
    rng = np.random.default_rng(4)
    for i in rng.choice(M.NTRAIN, 60, replace=False):
        h = 1e-6
        Pp, Pm = P.copy(), P.copy()
        Pp[2 * M.NF + i] += h
        Pm[2 * M.NF + i] -= h
        lp = ((M.forward(Pp.astype(np.float64), X, bf=False)["y"] - t) ** 2).mean()
        lm = ((M.forward(Pm.astype(np.float64), X, bf=False)["y"] - t) ** 2).mean()
        assert abs((lp - lm) / (2 * h) - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_bf16_rounding():
    """Round to nearest even on the 8-bit BF16 mantissa: known values."""
    # 7 stored mantissa bits: the spacing at 1 is 2^-7.  1 + 2^-8 and 1 + 3*2^-8 are ties (to even:
    # down to 1, up to 1 + 2^-6); 1 + 1.5*2^-8 rounds up to 1 + 2^-7.
    x = np.array([1.0, 1.0078125, 1.00390625, 1.01171875, 1.005859375, 3.0e-8, -2.5], dtype=np.float32)
    want = np.array([1.0, 1.0078125, 1.0, 1.015625, 1.0078125, None, -2.5], dtype=object)
    got = M.bf16(x)
    for g, w in zip(got, want):
        if w is not None:
            assert g == w
    assert abs(got[5] - 3.0e-8) / 3.0e-8 <= 2 ** -8


def test_rounded_model_close_to_exact():
    X, t = _data(200)
    P = M.init_params(X, seed=5)
    y1 = M.forward(P, X, bf=True)["y"]
    y0 = M.forward(P, X, bf=False)["y"]
    assert np.abs(y1 - y0).max() <= 0.05 * np.abs(y0).max()


def _hand_params():
    """A network whose output is worked out by hand: only a few weights are non-zero, and every value
    on the way (inputs, weights, activations) is exact in BF16, so both modes give the same result."""
    P = np.zeros(M.NPARAMS)
    o = 0
    mu, sd = P[o:o + M.NF], P[o + M.NF:o + 2 * M.NF]
    o += 2 * M.NF
    sd[:] = 1.0
    mu[0], sd[0] = 1.0, 2.0
    W1 = P[o:o + M.NH * M.NF].reshape(M.NH, M.NF); o += M.NH * M.NF
    b1 = P[o:o + M.NH]; o += M.NH
    W2 = P[o:o + M.NH * M.NH].reshape(M.NH, M.NH); o += M.NH * M.NH
    b2 = P[o:o + M.NH]; o += M.NH
    w3 = P[o:o + M.NH]; o += M.NH
    W1[0, 0] = 1.0; W1[1, 1] = 1.0; W1[2, 0] = 1.0; W1[2, 1] = 1.0
    b1[0], b1[1], b1[2] = 0.5, 1.0, 3.0
    W2[0, 0] = 2.0; W2[0, 2] = 1.0; W2[1, 0] = -1.0; W2[2, 1] = 5.0; W2[2, 2] = 0.5
    b2[0], b2[1] = -1.0, 0.25
    w3[0], w3[1], w3[2] = 0.5, 10.0, -2.0
    P[o] = 0.125
    return P


def test_forward_worked_by_hand():
    """Row 1, x = (5, -3, 0, ...): standardised (2, -3); layer 1 z = (2.5, -2, 2) -> h1 = (2.5, 0, 2);
    layer 2 z = (2*2.5 + 2 - 1, -2.5 + 0.25, 0 + 0.5*2) -> h2 = (6, 0, 1); y = 0.5*6 - 2*1 + 0.125 = 1.125.
    Row 2, x = (1, 2, 0, ...): standardised (0, 2); h1 = (0.5, 3, 5); h2 = (5, 0, 17.5);
    y = 2.5 - 35 + 0.125 = -32.375.  A dropped bias, a missing ReLU, a transposed weight matrix or the
    two hidden layers swapped each change these values."""
    P = _hand_params()
    X = np.zeros((2, M.NF))
    X[0, 0], X[0, 1] = 5.0, -3.0
    X[1, 0], X[1, 1] = 1.0, 2.0
    for bf in (False, True):
        for blob in (P, P.astype(np.float32)):
            f = M.forward(blob, X.astype(np.float32), bf=bf)
            assert f["y"][0] == 1.125 and f["y"][1] == -32.375, (bf, blob.dtype, f["y"])
            assert np.array_equal(f["h1"][0, :3], [2.5, 0.0, 2.0]) and np.array_equal(f["h2"][0, :3], [6.0, 0.0, 1.0])
            assert np.array_equal(f["h1"][1, :3], [0.5, 3.0, 5.0]) and np.array_equal(f["h2"][1, :3], [5.0, 0.0, 17.5])
