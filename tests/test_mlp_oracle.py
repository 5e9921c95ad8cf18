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
