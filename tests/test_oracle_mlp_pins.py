"""Pins for the FP64 surrogate reference: central finite differences of the
loss, the least-squares closed form of the output layer, and Adam's first
step (which moves every parameter by lr against the gradient sign)."""
import numpy as np

from oracle import mlp


def _tiny(seed=0, d_bits=11, d_dense=3, H=6, B=5):
    rng = np.random.default_rng(seed)
    p = {
        "W1b": rng.normal(0, 0.5, (d_bits, H)), "W1d": rng.normal(0, 0.5, (d_dense, H)),
        "b1": rng.normal(0, 0.1, H), "W2": rng.normal(0, 0.5, (H, H)), "b2": rng.normal(0, 0.1, H),
        "W3": rng.normal(0, 0.5, (H, H)), "b3": rng.normal(0, 0.1, H),
        "W4": rng.normal(0, 0.5, (H, 2)), "b4": rng.normal(0, 0.1, 2),
    }
    bits = [rng.choice(d_bits, size=int(rng.integers(0, 4)), replace=False) for _ in range(B)]
    bits[0] = np.array([2, 2 + 1])
    dense = rng.normal(0, 1, (B, d_dense))
    t = rng.normal(0, 1, (B, 2))
    return p, bits, dense, t


def test_gradients_match_central_differences():
    p, bits, dense, t = _tiny()
    y, cache = mlp.forward(p, bits, dense)
    g = mlp.backward(p, bits, dense, cache, y, t)
    h = 1e-6
    for name in mlp.PARAM_NAMES:
        it = np.nditer(p[name], flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            old = p[name][idx]
            p[name][idx] = old + h
            lp = mlp.loss(mlp.forward(p, bits, dense)[0], t)
            p[name][idx] = old - h
            lm = mlp.loss(mlp.forward(p, bits, dense)[0], t)
            p[name][idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx)


def test_output_layer_gradient_vanishes_at_least_squares():
    """With the hidden layers fixed, (W4, b4) minimising the loss is the
    ordinary least-squares fit of t on [h3, 1]: the output-layer gradient
    vanishes there."""
    p, bits, dense, t = _tiny(seed=3, B=40)
    _, cache = mlp.forward(p, bits, dense)
    X = np.hstack([cache["h3"], np.ones((40, 1))])
    sol, *_ = np.linalg.lstsq(X, t, rcond=None)
    p["W4"], p["b4"] = sol[:-1], sol[-1]
    y, cache = mlp.forward(p, bits, dense)
    g = mlp.backward(p, bits, dense, cache, y, t)
    assert np.abs(g["W4"]).max() < 1e-12 and np.abs(g["b4"]).max() < 1e-12


def test_adam_first_step_is_signed_lr():
    p, bits, dense, t = _tiny(seed=5)
    y, cache = mlp.forward(p, bits, dense)
    g = mlp.backward(p, bits, dense, cache, y, t)
    p0 = {k: v.copy() for k, v in p.items()}
    st = mlp.adam_init(p)
    mlp.adam_step(p, g, st, lr=1e-3, eps=1e-300)
    for k in p:
        nz = g[k] != 0
        np.testing.assert_allclose((p0[k] - p[k])[nz], 1e-3 * np.sign(g[k][nz]), rtol=1e-9)
        np.testing.assert_array_equal(p[k][~nz], p0[k][~nz])
