"""CPU checks of the element-wise error bounds used by the surrogate's GPU
parity tests (tests/mlp_bounds.py): an FP32 emulation of the device's
arithmetic (BF16 storage where the device stores BF16, FP32 sums in the host
BLAS's order) stays inside the bounds element by element, and plausible
mistakes (a dropped bias, a transposed matrix, an unrounded activation on
the wrong side) leave them."""
import numpy as np
import pytest

import oracle.mlp as om
import mlp_bounds as mb


def _net(rng, d_bits, d_dense, H):
    p = {
        "W1b": rng.normal(0, 0.5, (d_bits, H)), "W1d": rng.normal(0, 0.3, (d_dense, H)),
        "b1": rng.normal(0, 0.3, H), "W2": rng.normal(0, np.sqrt(2 / H), (H, H)),
        "b2": rng.normal(0, 0.3, H), "W3": rng.normal(0, np.sqrt(2 / H), (H, H)),
        "b3": rng.normal(0, 0.3, H), "W4": rng.normal(0, np.sqrt(1 / H), (H, 2)),
        "b4": rng.normal(0, 0.3, 2),
    }
    q = {k: np.asarray(v, np.float32).astype(np.float64) for k, v in p.items()}
    for k in ("W1b", "W1d", "W2", "W3"):
        q[k] = mb.bf16(q[k])
    return q


def _rows(rng, B, d_bits):
    return [np.sort(rng.choice(d_bits, size=int(rng.integers(0, 10)), replace=False))
            for _ in range(B)]


def _emulate_forward(q, rows, dense, drop_b2=False, transpose_w3=False):
    f = lambda a: np.asarray(a, np.float32)
    zd = f(dense) @ f(q["W1d"])
    z1 = np.empty_like(zd)
    for b, r in enumerate(rows):
        acc = f(q["b1"]) + zd[b]
        for i in r:
            acc = acc + f(q["W1b"][int(i)])
        z1[b] = acc
    h1 = f(mb.bf16(np.maximum(z1, 0)))
    z2 = h1 @ f(q["W2"]) + (0 if drop_b2 else f(q["b2"]))
    h2 = f(mb.bf16(np.maximum(z2, 0)))
    W3 = f(q["W3"]).T if transpose_w3 else f(q["W3"])
    z3 = h2 @ W3 + f(q["b3"])
    h3 = f(mb.bf16(np.maximum(z3, 0)))
    y = h3 @ f(q["W4"]) + f(q["b4"])
    return y.astype(np.float64)


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(21)
    d_bits, d_dense, H, B = 150, 24, 64, 96
    q = _net(rng, d_bits, d_dense, H)
    rows = _rows(rng, B, d_bits)
    dense = mb.bf16(rng.normal(0, 1, (B, d_dense)))
    y, cache = om.forward(q, rows, dense, act_round=mb.bf16)
    fb = mb.forward_bounds(q, rows, dense, cache)
    return q, rows, dense, y, cache, fb


def test_fp32_emulation_stays_inside_the_forward_bounds(case):
    q, rows, dense, y, cache, fb = case
    ye = _emulate_forward(q, rows, dense)
    assert np.all(np.abs(ye - y) <= fb["E_y"])
    # the bound is informative: far below the outputs' own size
    assert np.median(fb["E_y"]) < 1e-3 * np.median(np.abs(y))


@pytest.mark.parametrize("mistake", ["drop_b2", "transpose_w3"])
def test_planted_forward_mistakes_leave_the_bounds(case, mistake):
    q, rows, dense, y, cache, fb = case
    ye = _emulate_forward(q, rows, dense, **{mistake: True})
    assert np.mean(np.abs(ye - y) > fb["E_y"]) > 0.5


def test_unrounded_reference_leaves_the_bounds(case):
    """The bounds are for the reference that rounds its activations where the
    device stores them; the unrounded reference differs by BF16 steps."""
    q, rows, dense, y, cache, fb = case
    y_plain, _ = om.forward(q, rows, dense)
    assert np.any(np.abs(y_plain - y) > fb["E_y"])


def test_gradient_bounds_cover_an_fp32_emulation(case):
    q, rows, dense, y, cache, fb = case
    rng = np.random.default_rng(5)
    t = y + 1.0 + 0.5 * rng.normal(0, 1, y.shape)
    gref = om.backward(q, rows, dense, cache, y, t)
    gb = mb.gradient_bounds(q, rows, dense, cache, y, t, fb, q["W1b"].shape[0])
    # FP32 emulation of the device backward: BF16 dz, FP32 sums
    f = lambda a: np.asarray(a, np.float32)
    B = y.shape[0]
    ye = _emulate_forward(q, rows, dense)
    dy = (f(ye) - f(t)) / np.float32(B)
    h3, h2, h1 = (f(cache[k]) for k in ("h3", "h2", "h1"))
    g = {"W4": h3.T @ dy, "b4": dy.sum(0)}
    dz3 = f(mb.bf16((dy @ f(q["W4"]).T) * (h3 != 0)))
    g["W3"], g["b3"] = h2.T @ dz3, dz3.sum(0)
    dz2 = f(mb.bf16((dz3 @ f(q["W3"]).T) * (h2 != 0)))
    g["W2"], g["b2"] = h1.T @ dz2, dz2.sum(0)
    dz1 = f(mb.bf16((dz2 @ f(q["W2"]).T) * (h1 != 0)))
    g["b1"] = dz1.sum(0)
    g["W1d"] = f(dense).T @ dz1
    w1b = np.zeros(q["W1b"].shape, np.float32)
    for b, r in enumerate(rows):
        for i in r:
            w1b[int(i)] += dz1[b]
    g["W1b"] = w1b
    for k in om.PARAM_NAMES:
        d = np.abs(g[k].astype(np.float64) - gref[k])
        assert np.all(d <= gb[k]), k
    # a wrong sign on dz3 leaves them
    assert np.mean(np.abs(-g["W3"] - gref["W3"]) > gb["W3"]) > 0.5


def test_adam_bounds_cover_an_fp32_step():
    rng = np.random.default_rng(8)
    shape = (40, 7)
    p = {"w": np.asarray(rng.normal(0, 1, shape), np.float32).astype(np.float64)}
    m = {"w": np.zeros(shape)}
    v = {"w": np.zeros(shape)}
    Em = {"w": np.zeros(shape)}
    Ev = {"w": np.zeros(shape)}
    wd = p["w"].astype(np.float32)
    md = np.zeros(shape, np.float32)
    vd = np.zeros(shape, np.float32)
    lr = 1e-3
    for step in (1, 2, 3):
        g = np.asarray(rng.normal(0, 1e-2, shape), np.float32)
        g[0, :3] = 0.0                       # zero gradients stay exact
        P, M, V, Ew, Em, Ev = mb.adam_bounds(p, {"w": g.astype(np.float64)}, m, v, Em, Ev,
                                             step, lr)
        b1, b2 = np.float32(0.9), np.float32(0.999)
        c1 = np.float32(1) - np.float32(b1) ** np.float32(step)
        c2 = np.float32(1) - np.float32(b2) ** np.float32(step)
        md = b1 * md + (np.float32(1) - b1) * g
        vd = b2 * vd + (np.float32(1) - b2) * g * g
        wd = wd - np.float32(lr) * (md / c1) / (np.sqrt(vd / c2) + np.float32(1e-8))
        assert np.all(np.abs(wd.astype(np.float64) - P["w"]) <= Ew["w"]), step
        assert np.all(np.abs(md.astype(np.float64) - M["w"]) <= Em["w"]), step
        assert np.all(np.abs(vd.astype(np.float64) - V["w"]) <= Ev["w"]), step
        # continue both from the FP32 weights (the device's)
        p = {"w": wd.astype(np.float64)}
        m, v = M, V
    # a step 1% too large leaves them
    g = np.asarray(rng.normal(0, 1e-2, shape), np.float64)
    P, M, V, Ew, _, _ = mb.adam_bounds(p, {"w": g}, m, v, Em, Ev, 4, lr)
    wrong = p["w"] - 1.01 * (p["w"] - P["w"])
    assert np.mean(np.abs(wrong - P["w"]) > Ew["w"]) > 0.5
