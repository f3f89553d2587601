"""Element-wise parity of the surrogate's kernels at the product's shape
(width 512, 4096 samples, the 2000-bus action vocabulary of 6971 bits plus a
24-step injection summary) against the FP64 reference, each element within a
bound derived from the device's BF16 storage and FP32 sums (tests/
mlp_bounds.py): forward outputs, every parameter's gradient, and three Adam
steps.  The gap between the device and the reference without activation
rounding is reported beside it."""
import numpy as np
import pytest

import mlp_bounds as mb
from parity_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

D_BITS, D_DENSE, H, B = 6971, 24, 512, 4096


@pytest.fixture(scope="module")
def net_case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_10128_amd import tto
    rng = np.random.default_rng(2024)
    flat = tto.he_init(D_BITS, D_DENSE, H, seed=17)
    p = tto.split_params(flat, D_BITS, D_DENSE, H)
    for name in ("b1", "b2", "b3", "b4"):
        p[name][:] = rng.normal(0, 0.3, p[name].shape)
    flat = np.concatenate([np.ravel(p[k]) for k in
                           ("W1b", "W1d", "b1", "W2", "b2", "W3", "b3", "W4", "b4")])
    flat = flat.astype(np.float32)
    net = tto.Surrogate(D_BITS, D_DENSE, width=H, max_batch=B, max_train_batch=B)
    net.set_params(flat)
    rows = [np.sort(rng.choice(D_BITS, size=int(rng.integers(0, 17)), replace=False))
            for _ in range(B)]
    off = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ids = np.concatenate(rows).astype(np.int32)
    dense = mb.bf16(rng.normal(0, 1, (B, D_DENSE)))
    dev = torch.device("cuda")
    d = dict(off=torch.as_tensor(off, device=dev), ids=torch.as_tensor(ids, device=dev),
             dense=torch.as_tensor(dense.astype(np.float32), device=dev))
    q = {k: np.asarray(v, np.float32).astype(np.float64)
         for k, v in tto.split_params(flat.astype(np.float64), D_BITS, D_DENSE, H).items()}
    for k in ("W1b", "W1d", "W2", "W3"):
        q[k] = mb.bf16(q[k])
    return tto, net, flat, rows, dense, d, q, rng


def test_forward_and_gradients_within_bounds(net_case):
    import oracle.mlp as om
    tto, net, flat, rows, dense, d, q, rng = net_case
    y = net.forward(d["off"], d["ids"], d["dense"], B).cpu().numpy().astype(np.float64)
    y_ref, cache = om.forward(q, rows, dense, act_round=mb.bf16)
    fb = mb.forward_bounds(q, rows, dense, cache)
    err = np.abs(y - y_ref)
    flips = sum(int(fb[f"flip{l}"].sum()) for l in (1, 2, 3))
    log(f"[mlp bounds] forward: max |dy| {err.max():.3e}, max |dy|/bound "
        f"{(err / fb['E_y']).max():.3f}, median bound {np.median(fb['E_y']):.3e}, "
        f"possible ReLU flips {flips} of {3 * B * H}")
    assert np.all(err <= fb["E_y"])
    y_plain, _ = om.forward(q, rows, dense)
    gap = np.abs(y - y_plain)
    log(f"[mlp bounds] forward against the reference without activation rounding: "
        f"max {gap.max():.3e}, p99 {np.quantile(gap, 0.99):.3e} "
        f"(outputs: median |y| {np.median(np.abs(y_plain)):.3e})")

    t = (y_ref + 1.0 + 0.5 * rng.normal(0, 1, y_ref.shape)).astype(np.float32)
    g, loss = net.gradients(d["off"], d["ids"], d["dense"], torch.as_tensor(t, device="cuda"), B)
    g = tto.split_params(g.cpu().numpy().astype(np.float64), D_BITS, D_DENSE, H)
    gref = om.backward(q, rows, dense, cache, y_ref, t.astype(np.float64))
    gb = mb.gradient_bounds(q, rows, dense, cache, y_ref, t.astype(np.float64), fb, D_BITS)
    for k in om.PARAM_NAMES:
        e = np.abs(g[k] - gref[k])
        r = (e / gb[k]).max() if e.size else 0.0
        log(f"[mlp bounds] grad {k}: max |dg| {e.max() if e.size else 0:.3e}, "
            f"max |dg|/bound {r:.3f}")
        assert np.all(e <= gb[k]), k
    # loss 1/(2B) sum (y - t)^2: first- and second-order terms of the output
    # bound, plus FP32 rounding of the per-sample terms and their sum
    l_ref = om.loss(y_ref, t.astype(np.float64))
    r = np.abs(y_ref - t.astype(np.float64))
    dl = float((r * fb["E_y"] + 0.5 * fb["E_y"] ** 2).sum()) / B
    assert abs(float(loss.item()) - l_ref) <= dl + mb.gamma(B + 4) * (l_ref + dl)


def test_three_adam_steps_within_bounds(net_case):
    import oracle.mlp as om
    tto, net, flat, rows, dense, d, q, rng = net_case
    net.set_params(flat)              # also clears the Adam moments and step
    t = torch.as_tensor(rng.normal(0, 1, (B, 2)).astype(np.float32), device="cuda")
    lr = 1e-3
    p = {k: np.array(v) for k, v in
         tto.split_params(flat.astype(np.float64), D_BITS, D_DENSE, H).items()}
    st = om.adam_init(p)
    m, v = st.m, st.v
    Em = {k: np.zeros_like(x) for k, x in p.items()}
    Ev = {k: np.zeros_like(x) for k, x in p.items()}
    for step in (1, 2, 3):
        g, _ = net.gradients(d["off"], d["ids"], d["dense"], t, B)
        gd = tto.split_params(g.cpu().numpy().astype(np.float64), D_BITS, D_DENSE, H)
        net.train_step(d["off"], d["ids"], d["dense"], t, B, lr)
        P, m, v, Ew, Em, Ev = mb.adam_bounds(p, gd, m, v, Em, Ev, step, lr)
        got = tto.split_params(net.get_params().cpu().numpy().astype(np.float64), D_BITS,
                               D_DENSE, H)
        worst = 0.0
        for k in om.PARAM_NAMES:
            e = np.abs(got[k] - P[k])
            if e.size:
                worst = max(worst, float((e / Ew[k]).max()))
            assert np.all(e <= Ew[k]), (step, k)
        log(f"[mlp bounds] Adam step {step}: max |dw|/bound {worst:.3f}")
        p = got    # continue from the device's FP32 weights
