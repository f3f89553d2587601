"""GPU tests of the learned pre-screen: forward/backward and Adam against the
FP64 reference, top-k and batch gather exactness, and the screen's gain on a
2000-bus grid (all through the C ABI)."""
import numpy as np
import pytest

import gridgen as gg
from parity_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    a = (a + 0x7FFF + ((a >> 16) & 1)) & 0xFFFF0000
    return a.astype(np.uint32).view(np.float32).astype(np.float64)


def _random_bits(rng, B, d_bits, max_bits=9):
    rows = [np.sort(rng.choice(d_bits, size=int(rng.integers(0, max_bits)), replace=False))
            for _ in range(B)]
    off = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ids = np.concatenate(rows).astype(np.int32) if off[-1] else np.zeros(0, np.int32)
    return rows, off, ids


def _setup_net(d_bits, d_dense, H, B, seed, max_batch=None):
    from paper_2605_10128_amd import tto
    rng = np.random.default_rng(seed)
    flat = tto.he_init(d_bits, d_dense, H, seed=seed)
    p = tto.split_params(flat, d_bits, d_dense, H)
    # non-zero biases so that ReLU patterns are not trivially tied to the sign of W x
    for name in ("b1", "b2", "b3", "b4"):
        p[name][:] = rng.normal(0, 0.3, p[name].shape)
    flat = np.concatenate([p[k].ravel() for k in
                           ("W1b", "W1d", "b1", "W2", "b2", "W3", "b3", "W4", "b4")])
    flat = flat.astype(np.float32)
    net = tto.Surrogate(d_bits, d_dense, width=H, max_batch=max_batch or B, max_train_batch=B)
    net.set_params(flat)
    return net, flat


def _oracle_params(flat, d_bits, d_dense, H):
    """The parameters as the kernels use them: BF16 matrices for the MFMA /
    gather operands, FP32 biases and output layer; all in float64."""
    from paper_2605_10128_amd import tto
    p = tto.split_params(flat.astype(np.float64), d_bits, d_dense, H)
    q = {k: np.array(v, dtype=np.float64) for k, v in p.items()}
    for k in ("W1b", "W1d", "W2", "W3"):
        q[k] = bf16_round(p[k])
    return q


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


# BF16 unit roundoff is 2^-9.  With the activations rounded alike on both
# sides, the forward differs only by FP32 against FP64 sums of the same
# values; the backward rounds dz3, dz2, dz1 to BF16 (three roundings on the
# path to the first layer).  A relative-L2 error of at most (roundings) * 2^-9
# with a factor 2 of margin gives 1.2e-2 for both; the forward keeps the
# looser of the two bounds.
TOL_FWD = 1.2e-2
TOL_GRAD = 1.2e-2


@pytest.mark.parametrize("d_bits,d_dense,H,B", [(700, 24, 128, 100), (131, 0, 64, 37)])
def test_mlp_forward_and_gradients_match_oracle(d_bits, d_dense, H, B):
    _need_gpu()
    import oracle.mlp as om
    log(f"[mlp parity] d_bits={d_bits} d_dense={d_dense} H={H} B={B}")
    rng = np.random.default_rng(11)
    net, flat = _setup_net(d_bits, d_dense, H, B, seed=5)
    rows, off, ids = _random_bits(rng, B, d_bits)
    dense = bf16_round(rng.normal(0, 1, (B, d_dense))).astype(np.float32)
    dev = torch.device("cuda")
    off_d = torch.as_tensor(off, device=dev)
    ids_d = torch.as_tensor(ids if ids.size else np.zeros(1, np.int32), device=dev)
    dense_d = torch.as_tensor(dense if d_dense else np.zeros((B, 1), np.float32), device=dev)
    y = net.forward(off_d, ids_d, dense_d, B).cpu().numpy().astype(np.float64)

    q = _oracle_params(flat, d_bits, d_dense, H)
    # the network keeps its hidden activations in BF16: the reference applies
    # the same rounding, so both take their ReLU decisions on the same values
    y_ref, cache = om.forward(q, rows, dense.astype(np.float64).reshape(B, d_dense),
                              act_round=bf16_round)
    log(f"  forward rel err {_rel(y, y_ref):.2e}")
    assert _rel(y, y_ref) <= TOL_FWD

    # targets offset from the prediction so that dy has a consistent sign
    t = (y_ref + 1.0 + 0.5 * rng.normal(0, 1, y_ref.shape)).astype(np.float32)
    g, loss = net.gradients(off_d, ids_d, dense_d, torch.as_tensor(t, device=dev), B)
    g = g.cpu().numpy().astype(np.float64)
    gref = om.backward(q, rows, dense.astype(np.float64).reshape(B, d_dense), cache, y_ref,
                       t.astype(np.float64))
    l_ref = om.loss(y_ref, t.astype(np.float64))
    assert abs(float(loss.item()) - l_ref) <= TOL_FWD * l_ref
    from paper_2605_10128_amd import tto
    gp = tto.split_params(g, d_bits, d_dense, H)
    for k in om.PARAM_NAMES:
        if gref[k].size == 0:
            continue
        e = _rel(gp[k], gref[k])
        log(f"  grad {k}: rel err {e:.2e}")
        assert e <= TOL_GRAD, k
    # rows of W1b for bits no sample uses have exactly zero gradient
    used = np.zeros(d_bits, bool)
    used[ids] = True
    assert np.all(gp["W1b"][~used] == 0.0)


def test_adam_steps_match_oracle():
    _need_gpu()
    import oracle.mlp as om
    from paper_2605_10128_amd import tto
    d_bits, d_dense, H, B = 300, 24, 64, 64
    rng = np.random.default_rng(3)
    net, flat = _setup_net(d_bits, d_dense, H, B, seed=9)
    rows, off, ids = _random_bits(rng, B, d_bits)
    dense = bf16_round(rng.normal(0, 1, (B, d_dense))).astype(np.float32)
    dev = torch.device("cuda")
    off_d, ids_d = torch.as_tensor(off, device=dev), torch.as_tensor(ids, device=dev)
    dense_d = torch.as_tensor(dense, device=dev)
    t = torch.as_tensor(rng.normal(0, 1, (B, 2)).astype(np.float32), device=dev)
    lr = 1e-3
    p = tto.split_params(flat.astype(np.float64), d_bits, d_dense, H)
    p = {k: np.array(v) for k, v in p.items()}
    st = om.adam_init(p)
    for step in range(3):
        g, _ = net.gradients(off_d, ids_d, dense_d, t, B)
        gd = tto.split_params(g.cpu().numpy().astype(np.float64), d_bits, d_dense, H)
        net.train_step(off_d, ids_d, dense_d, t, B, lr)
        om.adam_step(p, {k: np.array(v) for k, v in gd.items()}, st, lr)
        got = tto.split_params(net.get_params().cpu().numpy().astype(np.float64), d_bits,
                               d_dense, H)
        for k in om.PARAM_NAMES:
            err = np.abs(got[k] - p[k]).max() if p[k].size else 0.0
            # FP32 rounding of the weights (|w| 2^-24, twice) and of the update: the
            # FP32 constants 1 - beta2 and 1 - beta2^t are off by ~1.3e-5 relative,
            # so the update is good to ~1e-5 relative; bound it by lr * 1e-4
            bound = 2.0 ** -23 * max(1.0, np.abs(p[k]).max() if p[k].size else 1.0) + lr * 1e-4
            assert err <= bound, (step, k, err, bound)
            p[k] = got[k].copy()    # continue both from the kernel's FP32 weights
    log("[adam] 3 steps match the FP64 update")


@pytest.mark.parametrize("n,stride,k", [(1, 1, 1), (1000, 1, 100), (4097, 2, 410),
                                        (70000, 2, 7000), (5000, 1, 5000), (3000, 1, 0)])
def test_topk_smallest_exact(n, stride, k):
    _need_gpu()
    from paper_2605_10128_amd import tto
    rng = np.random.default_rng(n + k)
    v = np.round(rng.normal(0, 3, n * stride), 0).astype(np.float32)   # many ties
    v[rng.integers(0, n * stride, 5)] = np.inf
    v[rng.integers(0, n * stride, 5)] = -np.inf
    v[v == 0] = 0.5                      # no signed zeros
    col = v[::stride][:n]
    order = np.argsort(col, kind="stable")[:k]
    if k:
        thr = col[order[-1]]
        below = np.flatnonzero(col < thr)
        ties = np.flatnonzero(col == thr)[:k - len(below)]
        expect = np.concatenate([below, ties])
        assert set(expect.tolist()) == set(order.tolist())
    else:
        expect = np.zeros(0, np.int64)
    dev = torch.device("cuda")
    vd = torch.as_tensor(v, device=dev)
    out = torch.full((max(k, 1),), -7, dtype=torch.int32, device=dev)
    tto.tto_topk_smallest(int(vd.data_ptr()), n, stride, k, int(out.data_ptr()),
                          int(torch.cuda.current_stream().cuda_stream))
    got = out.cpu().numpy()
    if k:
        assert np.array_equal(got[:k], expect)
    else:
        assert got[0] == -7


def test_batch_gather_matches_host_subset_and_evaluation():
    _need_gpu()
    from paper_2605_10128_amd import tto
    from parity_util import make_session
    w = gg.build_config(3, B=512, n_mon=200, n_cont=300, move_frac=0.3)
    log(f"[gather] B=512 moved_p={'yes' if w.batch.moved_p is not None else 'no'}")
    s = make_session(w, tto.TTO_FLOW_F64, max_batch=512)
    db = tto.device_batch(w.batch)
    full = {k: v.cpu().numpy() for k, v in s.evaluate(db).items()}
    rng = np.random.default_rng(4)
    idx = rng.integers(0, 512, 300).astype(np.int32)
    sub = w.batch.subset(idx)
    total = int(sub.moved_off[-1])
    dev = s.device
    for cap in (total, total // 2):
        k = len(idx)
        g_open = torch.empty((k, 8), dtype=torch.int32, device=dev)
        g_split = torch.empty((k, 8), dtype=torch.int32, device=dev)
        g_moff = torch.empty(k * 8 + 1, dtype=torch.int32, device=dev)
        g_mbr = torch.full((max(cap, 1),), -5, dtype=torch.int32, device=dev)
        g_mp = torch.empty((k * 8, w.P.shape[1]), dtype=torch.float64, device=dev)
        idx_d = torch.as_tensor(idx, device=dev)
        tto.tto_batch_gather(db.struct(), int(idx_d.data_ptr()), k, w.P.shape[1],
                             int(g_open.data_ptr()), int(g_split.data_ptr()),
                             int(g_moff.data_ptr()), int(g_mbr.data_ptr()), cap,
                             int(g_mp.data_ptr()) if db.moved_p is not None else 0, s.stream)
        gb = tto.DeviceBatch(k, g_open, g_split, g_moff, g_mbr,
                             g_mp if db.moved_p is not None else None)
        got = {k_: v.cpu().numpy() for k_, v in s.evaluate(gb).items()}
        moff = g_moff.cpu().numpy()
        assert np.all(np.diff(moff) >= 0) and moff[0] == 0 and moff[-1] <= cap
        assert np.array_equal(g_open.cpu().numpy(), sub.open)
        ok_rows = np.ones(k, bool)
        if cap == total:
            assert np.array_equal(g_split.cpu().numpy(), sub.split_bus)
            assert np.array_equal(moff, sub.moved_off)
            assert np.array_equal(g_mbr.cpu().numpy()[:total], sub.moved_br)
            if sub.moved_p is not None:
                assert np.array_equal(g_mp.cpu().numpy(), sub.moved_p)
        else:
            # slots past the capacity get bus -2: their candidates are INVALID
            slot_end = sub.moved_off[1:]
            over = (slot_end > cap).reshape(k, 8) & (sub.split_bus >= 0)
            ok_rows = ~over.any(axis=1)
            assert (~ok_rows).sum() > 0
            assert np.all(got["status"][~ok_rows] & 2)
            gs = g_split.cpu().numpy()
            assert np.array_equal(gs[ok_rows], sub.split_bus[ok_rows])
        for name in full:
            assert np.array_equal(got[name][ok_rows], full[name][idx][ok_rows], equal_nan=True), name
        log(f"  cap={cap}: {ok_rows.sum()} of {k} rows identical to the full evaluation")


def test_surrogate_trains_and_screens_a_generation():
    """Gain of the screen on the 2000-bus, 24-step grid: train on exact
    evaluations over 8 injection scenarios, then screen a 65536-candidate
    generation of an unseen scenario down to 10% and compare with evaluating
    all of it exactly."""
    _need_gpu()
    from paper_2605_10128_amd import tto, screen
    from parity_util import make_session
    import time
    w = gg.build_config(3, B=16384)
    grid = w.grid
    n_train_scen, per_scen, n_gen, keep = 8, 32768, 65536, 6554
    s = make_session(w, tto.TTO_FLOW_F32, max_batch=16384)
    nb = gg.bridges(grid.n_bus, grid.from_bus, grid.to_bus)
    d_bits = int((~nb).sum()) + len(w.split_table)
    scen = [gg.make_injections(grid, 24, 0x7000 + i) for i in range(n_train_scen + 1)]
    scale = screen.FeatureScale.fit([screen.injection_summary(P) for P in scen[:n_train_scen]])
    t0 = time.time()
    parts = []
    for i in range(n_train_scen):
        s.set_injections(scen[i])
        ref = screen.unswitched_reference(s)
        b = gg.make_candidates_ranked(grid, per_scen, 0x8000 + i, w.split_table, P=scen[i])
        off, ids, nbits = gg.action_bits(grid, b, len(w.split_table))
        assert nbits == d_bits
        tg, ok = [], []
        for c0 in range(0, per_scen, 16384):
            o = s.evaluate(tto.device_batch(_slice(b, c0, 16384)))
            t_, ok_ = screen.targets_from_outputs(o, ref)
            tg.append(t_)
            ok.append(ok_)
        parts.append([off, ids, scale.apply(screen.injection_summary(scen[i])),
                      np.concatenate(tg), np.concatenate(ok)])
    tscale = screen.TargetScale.fit(np.concatenate([p[3] for p in parts]),
                                    np.concatenate([p[4] for p in parts]))
    for p in parts:
        p[3] = tscale.apply(p[3])
    data = screen.Dataset.assemble(parts, seed=1)
    log(f"[surrogate] {data.n} training samples from {n_train_scen} scenarios "
        f"({time.time() - t0:.1f} s)")
    sc = screen.Screener(s, d_bits, 24, width=512, max_screen=n_gen, max_keep=8192)
    _, l0 = sc.net.gradients(data.off, data.ids, data.dense, data.target, 4096)
    loss0 = float(l0.item())
    t0 = time.time()
    losses = sc.train(data, epochs=6, batch=4096, lr=1e-3)
    torch.cuda.synchronize()
    log(f"  initial loss {loss0:.4f}, epoch losses {['%.4f' % x for x in losses]} "
        f"({time.time() - t0:.1f} s)")
    assert losses[-1] < 0.5 * loss0

    # unseen scenario, fresh generation
    P = scen[-1]
    s.set_injections(P)
    ref_h = screen.unswitched_reference(s)
    gen = gg.make_candidates_ranked(grid, n_gen, 0x9999, w.split_table, P=P)
    off, ids, _ = gg.action_bits(grid, gen, len(w.split_table))
    exact = {}
    for c0 in range(0, n_gen, 16384):
        o = s.evaluate(tto.device_batch(_slice(gen, c0, 16384)))
        for k_, v in o.items():
            exact.setdefault(k_, []).append(v.cpu().numpy())
    exact = {k_: np.concatenate(v) for k_, v in exact.items()}
    dev = s.device
    db = tto.device_batch(gen)
    off_d = torch.as_tensor(off, device=dev)
    ids_d = torch.as_tensor(ids, device=dev)
    dense_d = sc.dense_rows(scale, P, n_gen)
    gb, o = sc.screen_and_evaluate(db, off_d, ids_d, dense_d, keep)
    idx = sc.idx[:keep].cpu().numpy()
    got = {k_: v.cpu().numpy() for k_, v in o.items()}
    assert len(np.unique(idx)) == keep
    # the survivors' exact results are those of the full exact pass
    same = ((got["status"] | exact["status"][idx]) & 8) == 0
    for name in ("status", "cell", "fitness", "overload_mw", "max_loading", "worst_branch"):
        assert np.array_equal(got[name][same], exact[name][idx][same], equal_nan=True), name
    # prediction error on the unseen scenario
    y = tscale.invert(sc.y[:n_gen].cpu().numpy()) + ref_h[None, :]
    valid = (exact["status"] & 3) == 0
    truth = screen.raw_targets(exact["max_loading"], exact["overload_mw"])
    mae_rho = np.abs(y[valid, 0] - truth[valid, 0]).mean()
    corr = np.corrcoef(y[valid, 1], truth[valid, 1])[0, 1]
    # gain: the screened tenth against the best tenth by exact fitness
    fit = np.where(valid, exact["fitness"], -np.inf)
    best = np.argsort(-fit, kind="stable")[:keep]
    recall = len(np.intersect1d(best, idx)) / keep
    # overload change against the unswitched grid: screened tenth, all, and
    # the tenth with the lowest exact overload (the best any screen can do)
    d_lam = exact["overload_mw"] - np.expm1(ref_h[1]) * screen.OVERLOAD_SCALE_MW
    mean_all = d_lam[valid].mean()
    mean_scr = d_lam[idx][valid[idx]].mean()
    lam_v = np.where(valid, d_lam, np.inf)
    mean_best = lam_v[np.argsort(lam_v, kind="stable")[:keep]].mean()
    efficiency = (mean_all - mean_scr) / max(mean_all - mean_best, 1e-9)
    # archives: exact-only (all 65536) against screened (6554 survivors)
    cells = s.n_cells
    def archive(cand_ids):
        a = {}
        for c in cand_ids:
            if not valid[c]:
                continue
            cell = int(exact["cell"][c])
            if cell not in a or fit[c] > fit[a[cell]] or (fit[c] == fit[a[cell]] and c < a[cell]):
                a[cell] = c
        return a
    a_all, a_scr = archive(range(n_gen)), archive(idx.tolist())
    kept = sum(1 for c, e in a_all.items() if a_scr.get(c) == e)
    # the method without the network at the same exact budget: a random tenth
    rng = np.random.default_rng(5)
    kept_rand = []
    for _ in range(8):
        a_r = archive(rng.choice(n_gen, size=keep, replace=False).tolist())
        kept_rand.append(sum(1 for c, e in a_all.items() if a_r.get(c) == e))
    log(f"  rho MAE {mae_rho:.4f}, overload corr {corr:.3f}, recall@10% {recall:.3f} "
        f"(random 0.100), overload change screened {mean_scr:.1f} vs all {mean_all:.1f} vs "
        f"best tenth {mean_best:.1f} MW (screen efficiency {efficiency:.2f}), "
        f"archive: {kept}/{len(a_all)} exact-only elites kept (random tenth: "
        f"{np.mean(kept_rand):.1f}), {len(a_scr)} cells filled "
        f"of {cells}")
    assert corr > 0.6
    assert efficiency >= 0.25
    assert kept >= 2 * np.mean(kept_rand) + 1


def _slice(b, c0, n):
    return b.subset(np.arange(c0, c0 + n))
