"""The learned pre-screen inside a MapElites generation (tto_screened_generation,
Alg. 3 with the screen between variation and evaluation), through the C ABI:
keeping every child reproduces tto_generation bit for bit; keeping a tenth
keeps exactly the children with the smallest predicted overload (ties to the
lower index, computed on the host from the device's children and the network's
own predictions) and evaluates them as tto_evaluate does; graph replays equal
eager generations."""
import numpy as np
import pytest

import gridgen as gg
from parity_util import log, make_session, to_numpy
from test_gpu_evolve import spaces

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tto():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_10128_amd import tto as t
    return t


def _net(tto, dev_space, n_child, seed):
    d_bits = dev_space.desc.n_disc + dev_space.desc.n_actions
    net = tto.Surrogate(d_bits, 24, width=128, max_batch=n_child, max_train_batch=256)
    flat = tto.he_init(d_bits, 24, 128, seed=seed)
    p = tto.split_params(flat, d_bits, 24, 128)
    rng = np.random.default_rng(seed)
    for k in ("b1", "b2", "b3", "b4"):
        p[k][:] = rng.normal(0, 0.3, p[k].shape)
    net.set_params(np.concatenate([np.ravel(p[k]) for k in
                                   ("W1b", "W1d", "b1", "W2", "b2", "W3", "b3", "W4", "b4")]))
    return net


def _features(children, n_a, n_disc, n_actions):
    """Host feature rows of genomes: action a -> n_disc + a, disconnection d -> d."""
    ids = np.full(children.shape, -1, dtype=np.int32)
    a = children[:, :n_a]
    d = children[:, n_a:]
    ids[:, :n_a] = np.where((a >= 0) & (a < n_actions), n_disc + a, -1)
    ids[:, n_a:] = np.where((d >= 0) & (d < n_disc), d, -1)
    off = (np.arange(children.shape[0] + 1) * children.shape[1]).astype(np.int32)
    return off, ids.ravel()


@pytest.mark.parametrize("flow", ["f64", "f32"])
def test_keeping_every_child_equals_the_plain_generation(tto, flow):
    import torch
    w = gg.build_config(1) if flow == "f64" else gg.build_config(2, B=512)
    fp = tto.TTO_FLOW_F64 if flow == "f64" else tto.TTO_FLOW_F32
    n_child = 64 if flow == "f64" else 512
    sess = make_session(w, fp, max_batch=n_child)
    dev, _ = spaces(sess, w, 3, 3, 60, seed=3)
    net = _net(tto, dev, n_child, seed=4)
    plain = tto.Repertoire(sess, dev)
    evo = tto.Evolver(sess, dev, plain, n_child, seed=9)
    scr = tto.Repertoire(sess, dev)
    sev = tto.ScreenedEvolver(sess, dev, scr, net, n_child, n_child, seed=9,
                              dense_row=np.linspace(-1, 1, 24))
    for g in range(5):
        evo.step()
        sev.step()
        torch.cuda.synchronize()
        assert torch.equal(evo.children, sev.children), g
        for a, b in ((plain.fitness, scr.fitness), (plain.id, scr.id), (plain.genome, scr.genome)):
            assert torch.equal(a, b), g
    log(f"[screened] {flow}: keeping all {n_child} children equals 5 plain generations, "
        f"{int((scr.id >= 0).sum().item())} cells")
    sess.close()


def test_screen_keeps_the_predicted_best_tenth(tto):
    import torch
    w = gg.build_config(2, B=512)
    n_child, n_keep = 4096, 410
    sess = make_session(w, tto.TTO_FLOW_F32, max_batch=n_child)
    dev, _ = spaces(sess, w, 4, 4, 300, seed=5)
    net = _net(tto, dev, n_child, seed=6)
    rep = tto.Repertoire(sess, dev)
    row = np.random.default_rng(1).normal(0, 1, 24).astype(np.float32)
    outs = sess.alloc_outputs(n_keep)
    sev = tto.ScreenedEvolver(sess, dev, rep, net, n_child, n_keep, seed=21, dense_row=row,
                              outputs=outs)
    plain = tto.Evolver(sess, dev, rep, n_child, seed=21)
    for _ in range(3):                       # a populated repertoire first
        plain.step()
    torch.cuda.synchronize()
    before_id = rep.id.clone()
    before_fit = rep.fitness.clone()
    gen = int(rep.generation.item())
    # the children this generation will draw, from the same repertoire state
    kids, _ = dev.vary(rep, 21, n_child)
    torch.cuda.synchronize()
    sev.step()
    torch.cuda.synchronize()
    children = sev.children.cpu().numpy()
    assert np.array_equal(children, kids.cpu().numpy())
    # the network's predictions on the host-built features of those children
    off, ids = _features(children, dev.n_a, dev.desc.n_disc, dev.desc.n_actions)
    dvc = torch.device("cuda")
    dense = torch.as_tensor(np.repeat(row[None, :], n_child, axis=0), device=dvc)
    y = net.forward(torch.as_tensor(off, device=dvc), torch.as_tensor(ids, device=dvc), dense,
                    n_child).cpu().numpy()
    order = np.argsort(y[:, 1], kind="stable")[:n_keep]
    kept = np.sort(order)
    assert np.array_equal(sev.kept.cpu().numpy(), kept)
    # outputs of the kept children equal a plain evaluation of them
    db = dev.expand(torch.as_tensor(children[kept], device=dvc).contiguous())
    ref = to_numpy(sess.evaluate(db))
    got = to_numpy(outs)
    for k in ref:
        assert np.array_equal(got[k], ref[k], equal_nan=True), k
    # insertion: every changed cell holds a kept child of this generation
    ids_after = rep.id.cpu().numpy()
    changed = np.flatnonzero(ids_after != before_id.cpu().numpy())
    assert len(changed) > 0
    for cl in changed:
        gid = int(ids_after[cl])
        assert gid // n_child == gen
        child = gid % n_child
        i = int(np.flatnonzero(kept == child)[0])
        assert got["cell"][i] == cl and (got["status"][i] & 3) == 0
        assert got["fitness"][i] == rep.fitness[cl].item()
        assert got["fitness"][i] > before_fit[cl].item() or before_id[cl].item() == -1
        assert np.array_equal(rep.genome[cl].cpu().numpy(), children[child])
    log(f"[screened] kept {n_keep} of {n_child} (host top-k of the device predictions), "
        f"{len(changed)} cells updated")
    sess.close()


def test_screened_graph_replays_equal_eager(tto):
    import torch
    w = gg.build_config(2, B=512)
    n_child, n_keep = 2048, 205
    sess = make_session(w, tto.TTO_FLOW_F32, max_batch=n_child)
    dev, _ = spaces(sess, w, 3, 3, 120, seed=8)
    net = _net(tto, dev, n_child, seed=9)
    row = np.linspace(-1, 1, 24)
    eager = tto.Repertoire(sess, dev)
    e_ev = tto.ScreenedEvolver(sess, dev, eager, net, n_child, n_keep, seed=5, dense_row=row)
    for _ in range(4):
        e_ev.step()
    torch.cuda.synchronize()
    rep = tto.Repertoire(sess, dev)
    g_ev = tto.ScreenedEvolver(sess, dev, rep, net, n_child, n_keep, seed=5, dense_row=row)
    with tto.Graph() as graph:
        g_ev.step()
    assert int(rep.generation.item()) == 0
    for _ in range(4):
        graph.launch()
        torch.cuda.synchronize()
        _ = rep.fitness.sum().item()
    graph.close()
    for a, b in ((eager.fitness, rep.fitness), (eager.id, rep.id), (eager.genome, rep.genome)):
        assert torch.equal(a, b)
    log(f"[screened] 4 graph replays equal 4 eager screened generations, "
        f"{int((rep.id >= 0).sum().item())} cells")
    sess.close()


def test_gain_rule_keeps_cell_winners_then_lowest_overload(tto):
    """TTO_SCREEN_GAIN: the children kept are, first, the best-predicted child
    of every cell some child is predicted to enter (predicted cell from the
    genome and the predicted maximum loading, predicted fitness minus the
    predicted overload, entering when the cell is empty or its elite worse),
    then the smallest predicted overload terms; recomputed on the host from
    the device's children, the network's predictions and the repertoire."""
    import torch
    w = gg.build_config(2, B=512)
    n_child, n_keep = 4096, 410
    sess = make_session(w, tto.TTO_FLOW_F32, max_batch=n_child)
    dev, _ = spaces(sess, w, 4, 4, 300, seed=5)
    net = _net(tto, dev, n_child, seed=6)
    rep = tto.Repertoire(sess, dev)
    row = np.random.default_rng(2).normal(0, 1, 24).astype(np.float32)
    mu, sd, ref = (0.2, -0.1), (0.3, 0.5), (1.5, 2.0)
    outs = sess.alloc_outputs(n_keep)
    sev = tto.ScreenedEvolver(sess, dev, rep, net, n_child, n_keep, seed=31, dense_row=row,
                              outputs=outs, rule=tto.TTO_SCREEN_GAIN, y_mu=mu, y_sd=sd, ref=ref)
    plain = tto.Evolver(sess, dev, rep, 1024, seed=31)
    for _ in range(4):
        plain.step()
    torch.cuda.synchronize()
    elite_fit = rep.fitness.cpu().numpy()
    elite_id = rep.id.cpu().numpy()
    kids, _ = dev.vary(rep, 31, n_child)
    torch.cuda.synchronize()
    sev.step()
    torch.cuda.synchronize()
    children = sev.children.cpu().numpy()
    assert np.array_equal(children, kids.cpu().numpy())
    off, ids = _features(children, dev.n_a, dev.desc.n_disc, dev.desc.n_actions)
    dvc = torch.device("cuda")
    dense = torch.as_tensor(np.repeat(row[None, :], n_child, axis=0), device=dvc)
    y32 = net.forward(torch.as_tensor(off, device=dvc), torch.as_tensor(ids, device=dvc), dense,
                      n_child).cpu().numpy()
    y = y32.astype(np.float64)
    rho = y[:, 0] * sd[0] + mu[0] + ref[0]
    fit = -100.0 * np.maximum(np.expm1(y[:, 1] * sd[1] + mu[1] + ref[1]), 0.0)
    a, d = children[:, :dev.n_a], children[:, dev.n_a:]
    n_sw = ((a >= 0) & (a < dev.desc.n_actions)).sum(1) + ((d >= 0) & (d < dev.desc.n_disc)).sum(1)
    edges = gg.default_load_edges()
    cell = np.minimum(n_sw, 31) * 32 + (edges[None, :] <= rho[:, None]).sum(1)
    enters = (elite_id[cell] < 0) | (fit > elite_fit[cell])
    first = np.zeros(n_child, bool)
    for cl in np.unique(cell[enters]):
        members = np.flatnonzero(enters & (cell == cl))
        best = members[np.flatnonzero(fit[members] == fit[members].max())[0]]
        first[best] = True
    score = np.where(first, -np.finfo(np.float32).max, y32[:, 1]).astype(np.float32)
    expect = np.sort(np.argsort(score, kind="stable")[:n_keep])
    kept = sev.kept.cpu().numpy()
    assert np.array_equal(kept, expect)
    # the outputs belong to the kept children, in that order
    db = dev.expand(torch.as_tensor(children[kept], device=dvc).contiguous())
    refo = to_numpy(sess.evaluate(db))
    got = to_numpy(outs)
    for k in refo:
        assert np.array_equal(got[k], refo[k], equal_nan=True), k
    log(f"[screened] gain rule: kept {n_keep} of {n_child}: {int(first.sum())} cell winners "
        f"(of {len(np.unique(cell[enters]))} predicted cells entered), the rest by overload")
    sess.close()
