"""GPU tests of graph capture: replays of a captured evaluate + archive, and
of the whole screened pipeline, against eager calls (through the C ABI).
Each replay is checked, with eager work and synchronisations in between."""
import numpy as np
import pytest

import gridgen as gg
from parity_util import log, make_session

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _np(out):
    return {k: v.detach().cpu().numpy() for k, v in out.items()}


def _spoil(out):
    for v in out.values():
        if v.dtype.is_floating_point:
            v.fill_(12345.0)
        else:
            v.fill_(77)


@pytest.mark.parametrize("flow", ["f32", "f64"])
def test_evaluate_graph_replays_match_eager(flow):
    _need_gpu()
    from paper_2605_10128_amd import tto
    fp = tto.TTO_FLOW_F32 if flow == "f32" else tto.TTO_FLOW_F64
    w = gg.build_config(3, B=1024, n_mon=300, n_cont=400, move_frac=0.2)
    log(f"[graph] evaluate+archive flow={flow} B=1024")
    s = make_session(w, fp, max_batch=1024)
    db = tto.device_batch(w.batch)
    ref = _np(s.evaluate(db))
    a_ref = s.new_archive()
    s.archive_insert(a_ref, {k: torch.as_tensor(v, device=s.device) for k, v in ref.items()},
                     id_base=1000)
    a_ref = [x.cpu().numpy() for x in a_ref]
    out = s.alloc_outputs(1024)
    arc = s.new_archive()
    g = s.capture_evaluate(db, out, arc, id_base=1000)
    try:
        for rep in range(3):
            _spoil(out)
            g.launch()
            eager = _np(s.evaluate(db))          # the program's own work in between
            torch.cuda.synchronize()
            got = _np(out)
            for k in ref:
                assert np.array_equal(got[k], ref[k], equal_nan=True), (rep, k)
                assert np.array_equal(eager[k], ref[k], equal_nan=True), (rep, k)
            assert np.array_equal(arc[0].cpu().numpy(), a_ref[0]), rep
            assert np.array_equal(arc[1].cpu().numpy(), a_ref[1]), rep
    finally:
        g.close()
    log("  3 replays identical to eager")


def test_profiling_stays_eager_under_capture():
    """Stage events come from eager calls only; a graph captured with profiling
    on records none and replays correctly."""
    _need_gpu()
    from paper_2605_10128_amd import tto
    w = gg.build_config(3, B=512, n_mon=200, n_cont=300)
    s = make_session(w, tto.TTO_FLOW_F32, max_batch=512)
    db = tto.device_batch(w.batch)
    out = s.alloc_outputs(512)
    tto.tto_profile_enable(s.handle, True)
    ref = _np(s.evaluate(db))
    ms0 = tto.tto_profile_read(s.handle)
    assert ms0[1] > 0.0
    g = s.capture_evaluate(db, out)
    try:
        for _ in range(2):
            _spoil(out)
            g.launch()
            torch.cuda.synchronize()
            got = _np(out)
            for k in ref:
                assert np.array_equal(got[k], ref[k], equal_nan=True), k
            s.evaluate(db)
            ms = tto.tto_profile_read(s.handle)
            log(f"[graph] eager stage ms after replay {['%.3f' % x for x in ms]}")
            assert ms[1] > 0.0
    finally:
        g.close()
        tto.tto_profile_enable(s.handle, False)


def test_capture_refuses_synchronising_calls():
    _need_gpu()
    from paper_2605_10128_amd import tto
    net = tto.Surrogate(64, 0, width=64, max_batch=8, max_train_batch=8)
    flat = torch.zeros(net.n_params, dtype=torch.float32, device="cuda")
    with pytest.raises(tto.TTOError) as ei:
        with tto.Graph():
            tto.tto_mlp_set_params(net.handle, int(flat.data_ptr()),
                                   int(torch.cuda.current_stream().cuda_stream))
    assert ei.value.code == tto.TTO_E_UNSUPPORTED


def test_screen_pipeline_graph_matches_eager():
    _need_gpu()
    from paper_2605_10128_amd import tto, screen
    w = gg.build_config(3, B=256, n_mon=300, n_cont=400)
    grid = w.grid
    n, k = 4096, 512
    log(f"[graph] screened pipeline n={n} k={k}")
    s = make_session(w, tto.TTO_FLOW_F32, max_batch=k)
    gen = gg.make_candidates_ranked(grid, n, 0x4242, w.split_table, P=w.P)
    off, ids, d_bits = gg.action_bits(grid, gen, len(w.split_table))
    sc = screen.Screener(s, d_bits, w.P.shape[1], width=256, max_screen=n, max_keep=k)
    scale = screen.FeatureScale.fit([screen.injection_summary(w.P)])
    dev = s.device
    db = tto.device_batch(gen)
    off_d, ids_d = torch.as_tensor(off, device=dev), torch.as_tensor(ids, device=dev)
    dense_d = sc.dense_rows(scale, w.P, n)
    o1 = s.alloc_outputs(k)
    sc.screen_and_evaluate(db, off_d, ids_d, dense_d, k, outputs=o1)
    ref, idx_ref = _np(o1), sc.idx[:k].cpu().numpy()
    y_ref = sc.y[:n].cpu().numpy()
    o2 = s.alloc_outputs(k)
    with tto.Graph() as g:
        sc.screen_and_evaluate(db, off_d, ids_d, dense_d, k, outputs=o2)
    try:
        for rep in range(3):
            _spoil(o2)
            sc.idx.fill_(-1)
            g.launch()
            sc.predict(off_d, ids_d, dense_d, n)      # eager work in between
            torch.cuda.synchronize()
            assert np.array_equal(sc.idx[:k].cpu().numpy(), idx_ref), rep
            assert np.array_equal(sc.y[:n].cpu().numpy(), y_ref), rep
            got = _np(o2)
            for name in ref:
                assert np.array_equal(got[name], ref[name], equal_nan=True), (rep, name)
    finally:
        g.close()
    log("  3 replays of forward + top-k + gather + evaluate identical to eager")
