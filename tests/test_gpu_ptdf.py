"""Importer on the GPU: tto_ptdf_build against the oracle's dense solve,
tto_bridges against brute-force connectivity, and a session built from the
device PTDF against one built from the host PTDF."""
import time

import numpy as np
import pytest

import gridgen as gg
from oracle import ptdf as optdf
from parity_util import log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg", [1, 2, 3, 4])
def test_ptdf_matches_oracle(cfg):
    import torch
    from paper_2605_10128_amd import tto
    g = gg.build_config(cfg, B=1).grid
    b = 1.0 / g.x_pu
    tto.ptdf_device(g.n_bus, g.from_bus, g.to_bus, b, g.slack)     # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = tto.ptdf_device(g.n_bus, g.from_bus, g.to_bus, b, g.slack)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    ref = optdf.ptdf(g.n_bus, g.from_bus, g.to_bus, b, g.slack)
    err = float(np.abs(P.cpu().numpy() - ref).max())
    log(f"[ptdf] {g.n_bus} buses, {len(b)} branches: built in {ms:.1f} ms, max |diff| {err:.2e}")
    assert err <= 1e-9


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_bridges_match_connectivity(cfg):
    import torch
    from paper_2605_10128_amd import tto
    from parity_util import make_session
    w = gg.build_config(cfg, B=1)
    sess = make_session(w, tto.TTO_FLOW_F64, max_batch=1)
    got = sess.bridges().cpu().numpy().astype(bool)
    torch.cuda.synchronize()
    want = optdf.bridges(w.grid.n_bus, w.grid.from_bus, w.grid.to_bus)
    log(f"[bridges] {w.grid.n_bus} buses: {int(want.sum())} bridges")
    assert np.array_equal(got, want)
    sess.close()


def test_session_from_device_ptdf():
    """A grid created from the device PTDF gives the same base flows and
    evaluation as one created from the oracle's PTDF (within FP64 rounding)."""
    import torch
    from paper_2605_10128_amd import tto
    w = gg.build_config(2, B=64)
    g = w.grid
    b = 1.0 / g.x_pu
    out = {}
    for name, P in (("host", optdf.ptdf(g.n_bus, g.from_bus, g.to_bus, b, g.slack)),
                    ("device", tto.ptdf_device(g.n_bus, g.from_bus, g.to_bus, b, g.slack))):
        s = tto.Session(g.n_bus, g.from_bus, g.to_bus, b, g.limit_mw, P, w.M, w.C, w.P.shape[1],
                        flow_precision=tto.TTO_FLOW_F64, gemm_precision=tto.TTO_GEMM_F64,
                        max_batch=64)
        s.set_injections(w.P)
        s.set_descriptor(gg.default_load_edges())
        o = s.evaluate(tto.device_batch(w.batch))
        torch.cuda.synchronize()
        out[name] = (s.base_flows().cpu().numpy(), o["overload_mw"].cpu().numpy(),
                     o["cell"].cpu().numpy())
        s.close()
    assert np.abs(out["host"][0] - out["device"][0]).max() <= 1e-8
    np.testing.assert_allclose(out["host"][1], out["device"][1], rtol=1e-9, atol=1e-6, equal_nan=True)
    assert np.array_equal(out["host"][2], out["device"][2])
