"""The allocation-free archive insertion (tto_archive_insert_noalloc, static
per-GPU scratch) against tto_archive_insert (caller's workspace), through the
C ABI: two calls in a row, the second with fewer cells and fewer candidates,
each from a fresh and from an already filled repertoire; element-wise equal
(integer ids bit-exact, fitness bitwise).  Oversized cell counts are refused."""
import numpy as np
import pytest

import gridgen as gg
from parity_util import log, make_session

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tto():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_10128_amd import tto as t
    return t


def _batch(torch, rng, n, n_cells):
    """Synthetic insertion inputs: fitness with exact ties, cells over the
    whole range (some out of range), a status mix."""
    fit = np.round(rng.normal(-1000.0, 300.0, n), 0)         # many exact ties
    cell = rng.integers(-1, n_cells + 1, n).astype(np.int32)  # -1 and n_cells are skipped
    st = rng.choice(np.array([0, 0, 0, 0, 1, 2, 4, 8], np.uint8), n)
    dev = "cuda"
    return (torch.tensor(fit, dtype=torch.float64, device=dev),
            torch.tensor(cell, dtype=torch.int32, device=dev),
            torch.tensor(st, dtype=torch.uint8, device=dev))


def _insert(tto, torch, s, noalloc, arch, batch, id_base):
    fit_e, id_e = arch
    fit, cell, st = batch
    stream = torch.cuda.current_stream().cuda_stream
    if noalloc:
        tto.tto_archive_insert_noalloc(s.handle, fit_e.data_ptr(), id_e.data_ptr(),
                                       int(fit_e.shape[0]), fit.data_ptr(), cell.data_ptr(),
                                       st.data_ptr(), int(fit.shape[0]), id_base, stream)
    else:
        tto.tto_archive_insert(s.handle, fit_e.data_ptr(), id_e.data_ptr(), int(fit_e.shape[0]),
                               fit.data_ptr(), cell.data_ptr(), st.data_ptr(),
                               int(fit.shape[0]), id_base, s.batch_ws.data_ptr(),
                               s.batch_bytes, stream)


def test_noalloc_insert_matches_workspace_insert(tto):
    import torch
    w = gg.build_config(1)
    s = make_session(w, tto.TTO_FLOW_F64)
    rng = np.random.default_rng(11)
    # (cells, candidates): the second call is smaller in both
    shapes = [(4096, 20000), (1024, 3000)]
    for n_cells, n in shapes:
        log(f"[noalloc] cells {n_cells} candidates {n}")
        b1 = _batch(torch, rng, n, n_cells)
        b2 = _batch(torch, rng, n, n_cells)
        res = []
        for noalloc in (False, True):
            arch = s.new_archive(n_cells)
            _insert(tto, torch, s, noalloc, arch, b1, 0)          # empty repertoire
            first = [a.clone() for a in arch]
            _insert(tto, torch, s, noalloc, arch, b2, n)          # filled repertoire
            torch.cuda.synchronize()
            res.append([x.cpu().numpy() for x in first + list(arch)])
        for a, b in zip(res[0], res[1]):
            assert a.dtype == b.dtype
            np.testing.assert_array_equal(a, b)
        filled = int((res[1][3] >= 0).sum())
        log(f"[noalloc] cells filled {filled} of {n_cells}")
        assert filled > 0


def test_noalloc_insert_refuses_oversized_archives(tto):
    import torch
    w = gg.build_config(1)
    s = make_session(w, tto.TTO_FLOW_F64)
    n_cells = tto.TTO_ARCHIVE_NOALLOC_MAX_CELLS + 1
    fit_e = torch.full((n_cells,), float("-inf"), dtype=torch.float64, device="cuda")
    id_e = torch.full((n_cells,), -1, dtype=torch.int64, device="cuda")
    with pytest.raises(tto.TTOError) as ei:
        tto.tto_archive_insert_noalloc(s.handle, fit_e.data_ptr(), id_e.data_ptr(), n_cells,
                                       0, 0, 0, 0, 0, torch.cuda.current_stream().cuda_stream)
    assert ei.value.code == tto.TTO_E_WORKSPACE
    torch.cuda.synchronize()
    assert (id_e == -1).all()
