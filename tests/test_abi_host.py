"""C ABI on the host (no GPU): the library loads, exports every declared entry
point, and rejects bad arguments before touching the device."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tto.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tto_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2605_10128_amd import tto
    names = _declared()
    assert len(names) >= 12
    lib = ct.CDLL(tto.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(tto.EXPORTED) == names


def test_version():
    from paper_2605_10128_amd import tto
    assert tto.tto_version() == (1, 1)


def _desc(tto, n=4, fr=(0, 1, 2, 3), to=(1, 2, 3, 0), mon=(0, 1, 2, 3), cont=(0, 1, 2, 3), **kw):
    keep = dict(fr=np.array(fr, np.int32), to=np.array(to, np.int32),
                b=np.full(len(fr), 10.0), lim=np.full(len(fr), 100.0),
                mon=np.array(mon, np.int32), cont=np.array(cont, np.int32))
    for k in ("b", "lim"):
        if k in kw:
            keep[k] = np.asarray(kw.pop(k), np.float64)
    d = tto.tto_grid_desc(n, len(fr), kw.pop("slack", 0), kw.pop("T", 1),
                          keep["fr"].ctypes.data, keep["to"].ctypes.data, keep["b"].ctypes.data,
                          keep["lim"].ctypes.data, 4096, len(mon), keep["mon"].ctypes.data,
                          len(cont), keep["cont"].ctypes.data, kw.pop("flow", tto.TTO_FLOW_F32),
                          kw.pop("gemm", tto.TTO_GEMM_F32), kw.pop("max_batch", 8))
    return d, keep


def test_workspace_sizes_and_argument_errors():
    from paper_2605_10128_amd import tto
    d, keep = _desc(tto)
    g, b = tto.tto_workspace_bytes(d)
    assert g > 0 and b > 0
    for field, bad, code in (("n_timesteps", 0, tto.TTO_E_INVALID),
                             ("n_timesteps", 33, tto.TTO_E_INVALID),
                             ("flow_precision", 7, tto.TTO_E_INVALID),
                             ("gemm_precision", 9, tto.TTO_E_INVALID),
                             ("slack", 4, tto.TTO_E_GRID),
                             ("max_batch", 0, tto.TTO_E_INVALID)):
        d2, k2 = _desc(tto)
        setattr(d2, field, bad)
        with pytest.raises(tto.TTOError) as ei:
            tto.tto_workspace_bytes(d2)
        assert ei.value.code == code, field


@pytest.mark.parametrize("case,code", [
    ("disconnected", -2), ("self_loop", -2), ("bad_endpoint", -2), ("neg_b", -2),
    ("zero_limit", -2), ("repeated_monitored", -2), ("null_ws", -4), ("small_ws", -4)])
def test_grid_create_rejects_before_any_device_work(case, code):
    from paper_2605_10128_amd import tto
    kw = {}
    if case == "disconnected":
        kw = dict(n=5, fr=(0, 1, 2, 3), to=(1, 2, 0, 4), mon=(0,), cont=(0,))
        d, keep = _desc(tto, **kw)
        d.n_bus = 6
    elif case == "self_loop":
        d, keep = _desc(tto, fr=(0, 1, 2, 3), to=(1, 1, 3, 0))
    elif case == "bad_endpoint":
        d, keep = _desc(tto, fr=(0, 1, 2, 9), to=(1, 2, 3, 0))
    elif case == "neg_b":
        d, keep = _desc(tto, b=[10.0, -1.0, 10.0, 10.0])
    elif case == "zero_limit":
        d, keep = _desc(tto, lim=[100.0, 0.0, 100.0, 100.0])
    elif case == "repeated_monitored":
        d, keep = _desc(tto, mon=(0, 1, 1))
    else:
        d, keep = _desc(tto)
    g, _ = tto.tto_workspace_bytes(d) if case in ("null_ws", "small_ws") else (0, 0)
    ws, nbytes = 0, 0
    if case == "small_ws":
        ws, nbytes = 256, g - 1
    with pytest.raises(tto.TTOError) as ei:
        tto.tto_grid_create(d, ws, nbytes, 0)
    assert ei.value.code == code
    assert tto.tto_last_error()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2605_10128_amd import tto
    monkeypatch.setattr(tto, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        tto._load()


def test_product_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2605_10128_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", src, re.M), f
                assert "oracle/" not in src, f
