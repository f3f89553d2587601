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


def test_mlp_workspace_sizes_and_descriptor_errors():
    from paper_2605_10128_amd import tto
    base = dict(d_bits=100, d_dense=24, width=512, max_batch=4096, max_train_batch=256)
    p0, b0 = tto.tto_mlp_workspace_bytes(tto.tto_mlp_desc(**base))
    assert p0 > 0 and b0 > 0
    p1, b1 = tto.tto_mlp_workspace_bytes(tto.tto_mlp_desc(**dict(base, width=1024)))
    assert p1 > p0 and b1 > b0
    p2, b2 = tto.tto_mlp_workspace_bytes(tto.tto_mlp_desc(**dict(base, max_batch=8192)))
    assert p2 == p0 and b2 > b0
    for field, bad in (("d_bits", 0), ("d_dense", -1), ("d_dense", 65), ("width", 96),
                       ("width", 32), ("width", 4096), ("max_batch", 0), ("max_train_batch", 0),
                       ("max_train_batch", 1 << 20)):
        with pytest.raises(tto.TTOError) as ei:
            tto.tto_mlp_workspace_bytes(tto.tto_mlp_desc(**dict(base, **{field: bad})))
        assert ei.value.code == tto.TTO_E_INVALID, (field, bad)


def test_ptdf_sizes_and_rejections_before_device_work():
    from paper_2605_10128_amd import tto
    assert tto.tto_ptdf_bytes(4, 4) > 0
    assert tto.tto_ptdf_bytes(2000, 3000) > tto.tto_ptdf_bytes(1000, 3000)
    for n, m in ((1, 4), (4, 0)):
        with pytest.raises(tto.TTOError):
            tto.tto_ptdf_bytes(n, m)
    cases = {"self_loop": ((0, 1, 2, 3), (1, 1, 3, 0), (1.0,) * 4, 0, tto.TTO_E_GRID),
             "bad_endpoint": ((0, 1, 2, 7), (1, 2, 3, 0), (1.0,) * 4, 0, tto.TTO_E_GRID),
             "zero_b": ((0, 1, 2, 3), (1, 2, 3, 0), (1.0, 0.0, 1.0, 1.0), 0, tto.TTO_E_GRID),
             "nan_b": ((0, 1, 2, 3), (1, 2, 3, 0), (1.0, np.nan, 1.0, 1.0), 0, tto.TTO_E_GRID),
             "disconnected": ((0, 2), (1, 3), (1.0, 1.0), 0, tto.TTO_E_GRID),
             "slack": ((0, 1, 2, 3), (1, 2, 3, 0), (1.0,) * 4, 4, tto.TTO_E_GRID),
             "no_ws": ((0, 1, 2, 3), (1, 2, 3, 0), (1.0,) * 4, 0, tto.TTO_E_WORKSPACE)}
    out = np.zeros(16)
    for name, (fr, to, b, slack, code) in cases.items():
        fr, to, b = np.array(fr, np.int32), np.array(to, np.int32), np.array(b, np.float64)
        rc = tto._lib.tto_ptdf_build(4, len(fr), slack, fr.ctypes.data, to.ctypes.data,
                                     b.ctypes.data, out.ctypes.data, None, 0, None)
        assert rc == code, name
        assert tto.tto_last_error()


def _genome_desc(tto, **kw):
    keep = dict(bus=np.array([0, 1, 1], np.int32), off=np.array([0, 2, 3, 5], np.int32),
                br=np.array([0, 3, 0, 1, 2], np.int32), disc=np.array([1, 2], np.int32))
    for k in list(kw):
        if k in keep:
            keep[k] = np.asarray(kw.pop(k), np.int32)
    d = tto.tto_genome_desc(kw.pop("n_a", 2), kw.pop("n_d", 2), len(keep["bus"]),
                            keep["bus"].ctypes.data, keep["off"].ctypes.data, keep["br"].ctypes.data,
                            len(keep["disc"]), keep["disc"].ctypes.data, kw.pop("mut_mean", 1.0),
                            (ct.c_int32 * 4)(*kw.pop("w_action", (1, 1, 1, 1))),
                            (ct.c_int32 * 4)(*kw.pop("w_disc", (1, 1, 1, 1))), kw.pop("p_c1", 0.5))
    assert not kw
    return d, keep


def test_genome_space_sizes_and_descriptor_errors():
    from paper_2605_10128_amd import tto
    d, keep = _genome_desc(tto)
    n0 = tto.tto_genome_space_bytes(d)
    assert n0 > 0
    many = 600                              # station tables grow with the action count
    d2, keep2 = _genome_desc(tto, bus=np.zeros(many), off=np.arange(many + 1),
                             br=np.zeros(many), disc=np.arange(400))
    assert tto.tto_genome_space_bytes(d2) > n0
    for kw, code in ((dict(n_a=9), tto.TTO_E_RANK), (dict(n_d=-1), tto.TTO_E_RANK),
                     (dict(mut_mean=-1.0), tto.TTO_E_INVALID),
                     (dict(mut_mean=float("inf")), tto.TTO_E_INVALID),
                     (dict(p_c1=1.5), tto.TTO_E_INVALID),
                     (dict(w_action=(1, -1, 1, 1)), tto.TTO_E_INVALID),
                     (dict(w_disc=(1, 1, 1 << 21, 1)), tto.TTO_E_INVALID),
                     (dict(off=[1, 2, 3, 5]), tto.TTO_E_INVALID),
                     (dict(off=[0, 0, 3, 5]), tto.TTO_E_INVALID)):
        dd, kk = _genome_desc(tto, **kw)
        with pytest.raises(tto.TTOError) as ei:
            tto.tto_genome_space_bytes(dd)
        assert ei.value.code == code, kw
