"""ctypes binding of libtto (include/tto.h): same entry-point names, argument
marshalling only.  Every step of the evaluation runs in the HIP library; torch
is used for device memory and streams.  Importing this module fails loudly if
the built library is missing."""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TTO_LIBRARY selects another build of the same library (the host-sanitized
# libtto_san.so); it is never a substitute for a missing one
LIB_PATH = os.environ.get("TTO_LIBRARY") or os.path.join(_HERE, "libtto.so")

TTO_OK = 0
TTO_E_INVALID, TTO_E_GRID, TTO_E_RANK, TTO_E_WORKSPACE, TTO_E_HIP, TTO_E_UNSUPPORTED = -1, -2, -3, -4, -5, -6
TTO_FLOW_F64, TTO_FLOW_F32 = 0, 1
TTO_GEMM_F64, TTO_GEMM_F32, TTO_GEMM_BF16, TTO_GEMM_F16 = 0, 1, 2, 3
TTO_GEMM_BF16X3, TTO_GEMM_F16X3 = 4, 5
TTO_ST_ISLANDED, TTO_ST_INVALID, TTO_ST_REFINED, TTO_ST_REFINE_SKIPPED = 1, 2, 4, 8
TTO_ST_NONFINITE = 0x10
TTO_MAX_RANK, TTO_MAX_T, TTO_MAX_MOVED, TTO_MAX_LOAD_BINS = 8, 32, 64, 64
TTO_ARCHIVE_NOALLOC_MAX_CELLS = 65536

_vp = ct.c_void_p
_i32 = ct.c_int32


class tto_grid_desc(ct.Structure):
    _fields_ = [("n_bus", _i32), ("n_branch", _i32), ("slack", _i32), ("n_timesteps", _i32),
                ("from_bus", _vp), ("to_bus", _vp), ("susceptance", _vp), ("limit_mw", _vp),
                ("ptdf", _vp), ("n_monitored", _i32), ("monitored", _vp),
                ("n_contingency", _i32), ("contingency", _vp), ("flow_precision", _i32),
                ("gemm_precision", _i32), ("max_batch", _i32)]


class tto_descriptor_cfg(ct.Structure):
    _fields_ = [("n_count_bins", _i32), ("n_load_bins", _i32), ("load_edges", _vp),
                ("w_c0", ct.c_double), ("w_c", ct.c_double), ("kind", _i32)]


TTO_DESC_COUNT_LOAD, TTO_DESC_PAPER = 0, 1
TTO_PAPER_CELLS = 552


class tto_batch(ct.Structure):
    _fields_ = [("n_cand", _i32), ("n_open_slots", _i32), ("n_split_slots", _i32),
                ("open", _vp), ("split_bus", _vp), ("moved_off", _vp), ("moved_br", _vp),
                ("moved_p_mw", _vp)]


OUTPUT_FIELDS = ["status", "n_island_cont", "overload_mw", "n_crit_n1", "n_crit_n0",
                 "max_loading", "worst_branch", "worst_cont", "worst_t", "fitness", "cell",
                 "base_flows", "fmax", "n1_flows"]


class tto_outputs(ct.Structure):
    _fields_ = [(f, _vp) for f in OUTPUT_FIELDS]


class tto_genome_desc(ct.Structure):
    _fields_ = [("n_action_slots", _i32), ("n_disc_slots", _i32), ("n_actions", _i32),
                ("action_bus", _vp), ("action_moved_off", _vp), ("action_moved_br", _vp),
                ("n_disc", _i32), ("disc_branch", _vp), ("mut_mean", ct.c_double),
                ("w_action", _i32 * 4), ("w_disc", _i32 * 4), ("p_c1", ct.c_double)]


class tto_repertoire(ct.Structure):
    _fields_ = [("n_cells", _i32), ("fitness", _vp), ("id", _vp), ("genome", _vp),
                ("generation", _vp)]


class tto_mlp_desc(ct.Structure):
    _fields_ = [("d_bits", _i32), ("d_dense", _i32), ("width", _i32), ("max_batch", _i32),
                ("max_train_batch", _i32)]


class TTOError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tto error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libtto.so not built at {LIB_PATH}; run __graft_entry__.build()")
    # torch's HIP runtime must be the one the library binds to: loaded first,
    # its libamdhip64 satisfies the library's dependency by soname, so device
    # memory and stream handles from torch are valid in library calls (loaded
    # the other way round, the process would hold two HIP runtimes)
    import torch  # noqa: F401
    lib = ct.CDLL(LIB_PATH)
    P = ct.POINTER
    sig = {
        "tto_version": (_i32, [P(_i32), P(_i32)]),
        "tto_last_error": (ct.c_char_p, []),
        "tto_workspace_bytes": (_i32, [P(tto_grid_desc), P(ct.c_size_t), P(ct.c_size_t)]),
        "tto_grid_create": (_i32, [P(tto_grid_desc), _vp, ct.c_size_t, _vp, P(_vp)]),
        "tto_grid_destroy": (None, [_vp]),
        "tto_set_injections": (_i32, [_vp, _vp, _vp]),
        "tto_get_base_flows": (_i32, [_vp, _vp, _vp]),
        "tto_set_descriptor": (_i32, [_vp, P(tto_descriptor_cfg)]),
        "tto_evaluate": (_i32, [_vp, P(tto_batch), P(tto_outputs), _vp, ct.c_size_t, _vp]),
        "tto_archive_insert": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _i32, ct.c_int64, _vp,
                                      ct.c_size_t, _vp]),
        "tto_archive_insert_noalloc": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _i32,
                                              ct.c_int64, _vp]),
        "tto_profile_enable": (_i32, [_vp, _i32]),
        "tto_profile_read": (_i32, [_vp, P(ct.c_double)]),
        "tto_set_sweep_plan": (_i32, [_vp, _i32, _i32, _i32, _i32]),
        "tto_set_refine": (_i32, [_vp, _i32, ct.c_double]),
        "tto_batch_gather": (_i32, [P(tto_batch), _vp, _i32, _i32, _vp, _vp, _vp, _vp, _i32, _vp,
                                    P(tto_batch), _vp]),
        "tto_mlp_workspace_bytes": (_i32, [P(tto_mlp_desc), P(ct.c_size_t), P(ct.c_size_t)]),
        "tto_mlp_create": (_i32, [P(tto_mlp_desc), _vp, ct.c_size_t, P(_vp)]),
        "tto_mlp_destroy": (None, [_vp]),
        "tto_mlp_n_params": (_i32, [_vp, P(ct.c_int64)]),
        "tto_mlp_set_params": (_i32, [_vp, _vp, _vp]),
        "tto_mlp_get_params": (_i32, [_vp, _vp, _vp]),
        "tto_mlp_forward": (_i32, [_vp, _vp, _vp, _vp, _i32, _vp, _vp, ct.c_size_t, _vp]),
        "tto_mlp_gradients": (_i32, [_vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, ct.c_size_t,
                                     _vp]),
        "tto_mlp_train_step": (_i32, [_vp, _vp, _vp, _vp, _vp, _i32, ct.c_float, _vp, _vp,
                                      ct.c_size_t, _vp]),
        "tto_topk_smallest": (_i32, [_vp, _i32, _i32, _i32, _vp, _vp]),
        "tto_graph_begin": (_i32, [P(_vp), P(_vp)]),
        "tto_graph_end": (_i32, [_vp]),
        "tto_graph_launch": (_i32, [_vp, _vp]),
        "tto_graph_destroy": (None, [_vp]),
        "tto_evaluate_capture": (_i32, [_vp, P(tto_batch), P(tto_outputs), _vp, ct.c_size_t, _vp,
                                        _vp, _i32, ct.c_int64, P(_vp)]),
        "tto_get_sweep_plan": (_i32, [_vp, P(_i32), P(_i32), P(_i32), P(_i32)]),
        "tto_ptdf_bytes": (_i32, [_i32, _i32, P(ct.c_size_t)]),
        "tto_ptdf_build": (_i32, [_i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, ct.c_size_t, _vp]),
        "tto_bridges": (_i32, [_vp, _vp, _vp]),
        "tto_busbar_set_bytes": (_i32, [_vp, _i32, P(ct.c_size_t)]),
        "tto_busbar_set_create": (_i32, [_vp, _i32, _vp, _vp, _vp, ct.c_size_t, _vp, P(_vp)]),
        "tto_busbar_set_destroy": (None, [_vp]),
        "tto_busbar_bytes": (_i32, [_vp, _vp, _i32, P(ct.c_size_t)]),
        "tto_busbar_evaluate": (_i32, [_vp, _vp, P(tto_batch), _vp, ct.c_double, _vp, _vp, _vp,
                                       _vp, _vp, ct.c_size_t, _vp, ct.c_size_t, _vp]),
        "tto_worst_k_bytes": (_i32, [_vp, _i32, P(ct.c_size_t)]),
        "tto_worst_contingencies": (_i32, [_vp, P(tto_batch), _i32, _vp, _vp, _vp, ct.c_size_t,
                                           _vp, ct.c_size_t, _vp]),
        "tto_genome_space_bytes": (_i32, [P(tto_genome_desc), P(ct.c_size_t)]),
        "tto_genome_space_create": (_i32, [_vp, P(tto_genome_desc), _vp, ct.c_size_t, _vp,
                                           P(_vp)]),
        "tto_genome_space_destroy": (None, [_vp]),
        "tto_genome_max_moved": (_i32, [_vp, P(_i32)]),
        "tto_vary": (_i32, [_vp, _vp, _vp, _i32, ct.c_uint64, _vp, _i32, _vp, _vp, _vp]),
        "tto_genome_expand": (_i32, [_vp, _vp, _i32, _vp, _vp, _vp, _vp, ct.c_int64, _vp]),
        "tto_generation_bytes": (_i32, [_vp, _vp, _i32, P(ct.c_size_t)]),
        "tto_screened_generation_bytes": (_i32, [_vp, _vp, _vp, _i32, _i32, P(ct.c_size_t)]),
        "tto_screened_generation": (_i32, [_vp, _vp, P(tto_repertoire), _vp, _vp, _vp,
                                           ct.c_uint64, _i32, _i32, _vp, _vp, _vp, ct.c_size_t,
                                           _vp, ct.c_size_t, _vp, ct.c_size_t, _vp]),
        "tto_generation": (_i32, [_vp, _vp, P(tto_repertoire), ct.c_uint64, _i32,
                                  P(tto_outputs), _vp, ct.c_size_t, _vp, ct.c_size_t, _vp]),
        "tto_autotune": (_i32, [_vp, P(tto_batch), P(tto_outputs), _vp, ct.c_size_t, _vp,
                                ct.c_char_p, P(_i32)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()

EXPORTED = ["tto_version", "tto_last_error", "tto_workspace_bytes", "tto_grid_create",
            "tto_grid_destroy", "tto_set_injections", "tto_get_base_flows", "tto_set_descriptor",
            "tto_evaluate", "tto_archive_insert", "tto_archive_insert_noalloc",
            "tto_profile_enable", "tto_profile_read",
            "tto_set_sweep_plan", "tto_get_sweep_plan", "tto_autotune", "tto_set_refine",
            "tto_batch_gather", "tto_mlp_workspace_bytes", "tto_mlp_create", "tto_mlp_destroy",
            "tto_mlp_n_params", "tto_mlp_set_params", "tto_mlp_get_params", "tto_mlp_forward",
            "tto_mlp_gradients", "tto_mlp_train_step", "tto_topk_smallest",
            "tto_graph_begin", "tto_graph_end", "tto_graph_launch", "tto_graph_destroy",
            "tto_evaluate_capture", "tto_genome_space_bytes", "tto_genome_space_create",
            "tto_genome_space_destroy", "tto_genome_max_moved", "tto_vary", "tto_genome_expand",
            "tto_generation_bytes", "tto_generation", "tto_worst_k_bytes",
            "tto_worst_contingencies", "tto_busbar_set_bytes", "tto_busbar_set_create",
            "tto_busbar_set_destroy", "tto_busbar_bytes", "tto_busbar_evaluate",
            "tto_ptdf_bytes", "tto_ptdf_build", "tto_bridges", "tto_screened_generation_bytes",
            "tto_screened_generation"]


def _check(code: int):
    if code != TTO_OK:
        raise TTOError(code, _lib.tto_last_error().decode())


# ---- entry points (same names as the C ABI) --------------------------------
def tto_version():
    a, b = _i32(), _i32()
    _check(_lib.tto_version(ct.byref(a), ct.byref(b)))
    return a.value, b.value


def tto_last_error() -> str:
    return _lib.tto_last_error().decode()


def tto_workspace_bytes(desc: tto_grid_desc):
    g, b = ct.c_size_t(), ct.c_size_t()
    _check(_lib.tto_workspace_bytes(ct.byref(desc), ct.byref(g), ct.byref(b)))
    return g.value, b.value


def tto_grid_create(desc: tto_grid_desc, grid_ws: int, grid_bytes: int, stream: int) -> int:
    h = _vp()
    _check(_lib.tto_grid_create(ct.byref(desc), _vp(grid_ws), grid_bytes, _vp(stream), ct.byref(h)))
    return h.value


def tto_grid_destroy(handle: int):
    _lib.tto_grid_destroy(_vp(handle))


def tto_set_injections(handle: int, p_mw: int, stream: int):
    _check(_lib.tto_set_injections(_vp(handle), _vp(p_mw), _vp(stream)))


def tto_get_base_flows(handle: int, out: int, stream: int):
    _check(_lib.tto_get_base_flows(_vp(handle), _vp(out), _vp(stream)))


def tto_set_descriptor(handle: int, cfg: tto_descriptor_cfg):
    _check(_lib.tto_set_descriptor(_vp(handle), ct.byref(cfg)))


def tto_evaluate(handle: int, batch: tto_batch, outputs: tto_outputs, ws: int, ws_bytes: int,
                 stream: int):
    _check(_lib.tto_evaluate(_vp(handle), ct.byref(batch), ct.byref(outputs), _vp(ws), ws_bytes,
                             _vp(stream)))


def tto_archive_insert(handle: int, elite_fit: int, elite_id: int, n_cells: int, fitness: int,
                       cell: int, status: int, n_cand: int, id_base: int, ws: int, ws_bytes: int,
                       stream: int):
    _check(_lib.tto_archive_insert(_vp(handle), _vp(elite_fit), _vp(elite_id), n_cells,
                                   _vp(fitness), _vp(cell), _vp(status), n_cand, id_base, _vp(ws),
                                   ws_bytes, _vp(stream)))


def tto_archive_insert_noalloc(handle: int, elite_fit: int, elite_id: int, n_cells: int,
                               fitness: int, cell: int, status: int, n_cand: int, id_base: int,
                               stream: int):
    _check(_lib.tto_archive_insert_noalloc(_vp(handle), _vp(elite_fit), _vp(elite_id), n_cells,
                                           _vp(fitness), _vp(cell), _vp(status), n_cand, id_base,
                                           _vp(stream)))


def tto_profile_enable(handle: int, enable: bool):
    _check(_lib.tto_profile_enable(_vp(handle), 1 if enable else 0))


def tto_profile_read(handle: int):
    ms = (ct.c_double * 4)()
    _check(_lib.tto_profile_read(_vp(handle), ms))
    return list(ms)


def tto_set_sweep_plan(handle: int, lanes: int = 256, branches_per_lane: int = 1, order: int = 0,
                       persistent: bool = False):
    _check(_lib.tto_set_sweep_plan(_vp(handle), int(lanes), int(branches_per_lane), int(order),
                                   int(persistent)))


def tto_set_refine(handle: int, enable: bool, margin_mw: float = 8e-3):
    _check(_lib.tto_set_refine(_vp(handle), 1 if enable else 0, float(margin_mw)))


def tto_get_sweep_plan(handle: int) -> dict:
    v = [_i32() for _ in range(4)]
    _check(_lib.tto_get_sweep_plan(_vp(handle), *[ct.byref(x) for x in v]))
    return {"lanes": v[0].value, "branches_per_lane": v[1].value, "order": v[2].value,
            "persistent": bool(v[3].value)}


def tto_autotune(handle: int, batch: tto_batch, outputs: tto_outputs, ws: int, ws_bytes: int,
                 stream: int, cache_path: str = ""):
    ch = (_i32 * 5)()
    _check(_lib.tto_autotune(_vp(handle), ct.byref(batch), ct.byref(outputs), _vp(ws), ws_bytes,
                             _vp(stream), cache_path.encode(), ch))
    return {"lanes": ch[0], "branches_per_lane": ch[1], "order": ch[2],
            "persistent": bool(ch[3]), "from_cache": bool(ch[4])}


def tto_topk_smallest(score: int, n: int, stride: int, k: int, idx_out: int, stream: int):
    _check(_lib.tto_topk_smallest(_vp(score), n, stride, k, _vp(idx_out), _vp(stream)))


def tto_batch_gather(src: tto_batch, idx: int, k: int, T: int, d_open: int, d_split: int,
                     d_moff: int, d_mbr: int, cap: int, d_mp: int, stream: int) -> tto_batch:
    dst = tto_batch()
    _check(_lib.tto_batch_gather(ct.byref(src), _vp(idx), k, T, _vp(d_open), _vp(d_split),
                                 _vp(d_moff), _vp(d_mbr), cap, _vp(d_mp), ct.byref(dst),
                                 _vp(stream)))
    return dst


def tto_mlp_workspace_bytes(desc: tto_mlp_desc):
    a, b = ct.c_size_t(), ct.c_size_t()
    _check(_lib.tto_mlp_workspace_bytes(ct.byref(desc), ct.byref(a), ct.byref(b)))
    return a.value, b.value


def tto_mlp_create(desc: tto_mlp_desc, ws: int, nbytes: int) -> int:
    h = _vp()
    _check(_lib.tto_mlp_create(ct.byref(desc), _vp(ws), nbytes, ct.byref(h)))
    return h.value


def tto_mlp_destroy(handle: int):
    _lib.tto_mlp_destroy(_vp(handle))


def tto_mlp_n_params(handle: int) -> int:
    n = ct.c_int64()
    _check(_lib.tto_mlp_n_params(_vp(handle), ct.byref(n)))
    return n.value


def tto_mlp_set_params(handle: int, params: int, stream: int):
    _check(_lib.tto_mlp_set_params(_vp(handle), _vp(params), _vp(stream)))


def tto_mlp_get_params(handle: int, params: int, stream: int):
    _check(_lib.tto_mlp_get_params(_vp(handle), _vp(params), _vp(stream)))


def tto_mlp_forward(handle, off, idx, dense, n, y, ws, nbytes, stream):
    _check(_lib.tto_mlp_forward(_vp(handle), _vp(off), _vp(idx), _vp(dense), n, _vp(y), _vp(ws),
                                nbytes, _vp(stream)))


def tto_mlp_gradients(handle, off, idx, dense, target, n, grad, loss, ws, nbytes, stream):
    _check(_lib.tto_mlp_gradients(_vp(handle), _vp(off), _vp(idx), _vp(dense), _vp(target), n,
                                  _vp(grad), _vp(loss), _vp(ws), nbytes, _vp(stream)))


def tto_mlp_train_step(handle, off, idx, dense, target, n, lr, loss, ws, nbytes, stream):
    _check(_lib.tto_mlp_train_step(_vp(handle), _vp(off), _vp(idx), _vp(dense), _vp(target), n,
                                   float(lr), _vp(loss), _vp(ws), nbytes, _vp(stream)))


def tto_graph_begin():
    g, cs = _vp(), _vp()
    _check(_lib.tto_graph_begin(ct.byref(g), ct.byref(cs)))
    return g.value, cs.value or 0


def tto_graph_end(graph: int):
    _check(_lib.tto_graph_end(_vp(graph)))


def tto_graph_launch(graph: int, stream: int):
    _check(_lib.tto_graph_launch(_vp(graph), _vp(stream)))


def tto_graph_destroy(graph: int):
    _lib.tto_graph_destroy(_vp(graph))


def tto_evaluate_capture(handle, batch: "tto_batch", outputs: "tto_outputs", ws, ws_bytes,
                         elite_fit, elite_id, n_cells, id_base) -> int:
    g = _vp()
    _check(_lib.tto_evaluate_capture(_vp(handle), ct.byref(batch), ct.byref(outputs), _vp(ws),
                                     ws_bytes, _vp(elite_fit), _vp(elite_id), int(n_cells),
                                     int(id_base), ct.byref(g)))
    return g.value


def tto_ptdf_bytes(n_bus: int, n_branch: int) -> int:
    n = ct.c_size_t()
    _check(_lib.tto_ptdf_bytes(int(n_bus), int(n_branch), ct.byref(n)))
    return n.value


def tto_ptdf_build(n_bus: int, n_branch: int, slack: int, from_bus: int, to_bus: int,
                   susceptance: int, ptdf: int, ws: int, nbytes: int, stream: int):
    _check(_lib.tto_ptdf_build(int(n_bus), int(n_branch), int(slack), _vp(from_bus), _vp(to_bus),
                               _vp(susceptance), _vp(ptdf), _vp(ws), nbytes, _vp(stream)))


def tto_bridges(grid: int, out: int, stream: int):
    _check(_lib.tto_bridges(_vp(grid), _vp(out), _vp(stream)))


def ptdf_device(n_bus, from_bus, to_bus, susceptance, slack=0, device="cuda"):
    """PTDF [n_branch][n_bus] (device FP64 tensor) built on the GPU."""
    import torch
    fr = np.ascontiguousarray(from_bus, dtype=np.int32)
    to = np.ascontiguousarray(to_bus, dtype=np.int32)
    b = np.ascontiguousarray(susceptance, dtype=np.float64)
    out = torch.empty((len(fr), int(n_bus)), dtype=torch.float64, device=device)
    nb = tto_ptdf_bytes(int(n_bus), len(fr))
    ws = torch.empty(nb, dtype=torch.uint8, device=device)
    tto_ptdf_build(int(n_bus), len(fr), int(slack), fr.ctypes.data, to.ctypes.data, b.ctypes.data,
                   _ptr(out), _ptr(ws), nb, int(torch.cuda.current_stream().cuda_stream))
    del ws
    return out


def tto_busbar_set_bytes(grid: int, n_busbars: int) -> int:
    n = ct.c_size_t()
    _check(_lib.tto_busbar_set_bytes(_vp(grid), int(n_busbars), ct.byref(n)))
    return n.value


def tto_busbar_set_create(grid: int, n_busbars: int, buses: int, ptdf: int, ws: int, nbytes: int,
                          stream: int) -> int:
    h = _vp()
    _check(_lib.tto_busbar_set_create(_vp(grid), int(n_busbars), _vp(buses), _vp(ptdf), _vp(ws),
                                      nbytes, _vp(stream), ct.byref(h)))
    return h.value


def tto_busbar_set_destroy(handle: int):
    _lib.tto_busbar_set_destroy(_vp(handle))


def tto_busbar_bytes(grid: int, bset: int, n_cand: int) -> int:
    n = ct.c_size_t()
    _check(_lib.tto_busbar_bytes(_vp(grid), _vp(bset), int(n_cand), ct.byref(n)))
    return n.value


def tto_busbar_evaluate(grid: int, bset: int, batch: "tto_batch", p_mw: int, lambda_b_pre: float,
                        fitness_f1: int, lambda_b: int, n_island: int, fitness_f2: int,
                        batch_ws: int, batch_bytes: int, bb_ws: int, bb_bytes: int, stream: int):
    _check(_lib.tto_busbar_evaluate(_vp(grid), _vp(bset), ct.byref(batch), _vp(p_mw),
                                    float(lambda_b_pre), _vp(fitness_f1), _vp(lambda_b),
                                    _vp(n_island), _vp(fitness_f2), _vp(batch_ws), batch_bytes,
                                    _vp(bb_ws), bb_bytes, _vp(stream)))


def tto_worst_k_bytes(grid: int, n_cand: int) -> int:
    n = ct.c_size_t()
    _check(_lib.tto_worst_k_bytes(_vp(grid), int(n_cand), ct.byref(n)))
    return n.value


def tto_worst_contingencies(grid: int, batch: "tto_batch", k: int, ids: int, energy: int,
                            batch_ws: int, batch_bytes: int, wk_ws: int, wk_bytes: int,
                            stream: int):
    _check(_lib.tto_worst_contingencies(_vp(grid), ct.byref(batch), int(k), _vp(ids),
                                        _vp(energy), _vp(batch_ws), batch_bytes, _vp(wk_ws),
                                        wk_bytes, _vp(stream)))


def tto_genome_space_bytes(desc: tto_genome_desc) -> int:
    n = ct.c_size_t()
    _check(_lib.tto_genome_space_bytes(ct.byref(desc), ct.byref(n)))
    return n.value


def tto_genome_space_create(grid: int, desc: tto_genome_desc, ws: int, nbytes: int,
                            stream: int) -> int:
    h = _vp()
    _check(_lib.tto_genome_space_create(_vp(grid), ct.byref(desc), _vp(ws), nbytes, _vp(stream),
                                        ct.byref(h)))
    return h.value


def tto_genome_space_destroy(gs: int):
    _lib.tto_genome_space_destroy(_vp(gs))


def tto_genome_max_moved(gs: int) -> int:
    n = _i32()
    _check(_lib.tto_genome_max_moved(_vp(gs), ct.byref(n)))
    return n.value


def tto_vary(gs: int, elite_id: int, elite_genome: int, n_cells: int, seed: int,
             generation: int, n_child: int, children: int, b_mc: int, stream: int):
    _check(_lib.tto_vary(_vp(gs), _vp(elite_id), _vp(elite_genome), int(n_cells),
                         ct.c_uint64(seed), _vp(generation), int(n_child), _vp(children),
                         _vp(b_mc), _vp(stream)))


def tto_genome_expand(gs: int, genomes: int, n: int, open_: int, split_bus: int, moved_off: int,
                      moved_br: int, moved_cap: int, stream: int):
    _check(_lib.tto_genome_expand(_vp(gs), _vp(genomes), int(n), _vp(open_), _vp(split_bus),
                                  _vp(moved_off), _vp(moved_br), int(moved_cap), _vp(stream)))


def tto_generation_bytes(grid: int, gs: int, n_child: int) -> int:
    n = ct.c_size_t()
    _check(_lib.tto_generation_bytes(_vp(grid), _vp(gs), int(n_child), ct.byref(n)))
    return n.value


def tto_generation(grid: int, gs: int, rep: tto_repertoire, seed: int, n_child: int,
                   outputs: Optional["tto_outputs"], gen_ws: int, gen_bytes: int, batch_ws: int,
                   batch_bytes: int, stream: int):
    _check(_lib.tto_generation(_vp(grid), _vp(gs), ct.byref(rep), ct.c_uint64(seed),
                               int(n_child), ct.byref(outputs) if outputs is not None else None,
                               _vp(gen_ws), gen_bytes, _vp(batch_ws), batch_bytes, _vp(stream)))


def tto_screened_generation_bytes(grid: int, gs: int, net: int, n_child: int,
                                  n_keep: int) -> int:
    n = ct.c_size_t()
    _check(_lib.tto_screened_generation_bytes(_vp(grid), _vp(gs), _vp(net), int(n_child),
                                              int(n_keep), ct.byref(n)))
    return n.value


TTO_SCREEN_OVERLOAD, TTO_SCREEN_GAIN = 0, 1


class tto_screen_cfg(ct.Structure):
    _fields_ = [("rule", _i32), ("y_mu", ct.c_double * 2), ("y_sd", ct.c_double * 2),
                ("ref", ct.c_double * 2), ("overload_scale_mw", ct.c_double)]


def tto_screened_generation(grid: int, gs: int, rep: tto_repertoire, net: int, dense_row: int,
                            cfg: Optional[tto_screen_cfg], seed: int, n_child: int, n_keep: int,
                            outputs: Optional["tto_outputs"], kept_out: int, gen_ws: int,
                            gen_bytes: int, mlp_ws: int, mlp_bytes: int, batch_ws: int,
                            batch_bytes: int, stream: int):
    _check(_lib.tto_screened_generation(
        _vp(grid), _vp(gs), ct.byref(rep), _vp(net), _vp(dense_row),
        ct.byref(cfg) if cfg is not None else None, ct.c_uint64(seed), int(n_child), int(n_keep),
        ct.byref(outputs) if outputs is not None else None, _vp(kept_out), _vp(gen_ws),
        gen_bytes, _vp(mlp_ws), mlp_bytes, _vp(batch_ws), batch_bytes, _vp(stream)))


class Graph:
    """A captured sequence of library calls, replayed with launch().

    Use as a context manager: inside the `with` block torch's current stream
    is the capture stream, so Session / Surrogate / Screener calls made there
    are recorded (their buffers must already be allocated)."""

    def __init__(self, handle: int = 0):
        self.handle = handle
        self._ctx = None

    def __enter__(self):
        import torch
        self.handle, cs = tto_graph_begin()
        self._ctx = torch.cuda.stream(torch.cuda.ExternalStream(cs))
        self._ctx.__enter__()
        return self

    def __exit__(self, et, ev, tb):
        self._ctx.__exit__(et, ev, tb)
        self._ctx = None
        if et is None:
            try:
                tto_graph_end(self.handle)
            except Exception:
                self.close()
                raise
        else:
            self.close()          # ends the open capture before anything else runs
        return False

    def launch(self, stream: Optional[int] = None):
        import torch
        s = int(torch.cuda.current_stream().cuda_stream) if stream is None else stream
        tto_graph_launch(self.handle, s)

    def close(self):
        if self.handle:
            tto_graph_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Surrogate:
    """Torch-allocated workspaces around the tto_mlp_* entry points."""

    def __init__(self, d_bits, d_dense, width=512, max_batch=65536, max_train_batch=4096,
                 device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.desc = tto_mlp_desc(int(d_bits), int(d_dense), int(width), int(max_batch),
                                 int(max_train_batch))
        self.pbytes, self.bbytes = tto_mlp_workspace_bytes(self.desc)
        self.pws = torch.empty(self.pbytes, dtype=torch.uint8, device=self.device)
        self.bws = torch.empty(self.bbytes, dtype=torch.uint8, device=self.device)
        self.handle = tto_mlp_create(self.desc, _ptr(self.pws), self.pbytes)
        self.n_params = tto_mlp_n_params(self.handle)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    @property
    def stream(self) -> int:
        return int(self.torch.cuda.current_stream(self.device).cuda_stream)

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                tto_mlp_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def set_params(self, flat):
        t = self.torch.as_tensor(np.ascontiguousarray(flat, dtype=np.float32), device=self.device)
        tto_mlp_set_params(self.handle, _ptr(t), self.stream)
        self.torch.cuda.current_stream(self.device).synchronize()

    def get_params(self):
        out = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.device)
        tto_mlp_get_params(self.handle, _ptr(out), self.stream)
        return out

    def forward(self, off, idx, dense, n, y=None):
        if y is None:
            y = self.torch.empty((n, 2), dtype=self.torch.float32, device=self.device)
        tto_mlp_forward(self.handle, _ptr(off), _ptr(idx), _ptr(dense), n, _ptr(y),
                        _ptr(self.bws), self.bbytes, self.stream)
        return y

    def gradients(self, off, idx, dense, target, n):
        g = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.device)
        tto_mlp_gradients(self.handle, _ptr(off), _ptr(idx), _ptr(dense), _ptr(target), n,
                          _ptr(g), _ptr(self.loss), _ptr(self.bws), self.bbytes, self.stream)
        return g, self.loss

    def train_step(self, off, idx, dense, target, n, lr):
        tto_mlp_train_step(self.handle, _ptr(off), _ptr(idx), _ptr(dense), _ptr(target), n, lr,
                           _ptr(self.loss), _ptr(self.bws), self.bbytes, self.stream)
        return self.loss


def he_init(d_bits, d_dense, width, seed=0):
    """He-normal weights, zero biases, flat in the tto_mlp parameter order."""
    rng = np.random.default_rng(seed)
    H = width
    parts = [
        rng.normal(0, np.sqrt(2.0 / 8.0), (d_bits, H)),          # ~8 set bits per sample
        rng.normal(0, np.sqrt(2.0 / max(d_dense, 1)), (d_dense, H)),
        np.zeros(H), rng.normal(0, np.sqrt(2.0 / H), (H, H)), np.zeros(H),
        rng.normal(0, np.sqrt(2.0 / H), (H, H)), np.zeros(H),
        rng.normal(0, np.sqrt(1.0 / H), (H, 2)), np.zeros(2),
    ]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def split_params(flat, d_bits, d_dense, width):
    H = width
    shapes = [("W1b", (d_bits, H)), ("W1d", (d_dense, H)), ("b1", (H,)), ("W2", (H, H)),
              ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)), ("W4", (H, 2)), ("b4", (2,))]
    out, o = {}, 0
    for name, shp in shapes:
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + n]).reshape(shp)
        o += n
    return out


# ---- torch-backed session (device memory and streams only) -----------------
def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


@dataclass
class DeviceBatch:
    n_cand: int
    open: object
    split_bus: object
    moved_off: object
    moved_br: object
    moved_p: Optional[object]

    @property
    def n_open_slots(self):
        return int(self.open.shape[1])

    @property
    def n_split_slots(self):
        return int(self.split_bus.shape[1])

    def struct(self) -> tto_batch:
        return tto_batch(self.n_cand, self.n_open_slots, self.n_split_slots, _ptr(self.open),
                         _ptr(self.split_bus), _ptr(self.moved_off), _ptr(self.moved_br),
                         _ptr(self.moved_p))


def device_batch(batch, device="cuda") -> DeviceBatch:
    """Copy a gridgen.Batch (numpy) to device tensors."""
    import torch
    op = torch.as_tensor(np.ascontiguousarray(batch.open, dtype=np.int32), device=device)
    sb = torch.as_tensor(np.ascontiguousarray(batch.split_bus, dtype=np.int32), device=device)
    mo = torch.as_tensor(np.ascontiguousarray(batch.moved_off, dtype=np.int32), device=device)
    mb = np.ascontiguousarray(batch.moved_br, dtype=np.int32)
    mbt = torch.as_tensor(mb if mb.size else np.zeros(1, np.int32), device=device)
    mp = None
    if batch.moved_p is not None:
        mp = torch.as_tensor(np.ascontiguousarray(batch.moved_p, dtype=np.float64), device=device)
    return DeviceBatch(int(batch.open.shape[0]), op, sb, mo, mbt, mp)


class Session:
    """Owns the torch-allocated workspaces of one grid and calls the C ABI."""

    def __init__(self, n_bus, from_bus, to_bus, susceptance, limit_mw, ptdf, monitored,
                 contingency, n_timesteps, flow_precision=TTO_FLOW_F32,
                 gemm_precision=TTO_GEMM_F32, max_batch=4096, slack=0, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self._host = dict(
            from_bus=np.ascontiguousarray(from_bus, dtype=np.int32),
            to_bus=np.ascontiguousarray(to_bus, dtype=np.int32),
            b=np.ascontiguousarray(susceptance, dtype=np.float64),
            lim=np.ascontiguousarray(limit_mw, dtype=np.float64),
            mon=np.ascontiguousarray(monitored, dtype=np.int32),
            cont=np.ascontiguousarray(contingency, dtype=np.int32),
        )
        h = self._host
        self.n_bus, self.n_branch, self.T = int(n_bus), len(h["from_bus"]), int(n_timesteps)
        self.nM, self.nC = len(h["mon"]), len(h["cont"])
        self.max_batch = int(max_batch)
        if hasattr(ptdf, "data_ptr") and ptdf.is_cuda:     # e.g. from ptdf_device
            ptdf_t = ptdf.to(torch.float64).contiguous()
        else:
            ptdf_t = torch.as_tensor(np.ascontiguousarray(ptdf, dtype=np.float64),
                                     device=self.device)
        cptr = lambda a: a.ctypes.data
        self.desc = tto_grid_desc(
            self.n_bus, self.n_branch, int(slack), self.T, cptr(h["from_bus"]), cptr(h["to_bus"]),
            cptr(h["b"]), cptr(h["lim"]), _ptr(ptdf_t), self.nM, cptr(h["mon"]), self.nC,
            cptr(h["cont"]) if self.nC else 0, int(flow_precision), int(gemm_precision),
            self.max_batch)
        self.grid_bytes, self.batch_bytes = tto_workspace_bytes(self.desc)
        self.grid_ws = torch.empty(self.grid_bytes, dtype=torch.uint8, device=self.device)
        self.batch_ws = torch.empty(self.batch_bytes, dtype=torch.uint8, device=self.device)
        self.handle = tto_grid_create(self.desc, _ptr(self.grid_ws), self.grid_bytes, self.stream)
        del ptdf_t

    @property
    def stream(self) -> int:
        return int(self.torch.cuda.current_stream(self.device).cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            tto_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_injections(self, P):
        t = P if hasattr(P, "data_ptr") else self.torch.as_tensor(
            np.ascontiguousarray(P, dtype=np.float64), device=self.device)
        self._P = t
        tto_set_injections(self.handle, _ptr(t), self.stream)

    def base_flows(self):
        out = self.torch.empty((self.n_branch, self.T), dtype=self.torch.float64, device=self.device)
        tto_get_base_flows(self.handle, _ptr(out), self.stream)
        return out

    def set_descriptor(self, load_edges, n_count_bins=32, w_c0=200.0, w_c=50.0,
                       kind=TTO_DESC_COUNT_LOAD):
        self._edges = np.ascontiguousarray(load_edges, dtype=np.float64)
        cfg = tto_descriptor_cfg(int(n_count_bins), len(self._edges) + 1,
                                 self._edges.ctypes.data if len(self._edges) else 0,
                                 float(w_c0), float(w_c), int(kind))
        tto_set_descriptor(self.handle, cfg)
        self.n_cells = (TTO_PAPER_CELLS if kind == TTO_DESC_PAPER
                        else int(n_count_bins) * (len(self._edges) + 1))

    def alloc_outputs(self, B, base_flows=False, fmax=False, n1=False):
        torch, d = self.torch, self.device
        o = dict(
            status=torch.empty(B, dtype=torch.uint8, device=d),
            n_island_cont=torch.empty(B, dtype=torch.int32, device=d),
            overload_mw=torch.empty(B, dtype=torch.float64, device=d),
            n_crit_n1=torch.empty(B, dtype=torch.int32, device=d),
            n_crit_n0=torch.empty(B, dtype=torch.int32, device=d),
            max_loading=torch.empty(B, dtype=torch.float64, device=d),
            worst_branch=torch.empty(B, dtype=torch.int32, device=d),
            worst_cont=torch.empty(B, dtype=torch.int32, device=d),
            worst_t=torch.empty(B, dtype=torch.int32, device=d),
            fitness=torch.empty(B, dtype=torch.float64, device=d),
            cell=torch.empty(B, dtype=torch.int32, device=d),
        )
        if base_flows:
            o["base_flows"] = torch.empty((B, self.n_branch, self.T), dtype=torch.float64, device=d)
        if fmax:
            o["fmax"] = torch.empty((B, self.nM, self.T), dtype=torch.float64, device=d)
        if n1:
            o["n1_flows"] = torch.empty((B, self.nC, self.nM, self.T), dtype=torch.float64, device=d)
        return o

    def evaluate(self, dbatch: DeviceBatch, outputs=None, **want):
        if outputs is None:
            outputs = self.alloc_outputs(dbatch.n_cand, **want)
        st = tto_outputs(*[_ptr(outputs.get(f)) for f in OUTPUT_FIELDS])
        tto_evaluate(self.handle, dbatch.struct(), st, _ptr(self.batch_ws), self.batch_bytes,
                     self.stream)
        return outputs

    def autotune(self, dbatch: DeviceBatch, outputs=None, cache_path: str = ""):
        if outputs is None:
            outputs = self.alloc_outputs(dbatch.n_cand)
        st = tto_outputs(*[_ptr(outputs.get(f)) for f in OUTPUT_FIELDS])
        return tto_autotune(self.handle, dbatch.struct(), st, _ptr(self.batch_ws),
                            self.batch_bytes, self.stream, cache_path)

    def capture_evaluate(self, dbatch: DeviceBatch, outputs, archive=None, id_base=0) -> Graph:
        """Graph of evaluate (+ archive insertion) on these buffers."""
        st = tto_outputs(*[_ptr(outputs.get(f)) for f in OUTPUT_FIELDS])
        fit, ids = archive if archive is not None else (None, None)
        h = tto_evaluate_capture(self.handle, dbatch.struct(), st, _ptr(self.batch_ws),
                                 self.batch_bytes, _ptr(fit), _ptr(ids),
                                 int(fit.shape[0]) if fit is not None else 0, id_base)
        return Graph(h)

    def bridges(self):
        """Bridge mask [n_branch] (device uint8) of the grid (tto_bridges)."""
        out = self.torch.empty(self.n_branch, dtype=self.torch.uint8, device=self.device)
        tto_bridges(self.handle, _ptr(out), self.stream)
        return out

    def busbar_set(self, buses, ptdf) -> "BusbarSet":
        return BusbarSet(self, buses, ptdf)

    def busbar_evaluate(self, bset: "BusbarSet", dbatch: DeviceBatch, lambda_b_pre=float("nan"),
                        fitness_f1=None):
        """(lambda_b [B], n_island [B], lambda_f2 [B] or None) of the busbar
        outages (tto_busbar_evaluate) under the installed injections."""
        torch, d = self.torch, self.device
        B = dbatch.n_cand
        lam = torch.empty(B, dtype=torch.float64, device=d)
        nis = torch.empty(B, dtype=torch.int32, device=d)
        f2 = torch.empty(B, dtype=torch.float64, device=d) if fitness_f1 is not None else None
        nb = tto_busbar_bytes(self.handle, bset.handle, B)
        if getattr(self, "_bb_ws", None) is None or self._bb_ws.numel() < nb:
            self._bb_ws = None
            self._bb_ws = torch.empty(nb, dtype=torch.uint8, device=d)
        tto_busbar_evaluate(self.handle, bset.handle, dbatch.struct(), _ptr(self._P),
                            lambda_b_pre, _ptr(fitness_f1), _ptr(lam), _ptr(nis), _ptr(f2),
                            _ptr(self.batch_ws), self.batch_bytes, _ptr(self._bb_ws),
                            self._bb_ws.numel(), self.stream)
        return lam, nis, f2

    def worst_contingencies(self, dbatch: DeviceBatch, k: int = 20):
        """(ids [B][k] int32, energy [B][k] FP64) of the k worst N-1 cases
        per candidate by overload energy (tto_worst_contingencies)."""
        torch, d = self.torch, self.device
        B = dbatch.n_cand
        ids = torch.empty((B, k), dtype=torch.int32, device=d)
        en = torch.empty((B, k), dtype=torch.float64, device=d)
        nb = tto_worst_k_bytes(self.handle, B)
        if getattr(self, "_wk_ws", None) is None or self._wk_ws.numel() < nb:
            self._wk_ws = torch.empty(nb, dtype=torch.uint8, device=d)
        tto_worst_contingencies(self.handle, dbatch.struct(), k, _ptr(ids), _ptr(en),
                                _ptr(self.batch_ws), self.batch_bytes, _ptr(self._wk_ws),
                                self._wk_ws.numel(), self.stream)
        return ids, en

    def set_sweep_plan(self, lanes=256, branches_per_lane=1, order=0, persistent=False):
        tto_set_sweep_plan(self.handle, lanes, branches_per_lane, order, persistent)

    def new_archive(self, n_cells=None):
        n = self.n_cells if n_cells is None else n_cells
        fit = self.torch.full((n,), float("-inf"), dtype=self.torch.float64, device=self.device)
        ids = self.torch.full((n,), -1, dtype=self.torch.int64, device=self.device)
        return fit, ids

    def archive_insert(self, archive, outputs, id_base=0, n_cand=None):
        fit, ids = archive
        B = int(outputs["fitness"].shape[0]) if n_cand is None else n_cand
        tto_archive_insert(self.handle, _ptr(fit), _ptr(ids), int(fit.shape[0]),
                           _ptr(outputs["fitness"]), _ptr(outputs["cell"]),
                           _ptr(outputs["status"]), B, int(id_base), _ptr(self.batch_ws),
                           self.batch_bytes, self.stream)


# ---- MapElites generation on the device -------------------------------------
class GenomeSpace:
    """Torch-held genome tables (tto_genome_space_*) of a Session's grid:
    the split-action set A (bus and moved branches per action), the
    disconnectable set D and the operator parameters."""

    def __init__(self, session: "Session", action_bus, action_moved, disc_branch,
                 n_action_slots: int, n_disc_slots: int, mut_mean=2.0,
                 w_action=(20, 20, 50, 10), w_disc=(25, 25, 50, 0), p_c1=0.5):
        torch = session.torch
        self.session = session
        bus = np.ascontiguousarray(action_bus, dtype=np.int32)
        off = np.zeros(len(bus) + 1, dtype=np.int32)
        off[1:] = np.cumsum([len(m) for m in action_moved]) if len(bus) else []
        br = np.ascontiguousarray(
            np.concatenate([np.asarray(m, dtype=np.int32) for m in action_moved])
            if len(bus) else np.zeros(1, np.int32), dtype=np.int32)
        disc = np.ascontiguousarray(disc_branch, dtype=np.int32)
        if disc.size == 0:
            disc = np.zeros(1, np.int32)[:0]
        self._host = (bus, off, br, disc)
        self.desc = tto_genome_desc(
            int(n_action_slots), int(n_disc_slots), len(bus), bus.ctypes.data if len(bus) else 0,
            off.ctypes.data, br.ctypes.data, len(disc), disc.ctypes.data if len(disc) else 0,
            float(mut_mean), (_i32 * 4)(*w_action), (_i32 * 4)(*w_disc), float(p_c1))
        n = tto_genome_space_bytes(self.desc)
        self.ws = torch.empty(max(n, 256), dtype=torch.uint8, device=session.device)
        self.handle = tto_genome_space_create(session.handle, self.desc, _ptr(self.ws), n,
                                              session.stream)
        self.n_a, self.n_d = int(n_action_slots), int(n_disc_slots)
        self.G = self.n_a + self.n_d
        self.max_moved = tto_genome_max_moved(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            tto_genome_space_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def vary(self, rep: "Repertoire", seed: int, n_child: int, children=None, b_mc=None):
        torch, s = self.session.torch, self.session
        if children is None:
            children = torch.empty((n_child, max(self.G, 1)), dtype=torch.int32, device=s.device)
        if b_mc is None:
            b_mc = torch.empty(1, dtype=torch.int32, device=s.device)
        tto_vary(self.handle, _ptr(rep.id), _ptr(rep.genome), rep.n_cells, seed,
                 _ptr(rep.generation), n_child, _ptr(children), _ptr(b_mc), s.stream)
        return children, b_mc

    def expand(self, genomes, n: Optional[int] = None) -> "DeviceBatch":
        torch, s = self.session.torch, self.session
        n = int(genomes.shape[0]) if n is None else n
        d = s.device
        op = torch.empty((n, self.n_d), dtype=torch.int32, device=d)
        sb = torch.empty((n, self.n_a), dtype=torch.int32, device=d)
        mo = torch.empty(n * self.n_a + 1, dtype=torch.int32, device=d)
        cap = max(1, n * self.max_moved)
        mb = torch.empty(cap, dtype=torch.int32, device=d)
        tto_genome_expand(self.handle, _ptr(genomes), n, _ptr(op) if self.n_d else 0,
                          _ptr(sb) if self.n_a else 0, _ptr(mo) if self.n_a else 0,
                          _ptr(mb) if self.n_a else 0, cap, s.stream)
        return DeviceBatch(n, op, sb, mo, mb, None)


class Repertoire:
    """Device repertoire (tto_repertoire): per cell fitness, id and genome,
    plus the generation counter."""

    def __init__(self, session: "Session", gs: GenomeSpace, n_cells: Optional[int] = None):
        torch, d = session.torch, session.device
        n = session.n_cells if n_cells is None else int(n_cells)
        self.n_cells = n
        self.fitness = torch.full((n,), float("-inf"), dtype=torch.float64, device=d)
        self.id = torch.full((n,), -1, dtype=torch.int64, device=d)
        self.genome = torch.full((n, max(gs.G, 1)), -1, dtype=torch.int32, device=d)
        self.generation = torch.zeros(1, dtype=torch.int64, device=d)

    def struct(self) -> tto_repertoire:
        return tto_repertoire(self.n_cells, _ptr(self.fitness), _ptr(self.id), _ptr(self.genome),
                              _ptr(self.generation))


class Evolver:
    """One device generation per call (tto_generation) on pre-allocated
    buffers, so that calls can be captured in a Graph and replayed."""

    def __init__(self, session: "Session", gs: GenomeSpace, rep: Repertoire, n_child: int,
                 seed: int, outputs=None):
        torch = session.torch
        self.session, self.gs, self.rep = session, gs, rep
        self.n_child, self.seed = int(n_child), int(seed)
        self.gen_bytes = tto_generation_bytes(session.handle, gs.handle, self.n_child)
        self.gen_ws = torch.empty(self.gen_bytes, dtype=torch.uint8, device=session.device)
        self.outputs = outputs
        self._rep_struct = rep.struct()
        self._out_struct = (tto_outputs(*[_ptr(outputs.get(f)) for f in OUTPUT_FIELDS])
                            if outputs is not None else None)
        G = gs.G
        self.children = self.gen_ws[: 4 * self.n_child * G].view(torch.int32).view(self.n_child, G)
        off = (4 * self.n_child * G + 255) // 256 * 256
        self.b_mc = self.gen_ws[off: off + 4].view(torch.int32)

    def step(self):
        s = self.session
        tto_generation(s.handle, self.gs.handle, self._rep_struct, self.seed, self.n_child,
                       self._out_struct, _ptr(self.gen_ws), self.gen_bytes, _ptr(s.batch_ws),
                       s.batch_bytes, s.stream)


class ScreenedEvolver:
    """One screened device generation per call (tto_screened_generation):
    n_child children varied, scored by the network `net`, the n_keep most
    promising evaluated exactly and inserted.  Buffers are pre-allocated, so
    calls can be captured in a Graph and replayed.  `dense_row` is the
    device FP32 [d_dense] injection summary of the current injections."""

    def __init__(self, session: "Session", gs: GenomeSpace, rep: Repertoire, net: "Surrogate",
                 n_child: int, n_keep: int, seed: int, dense_row=None, outputs=None,
                 rule: int = 0, y_mu=(0.0, 0.0), y_sd=(1.0, 1.0), ref=(0.0, 0.0),
                 overload_scale_mw: float = 100.0):
        torch = session.torch
        self.cfg = tto_screen_cfg(int(rule), (ct.c_double * 2)(*y_mu), (ct.c_double * 2)(*y_sd),
                                  (ct.c_double * 2)(*ref), float(overload_scale_mw))
        self.session, self.gs, self.rep, self.net = session, gs, rep, net
        self.n_child, self.n_keep, self.seed = int(n_child), int(n_keep), int(seed)
        self.gen_bytes = tto_screened_generation_bytes(session.handle, gs.handle, net.handle,
                                                       self.n_child, self.n_keep)
        self.gen_ws = torch.empty(self.gen_bytes, dtype=torch.uint8, device=session.device)
        d = int(net.desc.d_dense)
        self.dense_row = torch.zeros(max(d, 1), dtype=torch.float32, device=session.device)
        if dense_row is not None:
            self.set_dense_row(dense_row)
        self.outputs = outputs
        self._rep_struct = rep.struct()
        self._out_struct = (tto_outputs(*[_ptr(outputs.get(f)) for f in OUTPUT_FIELDS])
                            if outputs is not None else None)
        G = gs.G
        self.children = self.gen_ws[: 4 * self.n_child * G].view(torch.int32).view(self.n_child, G)
        self.kept = torch.empty(self.n_keep, dtype=torch.int32, device=session.device)

    def set_dense_row(self, row):
        """Copy a new injection summary into the buffer the calls read."""
        t = self.session.torch.as_tensor(np.ascontiguousarray(row, dtype=np.float32),
                                         device=self.session.device)
        self.dense_row[: t.numel()].copy_(t)

    def step(self):
        s = self.session
        tto_screened_generation(s.handle, self.gs.handle, self._rep_struct, self.net.handle,
                                _ptr(self.dense_row), self.cfg, self.seed, self.n_child,
                                self.n_keep, self._out_struct, _ptr(self.kept),
                                _ptr(self.gen_ws), self.gen_bytes,
                                _ptr(self.net.bws), self.net.bbytes, _ptr(s.batch_ws),
                                s.batch_bytes, s.stream)


class BusbarSet:
    """Device busbar outage set O_b of a Session's grid (tto_busbar_set_*)."""

    def __init__(self, session: "Session", buses, ptdf):
        torch = session.torch
        self.buses = np.ascontiguousarray(buses, dtype=np.int32)
        pt = ptdf if hasattr(ptdf, "data_ptr") else torch.as_tensor(
            np.ascontiguousarray(ptdf, dtype=np.float64), device=session.device)
        n = tto_busbar_set_bytes(session.handle, len(self.buses))
        self.ws = torch.empty(n, dtype=torch.uint8, device=session.device)
        self.handle = tto_busbar_set_create(session.handle, len(self.buses),
                                            self.buses.ctypes.data if len(self.buses) else 0,
                                            _ptr(pt), _ptr(self.ws), n, session.stream)

    def close(self):
        if getattr(self, "handle", None):
            tto_busbar_set_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
