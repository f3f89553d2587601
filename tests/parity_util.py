"""Helpers for GPU-vs-oracle parity tests (imported by test modules only)."""
from __future__ import annotations

import os
import sys

import numpy as np

import gridgen as gg

# Stated flow tolerances (MW) of the two flow precisions.
TOL_F64 = 1e-6
TOL_F32 = 1e-2


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def make_session(w, flow_prec, gemm_prec=None, max_batch=None, edges=None):
    from paper_2605_10128_amd import tto
    grid = w.grid
    b = 1.0 / grid.x_pu
    if gemm_prec is None:
        gemm_prec = tto.TTO_GEMM_F64 if flow_prec == tto.TTO_FLOW_F64 else tto.TTO_GEMM_F32
    ptdf = tto.ptdf_device(grid.n_bus, grid.from_bus, grid.to_bus, b, grid.slack)
    s = tto.Session(grid.n_bus, grid.from_bus, grid.to_bus, b, grid.limit_mw, ptdf, w.M, w.C,
                    w.P.shape[1], flow_precision=flow_prec, gemm_precision=gemm_prec,
                    max_batch=max_batch or w.batch.n_cand, slack=grid.slack)
    s.set_injections(w.P)
    s.set_descriptor(gg.default_load_edges() if edges is None else edges)
    return s


def to_numpy(out: dict) -> dict:
    return {k: v.detach().cpu().numpy() for k, v in out.items()}


def oracle_results(w, idx, keep_n1=True, processes=None, edges=None):
    import oracle
    if processes is None:
        processes = min(8, max(1, len(idx)), os.cpu_count() or 1)
    return oracle.evaluate_batch(w.grid, w.P, w.M, w.C, w.batch,
                                 gg.default_load_edges() if edges is None else edges,
                                 idx=idx, processes=processes, keep_n1=keep_n1)


def compare(w, gpu: dict, idx, ores, tol: float, edges=None, strict_discrete=False,
            decision_tol=None):
    """Compare GPU outputs with oracle results on candidates idx.

    Continuous values within `tol` MW; integers and cells exactly, except
    where the oracle itself sits within `decision_tol` MW (default `tol`) of
    the decision (then the GPU value must be one of the valid answers).  The
    FP32 path with FP64 refinement takes its discrete decisions in FP64, so
    its tests pass a decision_tol of FP64 size.  Returns counters.
    """
    dtol = tol if decision_tol is None else decision_tol
    edges = gg.default_load_edges() if edges is None else edges
    lim = w.grid.limit_mw[w.M]
    stats = dict(checked=0, near=0)
    for k, c in enumerate(idx):
        r = ores[k]
        st = int(gpu["status"][c])
        if not r.valid:
            assert st & 2, f"cand {c}: oracle invalid, gpu status {st}"
            continue
        if r.islanded:
            assert st & 1, f"cand {c}: oracle islanded, gpu status {st}"
            assert gpu["cell"][c] == -1 and gpu["fitness"][c] == -np.inf
            continue
        assert st & 3 == 0, f"cand {c}: gpu status {st} but oracle connected"
        stats["checked"] += 1
        met = r.metrics
        assert gpu["n_island_cont"][c] == met["n_island_cont"], c
        if "base_flows" in gpu:
            np.testing.assert_allclose(gpu["base_flows"][c], r.base_flows, atol=tol, rtol=0,
                                       err_msg=f"base flows cand {c}")
        if "fmax" in gpu:
            np.testing.assert_allclose(gpu["fmax"][c], r.fmax, atol=tol, rtol=0,
                                       err_msg=f"fmax cand {c}")
        if "n1_flows" in gpu and r.n1_flows is not None:
            a, b = gpu["n1_flows"][c], r.n1_flows
            assert np.array_equal(np.isnan(a), np.isnan(b)), f"n1 NaN pattern cand {c}"
            np.testing.assert_allclose(np.nan_to_num(a), np.nan_to_num(b), atol=tol, rtol=0,
                                       err_msg=f"n1 flows cand {c}")
        # lambda_c0 comes from FP64 post-switch flows in every mode
        f0M = r.base_flows[w.M]
        margin0 = np.abs(np.abs(f0M) - lim[:, None]).min()
        if margin0 > 1e-9 or strict_discrete:
            assert gpu["n_crit_n0"][c] == met["n_crit_n0"], c
        # lambda_c and lambda_o
        margin = np.abs(r.fmax - lim[:, None]).min()
        n_over = int((r.fmax > lim[:, None] - tol).sum())
        assert abs(gpu["overload_mw"][c] - met["overload_mw"]) <= tol * (n_over + 1), c
        near_c = margin <= tol
        if near_c and not strict_discrete:
            stats["near"] += 1
            lo = int((r.fmax > lim[:, None] + tol).sum())
            hi = int((r.fmax > lim[:, None] - tol).sum())
            assert lo <= gpu["n_crit_n1"][c] <= hi, c
        else:
            assert gpu["n_crit_n1"][c] == met["n_crit_n1"], c
        # max loading, arg-max branch/timestep
        rho = met["max_loading"]
        assert abs(gpu["max_loading"][c] - rho) <= tol / lim.min() + 1e-12, c
        ratio = r.fmax / lim[:, None]
        top = np.sort(ratio.ravel())[::-1]
        gap = top[0] - top[1] if top.size > 1 else np.inf
        rtol_ratio = dtol / lim.min()
        if gap > 2 * rtol_ratio or strict_discrete:
            assert gpu["worst_branch"][c] == met["worst_branch"], c
            assert gpu["worst_t"][c] == met["worst_t"], c
        else:
            stats["near"] += 1
            e_pos = int(np.flatnonzero(w.M == gpu["worst_branch"][c])[0])
            assert ratio[e_pos, gpu["worst_t"][c]] >= top[0] - 2 * rtol_ratio, c
        # worst contingency: the first entry of C within the tie tolerance of
        # the maximum |flow| at (e*, t*); unique unless a flow sits within the
        # decision tolerance of that cut, else any choice consistent with the
        # cut (first above it, none before it) is valid
        if r.n1_flows is not None and met["worst_cont"] >= 0:
            import oracle
            e_pos = int(np.flatnonzero(w.M == gpu["worst_branch"][c])[0])
            t_ = int(gpu["worst_t"][c])
            col = np.abs(r.n1_flows[:, e_pos, t_])
            col = np.where(np.isnan(col), -np.inf, col)
            cut = col.max() - oracle.dcflow.WORST_CONT_TIE_MW
            l_pos = int(np.flatnonzero(w.C == gpu["worst_cont"][c])[0])
            fin = np.isfinite(col)
            ambiguous = bool(np.any(np.abs(col[fin] - cut) <= 2 * dtol))
            if not ambiguous and gpu["worst_branch"][c] == met["worst_branch"] and \
                    t_ == met["worst_t"]:
                assert gpu["worst_cont"][c] == met["worst_cont"], c
            else:
                stats["near"] += 1
                assert col[l_pos] >= cut - 2 * tol, c
                assert np.all(col[:l_pos] < cut + 2 * tol), c
        # fitness and cell
        fit_tol = tol * (n_over + 1) + (50.0 * abs(int(gpu["n_crit_n1"][c]) - met["n_crit_n1"]))
        assert abs(gpu["fitness"][c] - r.fitness) <= fit_tol + 1e-9, c
        near_edge = np.abs(edges - rho).min() <= dtol / lim.min() if len(edges) else False
        if near_edge and not strict_discrete:
            stats["near"] += 1
            assert gpu["cell"][c] // (len(edges) + 1) == r.cell // (len(edges) + 1), c
        else:
            assert gpu["cell"][c] == r.cell, c
    return stats
