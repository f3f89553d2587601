"""Write the oracle fixtures of the large parity cases (calls only `oracle/`
for values and `gridgen/` for the seeded inputs).

    python tests/golden/make_fixtures.py [batch|precision|plain|all] [--procs N]

batch      2000 buses / 3200 branches, T = 24, |M| = 1200, |C| = 1600, the
           16384-candidate workload: 17 candidates, two per rank 1..8 (one
           with splits, one without where the rank allows) plus rank 0.
precision  6000 buses / 9500 branches, T = 24, |M| = 2000, |C| = 3000: four
           candidates of ranks 2, 4, 6, 8 with splits.
plain      500 buses / 800 branches, T = 1, all 4096 candidates (f^max kept for
           the first 64).

Per candidate (Fitness function heuristics, every contingency re-solved from
scratch in FP64): validity, islanding, the metrics lambda_o, lambda_c,
lambda_c0, max loading and its arg-max (e*, t*, l*), the count of islanding
contingencies, fitness lambda_f1 and the descriptor cell; f^max (FP64, so
that the FP64 flow tolerance of 1e-6 MW can be applied to it); and the
distances of each
discrete decision from its threshold in FP64, so that a test knows where a
decision is unique at a given flow tolerance:
  margin0   min over monitored (e, t) of ||f'_e(t)| - fbar_e|   (lambda_c0)
  gap       largest minus second largest f^max_e(t) / fbar_e   (e*, t*)
  edge_dist distance of the max loading to the nearest load edge (cell)
  cut_dist  min over non-islanding l of ||f^(l)_e*(t*)| - cut|, cut = the
            maximum minus the worst-contingency tie band (l*)
  worst_col |f^(l)_e*(t*)| over C (NaN where l islands; batch and precision)
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import gridgen as gg          # noqa: E402
import oracle                 # noqa: E402
from oracle.dcflow import WORST_CONT_TIE_MW, candidate_from_batch  # noqa: E402

FILES = {"batch": "oracle_batch_2000bus.npz", "precision": "oracle_precision_6000bus.npz",
         "plain": "oracle_plain_500bus.npz"}
CFG = {"batch": 3, "precision": 4, "plain": 2}


def pick_batch_candidates(batch) -> list:
    """Rank 0 once, then per rank 1..8 the first candidate with splits and
    the first without (encoding only, no evaluation)."""
    r = (batch.open != -1).sum(1) + (batch.split_bus != -1).sum(1)
    s = (batch.split_bus != -1).sum(1)
    out = [int(np.flatnonzero(r == 0)[0])]
    for rank in range(1, 9):
        for want_split in (True, False):
            hit = np.flatnonzero((r == rank) & ((s > 0) == want_split))
            if hit.size:
                out.append(int(hit[0]))
    return out


def pick_precision_candidates(batch) -> list:
    r = (batch.open != -1).sum(1) + (batch.split_bus != -1).sum(1)
    s = (batch.split_bus != -1).sum(1)
    return [int(np.flatnonzero((r == rank) & (s > 0))[0]) for rank in (2, 4, 6, 8)]


_W = None


def _init(cfg):
    from threadpoolctl import threadpool_limits
    global _W, _LIM
    _W = gg.build_config(cfg)
    _LIM = threadpool_limits(1)


def _one(args):
    c, keep_col = args
    w = _W
    edges = gg.default_load_edges()
    cand = candidate_from_batch(w.batch, c)
    r = oracle.evaluate_candidate(w.grid, w.P, w.M, w.C, cand, edges, keep_n1=True)
    rec = dict(idx=c, valid=r.valid, islanded=r.islanded)
    if not r.valid or r.islanded:
        return rec
    met = r.metrics
    lim = np.asarray(w.grid.limit_mw, np.float64)[w.M]
    f0M = r.base_flows[w.M]
    ratio = (r.fmax / lim[:, None]).ravel()
    top = np.sort(ratio)[::-1]
    rho = met["max_loading"]
    rec.update(
        n_island_cont=met["n_island_cont"], overload_mw=met["overload_mw"],
        n_crit_n1=met["n_crit_n1"], n_crit_n0=met["n_crit_n0"], max_loading=rho,
        worst_branch=met.get("worst_branch", -1), worst_t=met.get("worst_t", -1),
        worst_cont=met.get("worst_cont", -1), fitness=r.fitness, cell=r.cell,
        fmax=np.asarray(r.fmax, np.float64),
        margin0=float(np.abs(np.abs(f0M) - lim[:, None]).min()),
        gap=float(top[0] - top[1]) if top.size > 1 else np.inf,
        edge_dist=float(np.abs(edges - rho).min()),
    )
    if met["worst"] is None:           # every contingency islands
        rec["cut_dist"] = np.inf
        return rec
    e_i, t_i, _ = met["worst"]
    col = np.abs(r.n1_flows[:, e_i, t_i])
    cut = r.fmax[e_i, t_i] - WORST_CONT_TIE_MW
    fin = np.isfinite(col)
    rec["cut_dist"] = float(np.abs(col[fin] - cut).min()) if fin.any() else np.inf
    if keep_col:
        rec["worst_col"] = col
    return rec


SCALARS_I = ["idx", "valid", "islanded", "n_island_cont", "n_crit_n1", "n_crit_n0",
             "worst_branch", "worst_t", "worst_cont", "cell"]
SCALARS_F = ["overload_mw", "max_loading", "fitness", "margin0", "gap", "edge_dist", "cut_dist"]


def write(kind: str, procs: int):
    import multiprocessing as mp
    cfg = CFG[kind]
    w = gg.build_config(cfg)
    if kind == "batch":
        idx = pick_batch_candidates(w.batch)
    elif kind == "precision":
        idx = pick_precision_candidates(w.batch)
    else:
        idx = list(range(w.batch.n_cand))
    keep_col = kind != "plain"
    n_fmax = len(idx) if kind != "plain" else 64
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs, initializer=_init, initargs=(cfg,)) as pool:
        recs = pool.map(_one, [(c, keep_col) for c in idx], chunksize=1)
    dt = time.perf_counter() - t0
    n = len(recs)
    out = {}
    for k in SCALARS_I:
        out[k] = np.array([int(q.get(k, -1)) for q in recs], np.int64)
    for k in SCALARS_F:
        out[k] = np.array([float(q.get(k, np.nan)) for q in recs], np.float64)
    nM, T, nC = len(w.M), w.P.shape[1], len(w.C)
    fm = np.full((n_fmax, nM, T), np.nan, np.float64)
    for i in range(n_fmax):
        if "fmax" in recs[i]:
            fm[i] = recs[i]["fmax"]
    out["fmax"] = fm
    if keep_col:
        wc = np.full((n, nC), np.nan)
        for i in range(n):
            if "worst_col" in recs[i]:
                wc[i] = recs[i]["worst_col"]
        out["worst_col"] = wc
    out["meta"] = np.array([f"config={cfg} n_bus={w.grid.n_bus} n_branch={w.grid.n_branch} "
                            f"T={T} nM={nM} nC={nC} B={w.batch.n_cand} "
                            f"tie_mw={WORST_CONT_TIE_MW} written by tests/golden/make_fixtures.py "
                            f"{kind} (oracle re-solves, {dt:.0f} s on {procs} processes)"])
    path = os.path.join(HERE, FILES[kind])
    np.savez_compressed(path, **out)
    print(f"{kind}: {n} candidates in {dt:.0f} s -> {path} ({os.path.getsize(path) / 1e6:.2f} MB)",
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="?", default="all", choices=["batch", "precision", "plain", "all"])
    ap.add_argument("--procs", type=int, default=min(8, os.cpu_count() or 1))
    a = ap.parse_args()
    for kind in (["plain", "batch", "precision"] if a.which == "all" else [a.which]):
        write(kind, a.procs)


if __name__ == "__main__":
    main()
