"""Congestion metrics, fitness, descriptor cell and elite archive (oracle; test
infrastructure only).  FP64, written straight from the definitions."""
from __future__ import annotations

from typing import Optional

import numpy as np

# Relative band within which two loadings count as tied for the worst
# (branch, timestep): far above FP64 rounding of a flow, far below any
# loading difference that is not a tie.
LOAD_TIE_REL = 1e-9


def n1_metrics(fmax: np.ndarray, f0: np.ndarray, limit: np.ndarray,
               argl: Optional[np.ndarray] = None) -> dict:
    """Fitness function heuristics section: with f^max_e = max over outages of
    |f^(o)_e| and the clip Pi(x) = max(x, 0),

      lambda_o  = sum_e Pi(f^max_e - fbar_e)      (N-1 overload energy)
      lambda_c  = sum_e 1(f^max_e > fbar_e)       (N-1 critical branches, strict)
      lambda_c0 = sum_e 1(|f^n0_e| > fbar_e)      (N-0 critical branches, strict)

    Multi-timestep reading: sums run over timesteps as well; the maximum
    loading rho = max_{e,t} f^max_e(t) / fbar_e.  (e*, t*) is the
    lexicographically smallest pair whose loading is at least
    rho (1 - LOAD_TIE_REL): loadings that are equal in exact arithmetic (the
    two branches of a two-branch cut with equal limits each carry the cut's
    whole transfer when the other is out) differ only by rounding, and the
    band lets the order, not the rounding, decide.  The third entry of
    "worst" is argl[e*, t*] when argl is given (the candidate evaluation fills
    in the worst contingency by its own rule).

    fmax, f0: [|M|, T]; limit: [|M|]; argl: [|M|, T] positions in C, or None.
    """
    lim = limit[:, None]
    over = np.maximum(fmax - lim, 0.0)
    res = {
        "overload_mw": float(over.sum()),
        "n_crit_n1": int((fmax > lim).sum()),
        "n_crit_n0": int((np.abs(f0) > lim).sum()),
    }
    ratio = fmax / lim
    res["max_loading"] = float(ratio.max()) if ratio.size else 0.0
    res["worst"] = None
    if ratio.size:
        best = res["max_loading"]
        thr = best * (1.0 - LOAD_TIE_REL)
        E, T = ratio.shape
        found = None
        for e in range(E):
            for t in range(T):
                if ratio[e, t] >= thr:
                    found = (e, t)
                    break
            if found is not None:
                break
        e, t = found
        res["worst"] = (e, t, int(argl[e, t]) if argl is not None else -1)
    return res


def fitness_f1(overload_mw: float, n_crit_n0: int, n_crit_n1: int,
               w_c0: float = 200.0, w_c: float = 50.0) -> float:
    """High-level loop section: lambda_f1 = -(lambda_o + 200 lambda_c0 + 50 lambda_c),
    maximised."""
    return -(overload_mw + w_c0 * n_crit_n0 + w_c * n_crit_n1)


def descriptor_cell(n_switched: int, max_loading: float, load_edges: np.ndarray,
                    n_count_bins: int = 32) -> int:
    """Two-axis MapElites cell: (number of switched elements, max-loading bin).

    count axis: min(k + s, n_count_bins - 1) (each opening and each split counts 1);
    load axis:  number of edges <= rho (edges ascending), so n_load_bins =
                len(load_edges) + 1 bins with clamping at both ends.
    """
    n_load_bins = len(load_edges) + 1
    count = min(int(n_switched), n_count_bins - 1)
    b = 0
    for edge in load_edges:
        if edge <= max_loading:
            b += 1
    return count * n_load_bins + b


def descriptor_cell_paper(n_open: int, n_split: int, n_moved: int) -> int:
    """Repertoire design, the paper's map: lambda_d (disconnections, 0..2),
    lambda_s (splits, 0..3), lambda_r (reassigned assets, 0..45), each
    clamped; beta = lambda_d + 3 (lambda_s + 4 lambda_r) (reading of the
    garbled printed coefficient: it maps the three ranges one to one onto
    0..551)."""
    ld, ls, lr = min(n_open, 2), min(n_split, 3), min(n_moved, 45)
    return ld + 3 * (ls + 4 * lr)


def archive_insert_sequential(best_fit: np.ndarray, best_id: np.ndarray, fitness, cells,
                              ok, id_base: int = 0):
    """Unbatched insertion (High-level loop): candidates are offered one at a time
    in batch order; each cell keeps one elite, replaced only by a strictly
    better fitness.  Empty cells have best_id == -1.  Islanded or invalid
    candidates (ok == False) never enter."""
    best_fit = np.array(best_fit, dtype=np.float64, copy=True)
    best_id = np.array(best_id, dtype=np.int64, copy=True)
    for i in range(len(fitness)):
        if not ok[i]:
            continue
        c = int(cells[i])
        if best_id[c] == -1 or fitness[i] > best_fit[c]:
            best_fit[c] = fitness[i]
            best_id[c] = id_base + i
    return best_fit, best_id


def contingency_energies(n1_flows: np.ndarray, limit: np.ndarray) -> np.ndarray:
    """Overload energy of every N-1 case on its own (AC-Validator section:
    the worst-k filter): E_l = sum_{e,t} max(|f^(l)_e(t)| - fbar_e, 0).
    n1_flows [|C|, |M|, T] with NaN rows for islanding contingencies (their
    E_l is NaN); limit [|M|]."""
    n1 = np.asarray(n1_flows, dtype=np.float64)
    out = np.full(n1.shape[0], np.nan)
    for li in range(n1.shape[0]):
        if np.isnan(n1[li]).any():
            continue
        out[li] = float(np.maximum(np.abs(n1[li]) - limit[:, None], 0.0).sum())
    return out


def worst_k(energies: np.ndarray, C, k: int):
    """The k largest energies, descending, ties to the earlier entry of C;
    islanding (NaN) entries excluded; padded with (-1, NaN)."""
    order = sorted((li for li in range(len(energies)) if not np.isnan(energies[li])),
                   key=lambda li: (-energies[li], li))[:k]
    ids = [int(C[li]) for li in order] + [-1] * (k - len(order))
    en = [float(energies[li]) for li in order] + [float("nan")] * (k - len(order))
    return np.array(ids, dtype=np.int64), np.array(en)
