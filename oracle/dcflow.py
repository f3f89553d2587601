"""FP64 DC power flow by from-scratch re-solves (oracle; test infrastructure only).

DC model (reading of the Importer / DC-Optimizer sections, which linearise the
grid but do not print the equations): lossless branches with susceptance
b_e = 1 / x_e, no shunts, phase shifters or HVDC; nodal balance
sum_{e out of i} f_e - sum_{e into i} f_e = P_i; the slack bus has angle 0.

Bus split (switching actions, "two-node operation"): the split bus keeps
busbar A (and the slack role if it is the slack); a new busbar B receives the
moved branches and the moved part of the injection.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.sparse import csgraph

from .metrics import n1_metrics, fitness_f1, descriptor_cell, descriptor_cell_paper

MAX_RANK = 8
# Encoding limit: moved branches summed over one candidate's splits.
MAX_MOVED = 64
# Worst contingency reading: flows within this many MW of the maximum at
# (e*, t*) count as tied and the order of the contingency list decides
# (branches that no outage affects, such as bridges, tie exactly).
WORST_CONT_TIE_MW = 0.05


@dataclass
class Candidate:
    opened: List[int]                       # branch ids (non-empty slots, slot order)
    splits: List[Tuple[int, List[int]]]     # (bus, moved branch ids), slot order
    moved_p: List[Optional[np.ndarray]]     # per split: [T] MW moved to busbar B or None
    n_slots_filled: int = 0


def candidate_from_batch(batch, c: int) -> Candidate:
    opened = [int(v) for v in batch.open[c].tolist() if v != -1]
    splits, mps = [], []
    ns = batch.split_bus.shape[1]
    for j in range(ns):
        bus = int(batch.split_bus[c, j])
        if bus == -1:
            continue
        splits.append((bus, [int(v) for v in batch.moved(c, j).tolist()]))
        mps.append(None if batch.moved_p is None else np.asarray(batch.moved_p[c * ns + j], dtype=np.float64))
    return Candidate(opened=opened, splits=splits, moved_p=mps,
                     n_slots_filled=len(opened) + len(splits))


def validate_candidate(n_bus: int, from_bus, to_bus, cand: Candidate) -> bool:
    """Structural validity rules of the candidate encoding.

    Valid iff: opened ids in range and distinct; split buses in range and
    distinct; every split moves a non-empty list of distinct branches that are
    incident to its bus; no moved branch is also opened; rank (filled slots)
    at most 8; at most 64 moved branches over all splits.  (Genome of the
    Repertoire design section: distinct substations, distinct branches.)  A
    branch may be moved by the splits at both of its ends.
    """
    m = len(from_bus)
    if len(cand.opened) + len(cand.splits) > MAX_RANK:
        return False
    if sum(len(mv) for _, mv in cand.splits) > MAX_MOVED:
        return False
    if any(e < 0 or e >= m for e in cand.opened):
        return False
    if len(set(cand.opened)) != len(cand.opened):
        return False
    buses = [b for b, _ in cand.splits]
    if any(b < 0 or b >= n_bus for b in buses):
        return False
    if len(set(buses)) != len(buses):
        return False
    opened = set(cand.opened)
    for bus, moved in cand.splits:
        if len(moved) == 0 or len(set(moved)) != len(moved):
            return False
        for e in moved:
            if e < 0 or e >= m:
                return False
            if int(from_bus[e]) != bus and int(to_bus[e]) != bus:
                return False
            if e in opened:
                return False
    return True


@dataclass
class Network:
    n_node: int              # buses + new busbars
    fr: np.ndarray           # per original branch: from node after switching
    to: np.ndarray           # per original branch: to node after switching
    b: np.ndarray            # susceptance per branch
    in_service: np.ndarray   # bool per branch
    P: np.ndarray            # [n_node, T] injections
    slack: int


def post_switch_network(n_bus: int, from_bus, to_bus, b, slack: int, P: np.ndarray,
                        cand: Candidate) -> Network:
    """Step 1 of the definition: apply openings and bus splits."""
    fr = np.asarray(from_bus, dtype=np.int64).copy()
    to = np.asarray(to_bus, dtype=np.int64).copy()
    m = len(fr)
    T = P.shape[1]
    n_node = n_bus + len(cand.splits)
    Pn = np.zeros((n_node, T), dtype=np.float64)
    Pn[:n_bus] = P
    for j, (bus, moved) in enumerate(cand.splits):
        new = n_bus + j
        for e in moved:
            if fr[e] == bus:
                fr[e] = new
            if to[e] == bus:
                to[e] = new
        mp = cand.moved_p[j] if j < len(cand.moved_p) else None
        if mp is not None:
            Pn[new] += mp
            Pn[bus] -= mp
    ins = np.ones(m, dtype=bool)
    for e in cand.opened:
        ins[e] = False
    return Network(n_node=n_node, fr=fr, to=to, b=np.asarray(b, dtype=np.float64),
                   in_service=ins, P=Pn, slack=slack)


def is_connected(n_node: int, fr, to, in_service) -> bool:
    """True iff the in-service branches join all nodes into one component
    (library connected-components routine on the undirected graph).

    Islanding is a property of the post-switch graph over every node (the
    buses and the split buses' busbars B): a node left without an in-service
    branch is an island of its own whatever its injection, as the paper's
    importer decides islands from the graph (bridges) alone."""
    idx = np.flatnonzero(in_service)
    if n_node <= 1:
        return True
    g = sp.csr_matrix((np.ones(len(idx)), (np.asarray(fr)[idx], np.asarray(to)[idx])),
                      shape=(n_node, n_node))
    n_comp = csgraph.connected_components(g, directed=False, return_labels=False)
    return int(n_comp) == 1


def solve_flows(n_node: int, fr, to, b, in_service, P: np.ndarray, slack: int) -> np.ndarray:
    """Assemble B' (nodal susceptance matrix without the slack row/column), solve
    B' theta = P for all timesteps (sparse LU, a library primitive), return
    branch flows [m, T] (0 for branches out of service)."""
    idx = np.flatnonzero(in_service)
    f_n, t_n, bb = np.asarray(fr)[idx], np.asarray(to)[idx], np.asarray(b)[idx]
    rows = np.concatenate([f_n, t_n, f_n, t_n])
    cols = np.concatenate([f_n, t_n, t_n, f_n])
    vals = np.concatenate([bb, bb, -bb, -bb])
    keep = (rows != slack) & (cols != slack)
    red = lambda v: v - (v > slack)          # node id -> row/column of B'
    Bred = sp.csc_matrix((vals[keep], (red(rows[keep]), red(cols[keep]))),
                         shape=(n_node - 1, n_node - 1))
    theta = np.zeros((n_node, P.shape[1]), dtype=np.float64)
    if n_node > 1:
        lu = spla.splu(Bred, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                       options=dict(SymmetricMode=True))
        others = np.arange(n_node) != slack
        theta[others] = lu.solve(np.ascontiguousarray(P[others]))
    flows = np.zeros((len(fr), P.shape[1]), dtype=np.float64)
    flows[idx] = bb[:, None] * (theta[f_n] - theta[t_n])
    return flows


@dataclass
class CandidateResult:
    valid: bool
    islanded: bool
    base_flows: Optional[np.ndarray] = None     # [m, T] post-switch N-0 flows
    n1_flows: Optional[np.ndarray] = None       # [|C|, |M|, T]; NaN rows for islanding l
    fmax: Optional[np.ndarray] = None           # [|M|, T]
    island_cont: Optional[np.ndarray] = None    # bool [|C|]
    metrics: dict = field(default_factory=dict)
    fitness: float = float("-inf")
    cell: int = -1
    n_switched: int = 0
    nonfinite: bool = False


def evaluate_candidate(grid, P: np.ndarray, M: Sequence[int], C: Sequence[int], cand: Candidate,
                       load_edges: np.ndarray, n_count_bins: int = 32, w_c0: float = 200.0,
                       w_c: float = 50.0, keep_n1: bool = True,
                       cont_subset: Optional[Sequence[int]] = None,
                       descriptor: str = "count_load") -> CandidateResult:
    """Full oracle evaluation of one candidate (steps 1-4 of the definition).

    cont_subset restricts the contingency loop to some positions of C (the
    metrics are then not computed); used for sampled checks at large sizes.
    """
    b = 1.0 / np.asarray(grid.x_pu, dtype=np.float64)
    if not validate_candidate(grid.n_bus, grid.from_bus, grid.to_bus, cand):
        return CandidateResult(valid=False, islanded=False)
    net = post_switch_network(grid.n_bus, grid.from_bus, grid.to_bus, b, grid.slack, P, cand)
    if not is_connected(net.n_node, net.fr, net.to, net.in_service):
        return CandidateResult(valid=True, islanded=True, n_switched=cand.n_slots_filled)
    if not np.all(np.isfinite(net.P)):
        # a NaN or infinite injection (the grid's or a moved amount): no flow
        # is defined; decided after the encoding rules and the islanding test
        return CandidateResult(valid=False, islanded=False, nonfinite=True,
                               n_switched=cand.n_slots_filled)
    f0 = solve_flows(net.n_node, net.fr, net.to, net.b, net.in_service, net.P, net.slack)
    M = np.asarray(M, dtype=np.int64)
    C = np.asarray(C, dtype=np.int64)
    T = P.shape[1]
    positions = range(len(C)) if cont_subset is None else list(cont_subset)
    n1 = np.full((len(C), len(M), T), np.nan) if keep_n1 else None
    island = np.zeros(len(C), dtype=bool)
    fmax = np.zeros((len(M), T), dtype=np.float64)

    def contingency_flows(l):
        """All-branch flows with branch l out (None if that islands)."""
        if not net.in_service[l]:
            return f0                                # already open: N-0 state
        ins = net.in_service.copy()
        ins[l] = False
        if not is_connected(net.n_node, net.fr, net.to, ins):
            return None
        return solve_flows(net.n_node, net.fr, net.to, net.b, ins, net.P, net.slack)

    for li in positions:
        fl = contingency_flows(int(C[li]))
        if fl is None:
            island[li] = True
            continue
        fm = fl[M]
        if keep_n1:
            n1[li] = fm
        fmax = np.maximum(fmax, np.abs(fm))
    res = CandidateResult(valid=True, islanded=False, base_flows=f0, n1_flows=n1, fmax=fmax,
                          island_cont=island, n_switched=cand.n_slots_filled)
    if cont_subset is None:
        lim = np.asarray(grid.limit_mw, dtype=np.float64)[M]
        met = n1_metrics(fmax, f0[M], lim)
        if met["worst"] is not None:
            # worst contingency: first in C order whose |flow| at (e*, t*)
            # is within the tie tolerance of the maximum (a second pass)
            e_i, t_i, _ = met["worst"]
            l_star = -1
            for li in range(len(C)):
                if island[li]:
                    continue
                if keep_n1:
                    v = abs(n1[li, e_i, t_i])
                else:
                    v = abs(contingency_flows(int(C[li]))[M[e_i], t_i])
                if v >= fmax[e_i, t_i] - WORST_CONT_TIE_MW:
                    l_star = li
                    break
            met["worst"] = (e_i, t_i, l_star)
        res.metrics = met
        res.metrics["n_island_cont"] = int(island.sum())
        res.fitness = fitness_f1(met["overload_mw"], met["n_crit_n0"], met["n_crit_n1"], w_c0, w_c)
        if descriptor == "paper":
            res.cell = descriptor_cell_paper(len(cand.opened), len(cand.splits),
                                             sum(len(mv) for _, mv in cand.splits))
        else:
            res.cell = descriptor_cell(cand.n_slots_filled, met["max_loading"], load_edges,
                                       n_count_bins)
        if met["worst"] is not None:
            e_i, t_i, l_i = met["worst"]
            res.metrics["worst_branch"] = int(M[e_i])
            res.metrics["worst_t"] = int(t_i)
            res.metrics["worst_cont"] = int(C[l_i]) if l_i >= 0 else -1
    return res


def _eval_one(args):
    grid, P, M, C, cand, edges, kw = args
    return evaluate_candidate(grid, P, M, C, cand, edges, **kw)


def _one_thread_per_worker():
    """Pool initializer: each worker process runs its library calls (sparse LU,
    BLAS) on one thread, so that P workers use P cores, not P x cores."""
    from threadpoolctl import threadpool_limits
    global _WORKER_LIMITS
    _WORKER_LIMITS = threadpool_limits(1)


def evaluate_batch(grid, P, M, C, batch, load_edges, idx=None, processes: int = 1, **kw):
    """Evaluate candidates (optionally a subset idx), one candidate per task
    of a pool of single-threaded worker processes."""
    if idx is None:
        idx = range(batch.n_cand)
    cands = [candidate_from_batch(batch, int(c)) for c in idx]
    jobs = [(grid, P, M, C, cd, load_edges, kw) for cd in cands]
    if processes <= 1:
        return [_eval_one(j) for j in jobs]
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(processes, initializer=_one_thread_per_worker) as pool:
        return pool.map(_eval_one, jobs, chunksize=1)


def busbar_outage_flows(net: Network, bus: int):
    """Flows [m, T] of the post-switch network with busbar `bus` out (its node
    loses every in-service branch and its injection, which the slack picks
    up; a split's busbar B is another node and stays), or None if the rest of
    the network islands.  Node `bus` is removed before the re-solve."""
    ins = net.in_service.copy()
    ins[(net.fr == bus) | (net.to == bus)] = False
    keep = np.arange(net.n_node) != bus
    remap = np.cumsum(keep) - 1
    fr, to = remap[net.fr], remap[net.to]
    if not is_connected(net.n_node - 1, fr, to, ins):
        return None
    return solve_flows(net.n_node - 1, fr, to, net.b, ins, net.P[keep], int(remap[net.slack]))


def busbar_metrics(grid, P: np.ndarray, M, cand: Candidate, busbars) -> dict:
    """Fitness function heuristics, busbar penalty: with f^(b) the flows under
    busbar outage b, lambda_b = sum_{e in M, t} max(max_b |f^(b)_e(t)| -
    fbar_e, 0) over the busbar outages that do not island the grid (counted
    in n_island).  Candidate assumed valid and connected."""
    b = 1.0 / np.asarray(grid.x_pu, dtype=np.float64)
    net = post_switch_network(grid.n_bus, grid.from_bus, grid.to_bus, b, grid.slack, P, cand)
    M = np.asarray(M, dtype=np.int64)
    fmax = np.zeros((len(M), P.shape[1]))
    n_isl = 0
    for bus in busbars:
        f = busbar_outage_flows(net, int(bus))
        if f is None:
            n_isl += 1
            continue
        fmax = np.maximum(fmax, np.abs(f[M]))
    lim = np.asarray(grid.limit_mw, dtype=np.float64)[M]
    lam = float(np.maximum(fmax - lim[:, None], 0.0).sum())
    return dict(lambda_b=lam, n_island=n_isl, fmax=fmax)


def fitness_f2(fitness_f1: float, lambda_b: float, lambda_b_pre: float) -> float:
    """High-level loop, the second study case: lambda_f2 = lambda_f1 -
    max(lambda_b - lambda_b_pre, 0)."""
    return fitness_f1 - max(lambda_b - lambda_b_pre, 0.0)
