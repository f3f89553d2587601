"""Hand-built grids and candidate tables for the encoding's validity rules and
the method's degenerate cases, plus a test-side replica of the candidate's
bordered matrix that only selects candidates whose LU interchanges rows
(imported by test modules only).

Validity rules (genome of the Repertoire design section; the fixed-slot
encoding with -1 for an empty slot): opened ids in range and distinct; split
buses in range and distinct; each split moves a non-empty list of distinct
branches incident to its bus, none of them opened; at most 8 filled slots;
at most 64 moved branches over all splits.  Every invalid row below breaks
exactly one rule of a valid neighbour in the table, so both sides of each
boundary are present.
"""
from __future__ import annotations

import numpy as np

import gridgen as gg
from oracle.dcflow import Candidate

# 10 buses, 18 branches: a ring 0..9, five spokes across it and three chords.
TEN_BUS_BRANCHES = [
    (0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 6), (6, 7), (7, 8), (8, 9), (9, 0),
    (0, 5), (1, 6), (2, 7), (3, 8), (4, 9), (1, 3), (5, 7), (6, 8),
]
# bus 3 is incident to branches 2, 3, 13, 15; bus 1 to 0, 1, 11, 15; bus 8 to 7, 8, 13, 17


def ten_bus_grid() -> gg.Grid:
    fr = np.array([a for a, _ in TEN_BUS_BRANCHES], np.int32)
    to = np.array([b for _, b in TEN_BUS_BRANCHES], np.int32)
    m = len(fr)
    x = 0.02 + 0.01 * (np.arange(m) % 7)
    lim = np.full(m, 60.0)
    return gg.Grid(n_bus=10, from_bus=fr, to_bus=to, x_pu=x, limit_mw=lim)


def _c(opened, splits):
    return Candidate(opened=list(opened), splits=[(b, list(mv)) for b, mv in splits],
                     moved_p=[None] * len(splits), n_slots_filled=len(opened) + len(splits))


# (label, candidate, valid?)
TEN_BUS_TABLE = [
    ("empty candidate (rank 0)", _c([], []), True),
    ("base: one opening, one split", _c([0], [(3, [2, 13])]), True),
    ("two distinct openings", _c([0, 17], []), True),
    ("opening repeated", _c([0, 0], []), False),
    ("opening id m-1", _c([17], []), True),
    ("opening id m (out of range)", _c([18], []), False),
    ("opening id -2 (negative, not the empty marker)", _c([-2], []), False),
    ("split bus n-1", _c([], [(9, [8])]), True),
    ("split bus n (out of range)", _c([], [(10, [8])]), False),
    ("split bus -2", _c([], [(-2, [8])]), False),
    ("two splits at distinct buses", _c([], [(3, [2]), (8, [7])]), True),
    ("split bus repeated", _c([], [(3, [2]), (3, [13])]), False),
    ("moved list of one branch", _c([], [(3, [2])]), True),
    ("moved list empty", _c([], [(3, [])]), False),
    ("moved list distinct", _c([], [(3, [2, 13])]), True),
    ("moved branch repeated", _c([], [(3, [2, 2])]), False),
    ("moved branch incident (chord 1-3)", _c([], [(3, [15])]), True),
    ("moved branch not incident", _c([], [(3, [1])]), False),
    ("moved branch id m (out of range)", _c([], [(3, [18])]), False),
    ("moved branch id -1 inside a list", _c([], [(3, [-1])]), False),
    ("opened branch not moved", _c([1], [(3, [2])]), True),
    ("moved branch also opened", _c([2], [(3, [2])]), False),
    ("branch moved by the splits at both its ends", _c([], [(1, [15]), (3, [15])]), True),
    ("split moving every branch of its bus (busbar A left empty)",
     _c([], [(3, [2, 3, 13, 15])]), True),
    ("rank 8: eight openings", _c([0, 1, 2, 3, 4, 5, 6, 7], []), True),
    ("rank 8: seven openings and one split", _c([0, 1, 2, 4, 5, 6, 7], [(3, [13])]), True),
    ("rank 9: eight openings and one split", _c([0, 1, 2, 4, 5, 6, 7, 8], [(3, [13])]), False),
    ("rank 8: six openings and two splits",
     _c([4, 5, 6, 9, 10, 12], [(3, [2]), (1, [0])]), True),
    ("rank 9: seven openings and two splits",
     _c([4, 5, 6, 9, 10, 12, 14], [(3, [2]), (1, [0])]), False),
]


def star_grid():
    """Two hubs: bus 0 joined to buses 2..41 (40 branches), bus 1 to buses
    2..31 (30 branches), plus branch 0-1.  Branch ids: 0-1 is 0, 0-i is i-1
    (i = 2..41), 1-j is 39 + j (j = 2..31)."""
    br = [(0, 1)] + [(0, i) for i in range(2, 42)] + [(1, j) for j in range(2, 32)]
    fr = np.array([a for a, _ in br], np.int32)
    to = np.array([b for _, b in br], np.int32)
    m = len(br)
    return gg.Grid(n_bus=42, from_bus=fr, to_bus=to, x_pu=0.05 + 0.002 * np.arange(m),
                   limit_mw=np.full(m, 80.0))


STAR_HUB0 = list(range(1, 41))          # branches 0-i
STAR_HUB1 = list(range(41, 71))         # branches 1-j

STAR_TABLE = [
    ("64 moved branches over two splits", _c([], [(0, STAR_HUB0[:34]), (1, STAR_HUB1)]), True),
    ("65 moved branches over two splits", _c([], [(0, STAR_HUB0[:35]), (1, STAR_HUB1)]), False),
]


def as_batch(cands, T: int, n_open_slots: int = 8, n_split_slots: int = 8) -> gg.Batch:
    """Pack hand-built candidates into the fixed-slot encoding (filled slots
    first, -1 after)."""
    B = len(cands)
    op = np.full((B, n_open_slots), gg.EMPTY, np.int32)
    sb = np.full((B, n_split_slots), gg.EMPTY, np.int32)
    offs, br = [0], []
    for c, cd in enumerate(cands):
        op[c, :len(cd.opened)] = cd.opened
        for j in range(n_split_slots):
            if j < len(cd.splits):
                sb[c, j] = cd.splits[j][0]
                br.extend(cd.splits[j][1])
            offs.append(len(br))
    return gg.Batch(open=op, split_bus=sb, moved_off=np.asarray(offs, np.int32),
                    moved_br=np.asarray(br, np.int32))


# ----------------------------------------------------------------------------
# Row interchanges of the candidate's bordered system.  A test-side replica of
# the r x r matrix the set-up factors (openings K first, then one row per
# split scaled by 1/s_j; derived in the header of the set-up kernel's source),
# built from S = A L^-1 A^T computed here with a dense library inverse, and
# partial pivoting that swaps only on a strictly larger entry below.  Used to
# pick candidates whose LU must swap rows, so that the swapped path is shown
# to run; the values compared in the tests come from the oracle.
def sensitivity_s(grid) -> tuple:
    n, m = grid.n_bus, grid.n_branch
    A = np.zeros((m, n))
    A[np.arange(m), grid.from_bus] = 1.0
    A[np.arange(m), grid.to_bus] = -1.0
    b = 1.0 / np.asarray(grid.x_pu, np.float64)
    L = A.T @ (b[:, None] * A)
    keep = np.arange(n) != grid.slack
    Li = np.zeros((n, n))
    Li[np.ix_(keep, keep)] = np.linalg.inv(L[np.ix_(keep, keep)])
    return A @ Li @ A.T, b


def bordered_matrix(S, b, grid, opened, splits) -> np.ndarray:
    k, r = len(opened), len(opened) + len(splits)
    sg = [[(e, 1.0 if grid.from_bus[e] == bus else -1.0) for e in mv] for bus, mv in splits]
    M = np.zeros((r, r))
    for i in range(r):
        for q in range(r):
            if i < k:
                if q < k:
                    v = float(i == q) - b[opened[i]] * S[opened[i], opened[q]]
                else:
                    v = b[opened[i]] * sum(s * b[e] * S[opened[i], e] for e, s in sg[q - k])
            else:
                j = i - k
                if q < k:
                    v = sum(s * b[e] * S[e, opened[q]] for e, s in sg[j])
                else:
                    v = 0.0
                    for e, s in sg[j]:
                        for e2, s2 in sg[q - k]:
                            v -= s * b[e] * s2 * b[e2] * S[e, e2]
                            if e == e2:
                                v += s * s2 * b[e]
                v /= sum(b[e] for e, _ in sg[j])
            M[i, q] = v
    return M


def pivot_swaps(M) -> tuple:
    """(number of row interchanges, smallest pivot, smallest ratio by which a
    chosen pivot beat the diagonal entry) of partial pivoting."""
    M = np.array(M, dtype=np.float64)
    r = len(M)
    sw, minpiv, beat = 0, np.inf, np.inf
    for p in range(r):
        best, bv = p, abs(M[p, p])
        for i in range(p + 1, r):
            if abs(M[i, p]) > bv:
                best, bv = i, abs(M[i, p])
        if best != p:
            sw += 1
            beat = min(beat, bv / max(abs(M[p, p]), 1e-300))
            M[[p, best]] = M[[best, p]]
        minpiv = min(minpiv, bv)
        if bv > 0:
            for i in range(p + 1, r):
                f = M[i, p] / M[p, p]
                M[i, p] = f
                M[i, p + 1:] -= f * M[p, p + 1:]
    return sw, minpiv, beat
