"""PTDF and bridges of a grid (oracle; test infrastructure only).

Importer section of the paper: the DC optimizer starts from the power
transfer distribution factors of the pre-optimisation topology and from the
branches whose opening would split the grid.  Plain definitions:

  PTDF[e, j] = b_e (X[from_e, j] - X[to_e, j]),  X = B'^{-1} padded with a zero
  slack row and column, B' the nodal susceptance matrix without the slack
  row and column (a dense library solve of B' X = I);

  a branch is a bridge iff the grid without it is not connected (one
  connected-components call per branch).
"""
from __future__ import annotations

import numpy as np

from .dcflow import is_connected


def ptdf(n_bus: int, from_bus, to_bus, b, slack: int = 0) -> np.ndarray:
    fr = np.asarray(from_bus, dtype=np.int64)
    to = np.asarray(to_bus, dtype=np.int64)
    b = np.asarray(b, dtype=np.float64)
    m = len(fr)
    L = np.zeros((n_bus, n_bus))
    for e in range(m):
        L[fr[e], fr[e]] += b[e]
        L[to[e], to[e]] += b[e]
        L[fr[e], to[e]] -= b[e]
        L[to[e], fr[e]] -= b[e]
    keep = np.arange(n_bus) != slack
    X = np.zeros((n_bus, n_bus))
    X[np.ix_(keep, keep)] = np.linalg.solve(L[np.ix_(keep, keep)], np.eye(n_bus - 1))
    return b[:, None] * (X[fr] - X[to])


def bridges(n_bus: int, from_bus, to_bus) -> np.ndarray:
    m = len(from_bus)
    out = np.zeros(m, dtype=bool)
    for e in range(m):
        ins = np.ones(m, dtype=bool)
        ins[e] = False
        out[e] = not is_connected(n_bus, from_bus, to_bus, ins)
    return out
