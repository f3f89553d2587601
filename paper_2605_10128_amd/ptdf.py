"""Host FP64 PTDF of the unswitched grid: the library's input.

The paper's importer computes the PTDF of the pre-optimisation topology on the
CPU before the GPU loop starts; this helper plays that role for synthetic
grids.  PTDF = diag(b) A L_red^{-1} (slack row/column of the nodal susceptance
matrix L = A^T diag(b) A removed, slack column of the PTDF zero), computed
with a dense Cholesky factorisation.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def build_ptdf(n_bus: int, from_bus, to_bus, susceptance, slack: int = 0) -> np.ndarray:
    fr = np.asarray(from_bus, dtype=np.int64)
    to = np.asarray(to_bus, dtype=np.int64)
    b = np.asarray(susceptance, dtype=np.float64)
    m = len(fr)
    L = np.zeros((n_bus, n_bus))
    np.add.at(L, (fr, fr), b)
    np.add.at(L, (to, to), b)
    np.add.at(L, (fr, to), -b)
    np.add.at(L, (to, fr), -b)
    keep = np.arange(n_bus) != slack
    Lr = L[np.ix_(keep, keep)]
    cho = sla.cho_factor(Lr, lower=True, check_finite=False)
    Linv = sla.cho_solve(cho, np.eye(n_bus - 1), check_finite=False)
    X = np.zeros((n_bus, n_bus))
    X[np.ix_(keep, keep)] = Linv
    # row e of A X is X[from(e)] - X[to(e)]
    ptdf = b[:, None] * (X[fr] - X[to])
    return np.ascontiguousarray(ptdf)
