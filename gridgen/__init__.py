"""Seeded synthetic inputs: grids, injections, monitored/contingency sets and
candidate topologies.

This module is shared by the oracle and the GPU path and is deliberately free
of any DC power-flow arithmetic: it only draws random numbers and lays them
out as plain integer / float arrays.  The one graph routine here (bridge
finding) stands in for the importer's action-set construction (Importer
section: disconnectable branches are those whose removal does not island the
grid, found with Tarjan's bridge algorithm); it is never used to decide any
output of the method.

Recipe:
  * spanning tree: random recursive tree over a random bus permutation,
  * chords: uniform bus pairs, no self loops, no parallel branches,
  * reactance x ~ U(0.01, 0.3) pu, thermal limit ~ U(50, 300) MW, slack bus 0,
  * injections P_i ~ N(0, 40) MW; for T > 1 a daily sinusoid
    P_i(t) = P_i (1 + 0.5 sin(2 pi t / 24)) + N(0, 15); the slack takes minus
    the sum of all other injections in every timestep,
  * candidates: distinct non-bridge openings plus bus splits that move a
    non-trivial subset of a bus's incident branches to a second busbar.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "Grid", "Batch", "make_grid", "bridges", "make_injections",
    "select_sets", "select_busbars", "make_split_table", "make_candidates", "make_candidates_cfg1",
    "make_candidates_cfg2", "make_candidates_ranked", "CONFIGS", "build_config",
    "default_load_edges", "EMPTY",
]

EMPTY = -1  # empty genome slot


@dataclass
class Grid:
    n_bus: int
    from_bus: np.ndarray      # int32 [m]
    to_bus: np.ndarray        # int32 [m]
    x_pu: np.ndarray          # float64 [m] series reactance
    limit_mw: np.ndarray      # float64 [m] thermal limit
    slack: int = 0

    @property
    def n_branch(self) -> int:
        return int(self.from_bus.shape[0])

    def incident(self):
        """Per-bus list of incident branch ids (plain adjacency, no arithmetic)."""
        inc = [[] for _ in range(self.n_bus)]
        for e, (a, b) in enumerate(zip(self.from_bus.tolist(), self.to_bus.tolist())):
            inc[a].append(e)
            inc[b].append(e)
        return inc


@dataclass
class Batch:
    """Candidate topologies in the fixed-slot genome encoding.

    open[c, i]       branch id opened in slot i, or EMPTY
    split_bus[c, j]  bus split in slot j, or EMPTY
    moved_off        CSR offsets over the flattened (c, j) split slots
    moved_br         branch ids moved to the new busbar B of each split
    moved_p          optional [B * n_split_slots, T] MW moved to busbar B
    """
    open: np.ndarray
    split_bus: np.ndarray
    moved_off: np.ndarray
    moved_br: np.ndarray
    moved_p: Optional[np.ndarray] = None
    split_action: Optional[np.ndarray] = None   # [B, n_split_slots] action-table id or EMPTY

    @property
    def n_cand(self) -> int:
        return int(self.open.shape[0])

    def moved(self, c: int, j: int) -> np.ndarray:
        s = c * self.split_bus.shape[1] + j
        return self.moved_br[self.moved_off[s]:self.moved_off[s + 1]]

    def subset(self, idx) -> "Batch":
        """Candidates idx (repeats allowed) as a new batch."""
        idx = np.asarray(idx, dtype=np.int64)
        ns = self.split_bus.shape[1]
        slots = (idx[:, None] * ns + np.arange(ns)[None, :]).ravel()
        lo = self.moved_off[:-1][slots].astype(np.int64)
        lens = (self.moved_off[1:][slots] - self.moved_off[:-1][slots]).astype(np.int64)
        offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
        rep = np.repeat(lo - offs[:-1], lens)
        br = self.moved_br[np.arange(int(offs[-1])) + rep] if offs[-1] else np.zeros(0, np.int32)
        return Batch(
            open=self.open[idx].copy(),
            split_bus=self.split_bus[idx].copy(),
            moved_off=offs,
            moved_br=np.asarray(br, dtype=np.int32),
            moved_p=None if self.moved_p is None else self.moved_p[slots].copy(),
            split_action=None if self.split_action is None else self.split_action[idx].copy(),
        )


def make_grid(n_bus: int, n_branch: int, seed: int,
              x_range=(0.01, 0.3), limit_range=(50.0, 300.0)) -> Grid:
    """Random recursive spanning tree plus uniform chords."""
    if n_branch < n_bus - 1:
        raise ValueError("need at least n_bus - 1 branches for a spanning tree")
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n_bus)
    edges = []
    seen = set()
    for i in range(1, n_bus):
        j = int(rng.integers(0, i))
        a, b = int(perm[i]), int(perm[j])
        edges.append((a, b))
        seen.add((min(a, b), max(a, b)))
    max_edges = n_bus * (n_bus - 1) // 2
    if n_branch > max_edges:
        raise ValueError("too many branches for a simple graph")
    while len(edges) < n_branch:
        a, b = (int(v) for v in rng.integers(0, n_bus, size=2))
        if a == b:
            continue
        key = (min(a, b), max(a, b))
        if key in seen:
            continue
        seen.add(key)
        edges.append((a, b))
    edges = np.asarray(edges, dtype=np.int64)
    # random orientation and branch order
    flip = rng.random(n_branch) < 0.5
    fr = np.where(flip, edges[:, 1], edges[:, 0])
    to = np.where(flip, edges[:, 0], edges[:, 1])
    order = rng.permutation(n_branch)
    fr, to = fr[order], to[order]
    x = rng.uniform(x_range[0], x_range[1], size=n_branch)
    lim = rng.uniform(limit_range[0], limit_range[1], size=n_branch)
    return Grid(n_bus=n_bus, from_bus=fr.astype(np.int32), to_bus=to.astype(np.int32),
                x_pu=x, limit_mw=lim, slack=0)


def bridges(n_bus: int, from_bus, to_bus, in_service=None) -> np.ndarray:
    """Tarjan's bridge finding (iterative DFS).  Returns a bool mask over branches.

    Stand-in for the importer's action-set filter (disconnectable set D).
    """
    m = len(from_bus)
    if in_service is None:
        in_service = np.ones(m, dtype=bool)
    adj = [[] for _ in range(n_bus)]
    for e in range(m):
        if in_service[e]:
            a, b = int(from_bus[e]), int(to_bus[e])
            adj[a].append((b, e))
            adj[b].append((a, e))
    disc = [-1] * n_bus
    low = [0] * n_bus
    is_bridge = np.zeros(m, dtype=bool)
    timer = 0
    for root in range(n_bus):
        if disc[root] != -1:
            continue
        disc[root] = low[root] = timer
        timer += 1
        stack = [(root, -1, iter(adj[root]))]
        while stack:
            u, pe, it = stack[-1]
            advanced = False
            for v, e in it:
                if e == pe:
                    continue
                if disc[v] == -1:
                    disc[v] = low[v] = timer
                    timer += 1
                    stack.append((v, e, iter(adj[v])))
                    advanced = True
                    break
                low[u] = min(low[u], disc[v])
            if not advanced:
                stack.pop()
                if stack:
                    p = stack[-1][0]
                    low[p] = min(low[p], low[u])
                    if low[u] > disc[p]:
                        is_bridge[pe] = True
    return is_bridge


def make_injections(grid: Grid, T: int, seed: int, sigma=40.0, daily_amp=0.5,
                    noise=15.0) -> np.ndarray:
    """Nodal injections [n_bus, T] in MW, balanced by the slack bus each timestep."""
    rng = np.random.default_rng(seed)
    base = rng.normal(0.0, sigma, size=grid.n_bus)
    if T == 1:
        P = base[:, None].copy()
    else:
        t = np.arange(T)
        shape = 1.0 + daily_amp * np.sin(2.0 * np.pi * t / 24.0)
        P = base[:, None] * shape[None, :] + rng.normal(0.0, noise, size=(grid.n_bus, T))
    P[grid.slack, :] = 0.0
    P[grid.slack, :] = -P.sum(axis=0)
    return P


def select_sets(grid: Grid, n_monitored: Optional[int], n_contingency: Optional[int],
                seed: int):
    """Monitored set M (uniform over all branches) and contingency set C
    (uniform over base-grid non-bridge branches); None means 'all'."""
    rng = np.random.default_rng(seed)
    m = grid.n_branch
    nb = bridges(grid.n_bus, grid.from_bus, grid.to_bus)
    non_bridge = np.flatnonzero(~nb)
    if n_monitored is None or n_monitored >= m:
        M = np.arange(m)
    else:
        M = np.sort(rng.choice(m, size=n_monitored, replace=False))
    if n_contingency is None:
        C = np.arange(m)
    else:
        C = np.sort(rng.choice(non_bridge, size=min(n_contingency, len(non_bridge)), replace=False))
    return M.astype(np.int32), C.astype(np.int32)


def _random_assignment(rng, inc_list, max_tries=64):
    """Assign each incident branch to busbar A or B; reject trivial splits."""
    d = len(inc_list)
    for _ in range(max_tries):
        bits = rng.random(d) < 0.5
        k = int(bits.sum())
        if 0 < k < d:
            return [inc_list[i] for i in range(d) if bits[i]]
    # fallback: move exactly one branch
    return [inc_list[int(rng.integers(0, d))]]


def select_busbars(grid: Grid, n: int, seed: int, max_degree: int = 16) -> np.ndarray:
    """Seeded busbar outage set: n distinct non-slack buses with 1..max_degree
    branches (a stand-in for the operator's busbar outage list)."""
    deg = np.bincount(np.concatenate([grid.from_bus, grid.to_bus]), minlength=grid.n_bus)
    ok = np.flatnonzero((deg >= 1) & (deg <= max_degree) & (np.arange(grid.n_bus) != grid.slack))
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(ok, size=min(n, len(ok)), replace=False)).astype(np.int32)


def make_split_table(grid: Grid, size: int, seed: int, min_degree: int = 3):
    """Seeded split-action table: each entry is (bus, moved branch list),
    a stand-in for the importer's station-local reconfiguration set A."""
    rng = np.random.default_rng(seed)
    inc = grid.incident()
    eligible = [i for i in range(grid.n_bus) if len(inc[i]) >= min_degree]
    table = []
    for _ in range(size):
        bus = int(eligible[int(rng.integers(0, len(eligible)))])
        table.append((bus, sorted(_random_assignment(rng, inc[bus]))))
    return table


def _pack(opens, splits, n_open_slots, n_split_slots, T, moved_p_list, actions=None):
    B = len(opens)
    op = np.full((B, n_open_slots), EMPTY, dtype=np.int32)
    sb = np.full((B, n_split_slots), EMPTY, dtype=np.int32)
    offs = [0]
    br = []
    any_moved = moved_p_list is not None and any(
        v is not None for row in moved_p_list for v in row)
    mp = np.zeros((B * n_split_slots, T), dtype=np.float64) if any_moved else None
    for c in range(B):
        for i, e in enumerate(opens[c]):
            op[c, i] = e
        for j in range(n_split_slots):
            if j < len(splits[c]):
                bus, moved = splits[c][j]
                sb[c, j] = bus
                br.extend(moved)
                offs.append(offs[-1] + len(moved))
                if mp is not None and moved_p_list[c][j] is not None:
                    mp[c * n_split_slots + j] = moved_p_list[c][j]
            else:
                offs.append(offs[-1])
    sa = None
    if actions is not None:
        sa = np.full((B, n_split_slots), EMPTY, dtype=np.int32)
        for c in range(B):
            for j, a in enumerate(actions[c]):
                sa[c, j] = a
    return Batch(open=op, split_bus=sb, moved_off=np.asarray(offs, dtype=np.int32),
                 moved_br=np.asarray(br, dtype=np.int32), moved_p=mp, split_action=sa)


def _shuffle_slots(rng, batch: Batch) -> Batch:
    """Scatter filled slots over random slot positions (empty slots anywhere)."""
    B, no = batch.open.shape
    ns = batch.split_bus.shape[1]
    op = batch.open.copy()
    for c in range(B):
        op[c] = op[c][rng.permutation(no)]
    perm_s = [rng.permutation(ns) for _ in range(B)]
    sb = np.full_like(batch.split_bus, EMPTY)
    sa = None if batch.split_action is None else np.full_like(batch.split_action, EMPTY)
    offs = [0]
    br = []
    mp = None if batch.moved_p is None else np.zeros_like(batch.moved_p)
    for c in range(B):
        for j in range(ns):
            src = int(perm_s[c][j])
            sb[c, j] = batch.split_bus[c, src]
            if sa is not None:
                sa[c, j] = batch.split_action[c, src]
            mv = batch.moved(c, src)
            br.extend(mv.tolist())
            offs.append(offs[-1] + len(mv))
            if mp is not None:
                mp[c * ns + j] = batch.moved_p[c * ns + src]
    return Batch(open=op, split_bus=sb, moved_off=np.asarray(offs, dtype=np.int32),
                 moved_br=np.asarray(br, dtype=np.int32), moved_p=mp, split_action=sa)


def _moved_injection(rng, P_bus_row, move_frac):
    if move_frac <= 0.0 or rng.random() >= move_frac:
        return None
    share = rng.uniform(0.1, 0.9)
    return share * np.asarray(P_bus_row, dtype=np.float64)


def make_candidates_cfg1(grid: Grid, B: int, seed: int, max_open: int = 2,
                         n_open_slots: int = 2) -> Batch:
    """B candidates each opening 0..max_open distinct non-bridge branches."""
    rng = np.random.default_rng(seed)
    nb = bridges(grid.n_bus, grid.from_bus, grid.to_bus)
    D = np.flatnonzero(~nb)
    opens = []
    for _ in range(B):
        k = int(rng.integers(0, max_open + 1))
        opens.append(rng.choice(D, size=k, replace=False).tolist())
    return _shuffle_slots(rng, _pack(opens, [[] for _ in range(B)], n_open_slots, 0, 1, None))


def make_candidates_cfg2(grid: Grid, B: int, seed: int, P=None, open_range=(1, 4),
                         split_range=(0, 2), move_frac: float = 0.0,
                         n_open_slots: int = 4, n_split_slots: int = 2) -> Batch:
    """1-4 non-bridge openings plus 0-2 bus splits at distinct degree>=3 buses,
    each incident branch assigned to busbar A or B at random (non-trivial)."""
    rng = np.random.default_rng(seed)
    inc = grid.incident()
    nb = bridges(grid.n_bus, grid.from_bus, grid.to_bus)
    D = np.flatnonzero(~nb)
    eligible = np.asarray([i for i in range(grid.n_bus) if len(inc[i]) >= 3])
    T = 1 if P is None else P.shape[1]
    opens, splits, mps = [], [], []
    for _ in range(B):
        s = int(rng.integers(split_range[0], split_range[1] + 1))
        buses = rng.choice(eligible, size=s, replace=False).tolist()
        sp, mp, moved_all = [], [], set()
        for bus in buses:
            mv = sorted(_random_assignment(rng, inc[bus]))
            sp.append((int(bus), mv))
            moved_all.update(mv)
            mp.append(None if P is None else _moved_injection(rng, P[bus], move_frac))
        k = int(rng.integers(open_range[0], open_range[1] + 1))
        pool = np.asarray([e for e in D.tolist() if e not in moved_all])
        opens.append(rng.choice(pool, size=k, replace=False).tolist())
        splits.append(sp)
        mps.append(mp)
    batch = _pack(opens, splits, n_open_slots, n_split_slots, T, mps if P is not None else None)
    return _shuffle_slots(rng, batch)


def make_candidates_ranked(grid: Grid, B: int, seed: int, split_table, P=None,
                           rank_range=(0, 8), split_prob: float = 1.0 / 3.0,
                           move_frac: float = 0.0, n_open_slots: int = 8,
                           n_split_slots: int = 8) -> Batch:
    """Uneven-rank candidates: r ~ U{rank_range}, splits ~ Binomial(r, split_prob)
    drawn from the split-action table at distinct buses, the rest distinct
    non-bridge openings that are not moved by the candidate's own splits.
    Rows violating a rule are redrawn whole (vectorised rejection)."""
    rng = np.random.default_rng(seed)
    nb = bridges(grid.n_bus, grid.from_bus, grid.to_bus)
    D = np.flatnonzero(~nb).astype(np.int64)
    T = 1 if P is None else P.shape[1]
    m = grid.n_branch
    n_tab = len(split_table)
    tab_bus = np.asarray([b for b, _ in split_table], dtype=np.int64)
    tab_len = np.asarray([len(mv) for _, mv in split_table], dtype=np.int64)
    tab_off = np.concatenate([[0], np.cumsum(tab_len)])
    tab_flat = np.asarray([e for _, mv in split_table for e in mv], dtype=np.int64)
    moved_keys = np.sort(np.repeat(np.arange(n_tab, dtype=np.int64), tab_len) * m + tab_flat)

    r = rng.integers(rank_range[0], rank_range[1] + 1, size=B)
    s = np.minimum(rng.binomial(r, split_prob), n_split_slots)
    k = np.minimum(r - s, n_open_slots)
    S = max(1, n_split_slots)
    K = max(1, n_open_slots)
    act = np.full((B, S), EMPTY, dtype=np.int64)
    opn = np.full((B, K), EMPTY, dtype=np.int64)
    sm = np.arange(S)[None, :] < s[:, None]
    km = np.arange(K)[None, :] < k[:, None]
    todo = np.arange(B)
    while todo.size:
        a = rng.integers(0, max(n_tab, 1), size=(todo.size, S))
        o = D[rng.integers(0, len(D), size=(todo.size, K))]
        a = np.where(sm[todo], a, EMPTY)
        o = np.where(km[todo], o, EMPTY)
        bad = np.zeros(todo.size, dtype=bool)
        bus = np.where(a >= 0, tab_bus[np.maximum(a, 0)], -1)
        for j in range(S):
            for j2 in range(j):
                bad |= (bus[:, j] >= 0) & (bus[:, j] == bus[:, j2])
        for i in range(K):
            for i2 in range(i):
                bad |= (o[:, i] >= 0) & (o[:, i] == o[:, i2])
            for j in range(S):
                key = a[:, j] * m + o[:, i]
                hit = (a[:, j] >= 0) & (o[:, i] >= 0)
                pos = np.searchsorted(moved_keys, key)
                pos = np.minimum(pos, len(moved_keys) - 1)
                bad |= hit & (moved_keys[pos] == key)
        ok = ~bad
        act[todo[ok]] = a[ok]
        opn[todo[ok]] = o[ok]
        todo = todo[bad]
    # scatter the filled slots over random slot positions
    act = np.take_along_axis(act, np.argsort(rng.random((B, S)), axis=1), axis=1)[:, :n_split_slots]
    opn = np.take_along_axis(opn, np.argsort(rng.random((B, K)), axis=1), axis=1)[:, :n_open_slots]
    sb = np.where(act >= 0, tab_bus[np.maximum(act, 0)], EMPTY)
    lens = np.where(act >= 0, tab_len[np.maximum(act, 0)], 0).ravel()
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    starts = np.where(act >= 0, tab_off[np.maximum(act, 0)], 0).ravel()
    rep = np.repeat(starts - offs[:-1], lens)
    br = tab_flat[np.arange(int(offs[-1])) + rep] if offs[-1] else np.zeros(0, np.int64)
    mp = None
    if P is not None and move_frac > 0.0:
        flat_bus = sb.ravel()
        take = (flat_bus >= 0) & (rng.random(flat_bus.size) < move_frac)
        share = rng.uniform(0.1, 0.9, size=flat_bus.size)
        mp = np.zeros((flat_bus.size, T), dtype=np.float64)
        mp[take] = share[take, None] * np.asarray(P, dtype=np.float64)[flat_bus[take]]
        if not take.any():
            mp = None
    return Batch(open=opn.astype(np.int32), split_bus=sb.astype(np.int32), moved_off=offs,
                 moved_br=br.astype(np.int32), moved_p=mp,
                 split_action=act.astype(np.int32))


def action_bits(grid: Grid, batch: Batch, table_size: int):
    """Feature bitmask of each candidate as CSR (offsets, ids): bit d for the
    opening of the d-th base non-bridge branch, bit |D| + a for split action a
    of the action table.  Ids are sorted and distinct within a row.
    Returns (off [B+1], ids, n_bits)."""
    nb = bridges(grid.n_bus, grid.from_bus, grid.to_bus)
    D = np.flatnonzero(~nb)
    pos = -np.ones(grid.n_branch + 1, dtype=np.int64)
    pos[D] = np.arange(len(D))
    op = batch.open.astype(np.int64)
    cols = [np.where(op >= 0, pos[np.where(op >= 0, op, grid.n_branch)], -1)]
    if batch.split_action is not None:
        sa = batch.split_action.astype(np.int64)
        cols.append(np.where(sa >= 0, len(D) + sa, -1))
    ids = np.concatenate(cols, axis=1)
    big = np.iinfo(np.int64).max
    ids = np.sort(np.where(ids >= 0, ids, big), axis=1)
    valid = ids != big
    off = np.concatenate([[0], np.cumsum(valid.sum(axis=1))]).astype(np.int32)
    return off, ids[valid].astype(np.int32), len(D) + table_size


def make_candidates(kind: str, grid: Grid, B: int, seed: int, **kw) -> Batch:
    if kind == "cfg1":
        return make_candidates_cfg1(grid, B, seed, **kw)
    if kind == "cfg2":
        return make_candidates_cfg2(grid, B, seed, **kw)
    if kind == "ranked":
        return make_candidates_ranked(grid, B, seed, **kw)
    raise ValueError(kind)


def default_load_edges(n_load_bins: int = 32, lo: float = 0.25, hi: float = 64.0) -> np.ndarray:
    """Geometric max-loading bin edges from lo to hi: n_load_bins - 1 inner edges
    (bin 0 is rho < lo, the last bin rho >= hi)."""
    k = n_load_bins - 1
    return np.asarray([lo * (hi / lo) ** (i / (k - 1)) for i in range(k)], dtype=np.float64)


# Workload shapes (buses, branches, timesteps, candidates, |M|, |C|)
CONFIGS = {
    1: dict(name="tiny-30bus", n_bus=30, n_branch=41, T=1, B=64, n_mon=None, n_cont=None,
            kind="cfg1"),
    2: dict(name="gpu-500bus", n_bus=500, n_branch=800, T=1, B=4096, n_mon=None, n_cont=None,
            kind="cfg2"),
    3: dict(name="batch-2000bus", n_bus=2000, n_branch=3200, T=24, B=16384, n_mon=1200,
            n_cont=1600, kind="ranked"),
    4: dict(name="precision-6000bus", n_bus=6000, n_branch=9500, T=24, B=8192, n_mon=2000,
            n_cont=3000, kind="ranked"),
}


@dataclass
class Workload:
    cfg: int
    grid: Grid
    P: np.ndarray
    M: np.ndarray
    C: np.ndarray
    batch: Batch
    split_table: list = field(default_factory=list)


def build_config(cfg: int, B: Optional[int] = None, seed_offset: int = 0,
                 move_frac: float = 0.0, **overrides) -> Workload:
    """Assemble one seeded workload (grid, injections, M, C, candidates)."""
    spec = dict(CONFIGS[cfg])
    spec.update(overrides)
    seed = 0x5EED0000 + cfg + seed_offset
    grid = make_grid(spec["n_bus"], spec["n_branch"], seed)
    P = make_injections(grid, spec["T"], seed + 1)
    M, C = select_sets(grid, spec["n_mon"], spec["n_cont"], seed + 2)
    nB = spec["B"] if B is None else B
    table = []
    if spec["kind"] == "cfg1":
        batch = make_candidates_cfg1(grid, nB, seed + 3)
    elif spec["kind"] == "cfg2":
        batch = make_candidates_cfg2(grid, nB, seed + 3, P=P, move_frac=move_frac)
    else:
        table = make_split_table(grid, 4096, seed + 4)
        batch = make_candidates_ranked(grid, nB, seed + 3, table, P=P, move_frac=move_frac)
    return Workload(cfg=cfg, grid=grid, P=P, M=M, C=C, batch=batch, split_table=table)
