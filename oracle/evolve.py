"""Oracle of one MapElites generation: variation, genome expansion, insertion.

TEST INFRASTRUCTURE ONLY (see the package docstring): the test suite, the
package smoke check and the benchmark's CPU-baseline leg may use it; nothing
on the product path does.

What it follows (DC-Optimizer section of the paper):
  - Repertoire design: an individual holds N_a action slots (ids into the
    split-action set A, each action belonging to one substation) and N_d
    disconnection slots (ids into the disconnectable-branch set D); -1 is the
    empty slot; actions of one individual sit at distinct substations and
    disconnections name distinct branches.
  - Mutation (Alg. 1): a Poisson(N_mutmean) number of action steps clipped to
    [1, N_a], then one disconnection step; each step draws one feasible
    operation among Add / Remove / Change / Identity with the weights the
    paper gives (actions 0.2 / 0.2 / 0.5 / 0.1, disconnections
    0.25 / 0.25 / 0.5 / 0), Add forced for the disconnection step when the
    individual holds nothing.  Action Change picks a different action at a
    substation the individual already splits.
  - Crossover (Alg. 2): each child slot samples from what is left of the two
    parents (each parent a list of its slot entries, empty ones included):
    parent 1 with probability p_c1 (the other one when a parent has nothing
    left), then one of that parent's remaining entries uniformly; taking an
    entry also removes one equal entry from the other parent, so the union
    counts shared entries once; an action whose substation the child already
    splits becomes the empty slot.
  - High-level loop (Alg. 3): per generation a mutation/crossover split
    b_mc ~ U{0..b}; parents uniform over the occupied cells (the empty
    individual while the repertoire is empty); evaluation; one elite per
    cell, strictly-better replacement.  A parent is first made feasible:
    out-of-range entries, actions at a substation an earlier slot already
    splits and repeated disconnections read as empty.

Random numbers.  The method draws random numbers whose count depends on the
state (feasible operations, pool sizes), so they cannot be handed in as an
array.  Both this oracle and the device implement the same counter-based
generator, Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC 2011), from its published definition, and
address draws by position:

    word (j mod 4) of Philox4x32-10(counter = (j div 4, i, g mod 2^32,
    g div 2^32), key = (seed mod 2^32, seed div 2^32))

for draw j of child i in generation g; the generation-level draw (b_mc) uses
i = 0xFFFFFFFF.  A draw r in [0, 2^32) becomes an index in [0, n) as
(r * n) div 2^32 and a parent-1 choice as r < floor(p_c1 * 2^32).  Draw
positions: 0 and 1 pick the parents; mutation uses 2 for N_mut, 3 + 3s,
4 + 3s, 5 + 3s for action step s (operation, slot, item) and 3 + 3 N_a ..
5 + 3 N_a for the disconnection step; crossover uses 2 + 2i, 3 + 2i for
action slot i (parent, entry) and 2 + 2 N_a + 2i, 3 + 2 N_a + 2i for
disconnection slot i.

Orders.  "The u-th element" of a set of actions means in station order:
ascending (bus, action id); of a set of disconnections, ascending D index;
"the u-th empty/filled slot" counts slots in ascending slot index.

Pins: tests/test_oracle_evolve_pins.py (published Philox known-answer
vectors, the exact clipped-Poisson table, brute-force complements,
feasibility invariants, operation frequencies against the paper's weights,
the p_c1 = 1 / 0 reproductions, the generation loop against sequential
insertion).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from decimal import Decimal, getcontext
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

M32 = 0xFFFFFFFF
GEN_CHILD = 0xFFFFFFFF          # child index of the generation-level draw

# operation order used by the weighted choice
ADD, REMOVE, CHANGE, IDENTITY = 0, 1, 2, 3


# ---------------------------------------------------------------- Philox4x32-10
def _mulhilo(a: int, b: int) -> Tuple[int, int]:
    p = a * b
    return (p >> 32) & M32, p & M32


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> List[int]:
    """Ten rounds of Philox4x32 (multipliers 0xD2511F53, 0xCD9E8D57; key
    schedule by the Weyl constants 0x9E3779B9, 0xBB67AE85)."""
    c0, c1, c2, c3 = (int(v) & M32 for v in ctr)
    k0, k1 = (int(v) & M32 for v in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + 0x9E3779B9) & M32
            k1 = (k1 + 0xBB67AE85) & M32
        hi0, lo0 = _mulhilo(0xD2511F53, c0)
        hi1, lo1 = _mulhilo(0xCD9E8D57, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return [c0, c1, c2, c3]


def draw(seed: int, gen: int, child: int, j: int) -> int:
    """Draw j of `child` in generation `gen` (see the module docstring)."""
    w = philox4x32_10((j >> 2, child & M32, gen & M32, (gen >> 32) & M32),
                      (seed & M32, (seed >> 32) & M32))
    return w[j & 3]


def uniform_index(r: int, n: int) -> int:
    return (r * n) >> 32


def parent1_threshold(p_c1: float) -> int:
    return min(1 << 32, int(math.floor(p_c1 * 4294967296.0)))


def poisson_thresholds(mean: float, n_a: int) -> List[int]:
    """floor(P(K <= k) * 2^32) for k = 1 .. n_a - 1, K ~ Poisson(mean), in FP64."""
    out = []
    term = math.exp(-mean)
    cdf = term
    for k in range(1, max(n_a, 1)):
        term = term * mean / k
        cdf += term
        out.append(int(math.floor(cdf * 4294967296.0)))
    return out


def poisson_thresholds_exact(mean: Decimal, n_a: int, digits: int = 60) -> List[int]:
    """The same table from 60-digit decimal arithmetic (used as a pin)."""
    getcontext().prec = digits
    e = (-mean).exp()
    out, term, cdf = [], e, e
    for k in range(1, max(n_a, 1)):
        term = term * mean / k
        cdf += term
        out.append(int((cdf * (1 << 32)).to_integral_value(rounding="ROUND_FLOOR")))
    return out


def clipped_poisson(r: int, thresholds: Sequence[int], n_a: int) -> int:
    """N_mut = clip(K, 1, n_a) by inversion of the CDF table."""
    if n_a <= 0:
        return 0
    return 1 + sum(1 for t in thresholds[: n_a - 1] if r >= t)


# ---------------------------------------------------------------- genome tables
@dataclass
class GenomeSpace:
    """Action set A (bus and moved branches per action), set D, slot counts
    and the operator parameters."""
    action_bus: np.ndarray               # [|A|]
    action_moved: List[List[int]]        # per action, moved branch ids
    disc_branch: np.ndarray              # [|D|] branch ids
    n_a: int
    n_d: int
    mut_mean: float = 2.0
    w_action: Tuple[int, int, int, int] = (20, 20, 50, 10)   # add, remove, change, identity
    w_disc: Tuple[int, int, int, int] = (25, 25, 50, 0)
    p_c1: float = 0.5

    def __post_init__(self):
        self.action_bus = np.asarray(self.action_bus, dtype=np.int64)
        self.disc_branch = np.asarray(self.disc_branch, dtype=np.int64)
        n = len(self.action_bus)
        self.station_order = sorted(range(n), key=lambda a: (int(self.action_bus[a]), a))
        self.pos = [0] * n
        for p, a in enumerate(self.station_order):
            self.pos[a] = p
        self.first = {}
        self.count = {}
        for p, a in enumerate(self.station_order):
            q = int(self.action_bus[a])
            self.first.setdefault(q, p)
            self.count[q] = self.count.get(q, 0) + 1
        self.poisson = poisson_thresholds(self.mut_mean, self.n_a)
        self.thr_c1 = parent1_threshold(self.p_c1)

    @property
    def n_actions(self) -> int:
        return len(self.action_bus)

    @property
    def n_disc(self) -> int:
        return len(self.disc_branch)

    def bus(self, a: int) -> int:
        return int(self.action_bus[a])


def _kth(slots: Sequence[int], k: int, empty: bool) -> int:
    """Slot index of the k-th empty (or filled) slot, ascending."""
    seen = 0
    for i, v in enumerate(slots):
        if (v == -1) == empty:
            if seen == k:
                return i
            seen += 1
    raise IndexError("slot rank out of range")


def _complement_element(u: int, excluded_ranges: List[Tuple[int, int]]) -> int:
    """The u-th integer (from 0) not covered by the disjoint [start, start+len)
    ranges: shift u past every range that starts at or before it."""
    x = u
    for start, ln in sorted(excluded_ranges):
        if x >= start:
            x += ln
    return x


def _weighted(r: int, weights: Sequence[int], feasible: Sequence[bool]) -> Optional[int]:
    w = [wt if ok else 0 for wt, ok in zip(weights, feasible)]
    tot = sum(w)
    if tot == 0:
        return None
    x = uniform_index(r, tot)
    acc = 0
    for op, wt in enumerate(w):
        acc += wt
        if x < acc:
            return op
    raise AssertionError("unreachable")


# ---------------------------------------------------------------- Alg. 1
def action_step(gs: GenomeSpace, a: List[int], r_op: int, r_slot: int, r_item: int) -> None:
    """One action mutation step in place."""
    full = [v for v in a if v != -1]
    n_empty = len(a) - len(full)
    used = [gs.bus(v) for v in full]
    n_add = gs.n_actions - sum(gs.count[q] for q in used)
    n_chg = sum(gs.count[q] - 1 for q in used)
    op = _weighted(r_op, gs.w_action,
                   (n_empty >= 1 and n_add >= 1, len(full) >= 1, n_chg >= 1, True))
    if op == ADD:
        slot = _kth(a, uniform_index(r_slot, n_empty), True)
        p = _complement_element(uniform_index(r_item, n_add),
                                [(gs.first[q], gs.count[q]) for q in used])
        a[slot] = gs.station_order[p]
    elif op == REMOVE:
        slot = _kth(a, uniform_index(r_slot, len(full)), False)
        a[slot] = -1
    elif op == CHANGE:
        u = uniform_index(r_item, n_chg)
        for j, v in enumerate(a):
            if v == -1:
                continue
            q = gs.bus(v)
            c = gs.count[q] - 1
            if u < c:
                own = gs.pos[v] - gs.first[q]
                a[j] = gs.station_order[gs.first[q] + u + (1 if u >= own else 0)]
                return
            u -= c
        raise AssertionError("change rank out of range")


def disc_step(gs: GenomeSpace, d: List[int], force_add: bool, r_op: int, r_slot: int,
              r_item: int) -> None:
    """One disconnection mutation step in place (entries are D indices)."""
    full = [v for v in d if v != -1]
    n_empty = len(d) - len(full)
    n_add = gs.n_disc - len(full)
    feas = (n_empty >= 1 and n_add >= 1, len(full) >= 1, len(full) >= 1 and n_add >= 1, True)
    if force_add and feas[ADD]:
        op = ADD
    else:
        op = _weighted(r_op, gs.w_disc, feas)
    if op == ADD:
        slot = _kth(d, uniform_index(r_slot, n_empty), True)
        d[slot] = _complement_element(uniform_index(r_item, n_add), [(v, 1) for v in full])
    elif op == REMOVE:
        slot = _kth(d, uniform_index(r_slot, len(full)), False)
        d[slot] = -1
    elif op == CHANGE:
        item = _complement_element(uniform_index(r_item, n_add), [(v, 1) for v in full])
        slot = _kth(d, uniform_index(r_slot, len(full)), False)
        d[slot] = item


def mutate(gs: GenomeSpace, parent: Sequence[int], rnd: Callable[[int], int]) -> List[int]:
    """Alg. 1 on a genome [N_a action ids | N_d disconnection ids]."""
    a = [int(v) for v in parent[: gs.n_a]]
    d = [int(v) for v in parent[gs.n_a: gs.n_a + gs.n_d]]
    n_mut = clipped_poisson(rnd(2), gs.poisson, gs.n_a)
    for s in range(n_mut):
        action_step(gs, a, rnd(3 + 3 * s), rnd(4 + 3 * s), rnd(5 + 3 * s))
    j = 3 + 3 * gs.n_a
    empty = all(v == -1 for v in a) and all(v == -1 for v in d)
    disc_step(gs, d, empty, rnd(j), rnd(j + 1), rnd(j + 2))
    return a + d


# ---------------------------------------------------------------- Alg. 2
def _cross_part(p1: List[int], p2: List[int], thr: int, rnd: Callable[[int], int], j0: int,
                station: Optional[Callable[[int], int]]) -> List[int]:
    rem = [list(p1), list(p2)]
    child: List[int] = []
    taken_st = set()
    for i in range(len(p1)):
        side = 0 if rnd(j0 + 2 * i) < thr else 1
        if not rem[side]:
            side = 1 - side
        if not rem[side]:
            child.append(-1)
            continue
        k = uniform_index(rnd(j0 + 2 * i + 1), len(rem[side]))
        v = rem[side].pop(k)
        other = rem[1 - side]
        if v in other:                  # the union matches equal entries, empty ones too
            other.remove(v)
        if v != -1:
            if station is not None:
                q = station(v)
                if q in taken_st:
                    v = -1
                else:
                    taken_st.add(q)
        child.append(v)
    return child


def crossover(gs: GenomeSpace, g1: Sequence[int], g2: Sequence[int],
              rnd: Callable[[int], int]) -> List[int]:
    """Alg. 2: actions then disconnections."""
    na, nd = gs.n_a, gs.n_d
    a = _cross_part([int(v) for v in g1[:na]], [int(v) for v in g2[:na]], gs.thr_c1, rnd, 2,
                    gs.bus)
    d = _cross_part([int(v) for v in g1[na:na + nd]], [int(v) for v in g2[na:na + nd]],
                    gs.thr_c1, rnd, 2 + 2 * na, None)
    return a + d


# ---------------------------------------------------------------- Alg. 3
def feasible_parent(gs: GenomeSpace, genome: Sequence[int]) -> List[int]:
    a, d = [], []
    for v in (int(x) for x in genome[: gs.n_a]):
        if not 0 <= v < gs.n_actions or gs.bus(v) in {gs.bus(u) for u in a if u != -1}:
            v = -1
        a.append(v)
    for v in (int(x) for x in genome[gs.n_a: gs.n_a + gs.n_d]):
        if not 0 <= v < gs.n_disc or v in d:
            v = -1
        d.append(v)
    return a + d


def vary(gs: GenomeSpace, elite_id: np.ndarray, elite_genome: np.ndarray, seed: int, gen: int,
         n_child: int) -> Tuple[np.ndarray, int]:
    """Children genomes [n_child][N_a + N_d] and b_mc of generation `gen`."""
    G = gs.n_a + gs.n_d
    occ = [c for c in range(len(elite_id)) if elite_id[c] != -1]
    b_mc = uniform_index(draw(seed, gen, GEN_CHILD, 0), n_child + 1)
    out = np.full((n_child, G), -1, dtype=np.int32)
    empty = [-1] * G
    for i in range(n_child):
        def rnd(j, i=i):
            return draw(seed, gen, i, j)

        def pick(j):
            if not occ:
                return empty
            return feasible_parent(gs, elite_genome[occ[uniform_index(rnd(j), len(occ))]])

        if i < b_mc:
            out[i] = mutate(gs, pick(0), rnd)
        else:
            out[i] = crossover(gs, pick(0), pick(1), rnd)
    return out, b_mc


def _canonical(vals: Sequence[int], n: int, site) -> List[int]:
    """Slots in canonical order: valid ids ascending by (site, id), then
    out-of-range ids (in slot order), then empty slots."""
    valid = sorted((v for v in vals if 0 <= v < n), key=lambda v: (int(site[v]), v))
    bad = [v for v in vals if v != -1 and not 0 <= v < n]
    return valid + bad + [-1] * (len(vals) - len(valid) - len(bad))


def expand(gs: GenomeSpace, genomes: np.ndarray):
    """Genomes -> (open [n][N_d] branch ids, split_bus [n][N_a], moved lists
    per (candidate, slot)), slots in canonical order (actions by bus,
    disconnections by branch id, then invalid entries, then empty slots), so
    that a candidate's evaluation does not depend on its slot order.
    Out-of-range ids become -2 (an invalid slot)."""
    genomes = np.asarray(genomes)
    n = genomes.shape[0]
    na, nd = gs.n_a, gs.n_d
    opens = np.full((n, nd), -1, dtype=np.int32)
    sbus = np.full((n, na), -1, dtype=np.int32)
    moved: List[List[int]] = []
    for c in range(n):
        acts = _canonical([int(v) for v in genomes[c, :na]], gs.n_actions, gs.action_bus)
        for j, v in enumerate(acts):
            if v == -1:
                moved.append([])
            elif 0 <= v < gs.n_actions:
                sbus[c, j] = gs.bus(v)
                moved.append(list(gs.action_moved[v]))
            else:
                sbus[c, j] = -2
                moved.append([])
        discs = _canonical([int(v) for v in genomes[c, na:na + nd]], gs.n_disc, gs.disc_branch)
        for j, v in enumerate(discs):
            if v == -1:
                continue
            opens[c, j] = int(gs.disc_branch[v]) if 0 <= v < gs.n_disc else -2
    return opens, sbus, moved


def archive_insert_genomes(best_fit, best_id, best_genome, fitness, cells, ok, genomes,
                           id_base: int):
    """Sequential one-at-a-time insertion (High-level loop) that also keeps
    the elite's genome."""
    best_fit = np.array(best_fit, dtype=np.float64, copy=True)
    best_id = np.array(best_id, dtype=np.int64, copy=True)
    best_genome = np.array(best_genome, dtype=np.int32, copy=True)
    for i in range(len(fitness)):
        if not ok[i]:
            continue
        c = int(cells[i])
        if best_id[c] == -1 or fitness[i] > best_fit[c]:
            best_fit[c] = fitness[i]
            best_id[c] = id_base + i
            best_genome[c] = genomes[i]
    return best_fit, best_id, best_genome


def to_candidates(gs: GenomeSpace, genomes: np.ndarray):
    """Oracle candidates (dcflow.Candidate) of expanded genomes."""
    from .dcflow import Candidate
    opens, sbus, moved = expand(gs, genomes)
    out = []
    for c in range(opens.shape[0]):
        op = [int(v) for v in opens[c] if v != -1]
        sp = [(int(sbus[c, j]), moved[c * gs.n_a + j]) for j in range(gs.n_a) if sbus[c, j] != -1]
        out.append(Candidate(opened=op, splits=sp, moved_p=[None] * len(sp),
                             n_slots_filled=len(op) + len(sp)))
    return out


def run_generations(grid, P, M, C, gs: GenomeSpace, seed: int, n_gen: int, n_child: int,
                    load_edges, n_cells: int, n_count_bins: int = 32, gen0: int = 0,
                    state=None):
    """Alg. 3 for n_gen generations from `state` (fitness, id, genome per
    cell; an empty repertoire if None): vary, evaluate every child with the
    FP64 re-solve oracle, insert one at a time with ids gen * n_child + i."""
    from .dcflow import evaluate_candidate
    G = gs.n_a + gs.n_d
    if state is None:
        state = (np.full(n_cells, -np.inf), np.full(n_cells, -1, dtype=np.int64),
                 np.full((n_cells, G), -1, dtype=np.int32))
    fit, ids, gen = state
    log = []
    for g in range(gen0, gen0 + n_gen):
        kids, b_mc = vary(gs, ids, gen, seed, g, n_child)
        res = [evaluate_candidate(grid, P, M, C, cd, load_edges, n_count_bins=n_count_bins,
                                  keep_n1=False) for cd in to_candidates(gs, kids)]
        ok = np.array([r.valid and not r.islanded for r in res])
        f = np.array([r.fitness for r in res])
        cells = np.array([r.cell for r in res])
        fit, ids, gen = archive_insert_genomes(fit, ids, gen, f, cells, ok, kids, g * n_child)
        log.append(dict(children=kids, b_mc=b_mc, fitness=f, cell=cells, ok=ok))
    return (fit, ids, gen), log
