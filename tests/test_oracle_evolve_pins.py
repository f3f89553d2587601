"""Pins of oracle/evolve.py against facts outside it: the published Philox
known-answer vectors, exact and library distributions, brute-force
enumeration, the feasibility rules and operation probabilities stated in the
DC-Optimizer section (Mutation, Crossover, High-level loop)."""
from collections import Counter
from decimal import Decimal

import numpy as np
import pytest
from scipy import stats

from oracle import evolve as ev

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def small_space(n_a=4, n_d=4, p_c1=0.5, n_disc=12):
    """Actions at 5 substations with 1..4 actions each (station sizes known)."""
    bus = [7, 3, 7, 9, 3, 7, 11, 9, 7, 5]          # station 3: 2, 5: 1, 7: 4, 9: 2, 11: 1
    moved = [[i, i + 100] for i in range(len(bus))]
    return ev.GenomeSpace(np.array(bus), moved, np.arange(200, 200 + n_disc), n_a, n_d,
                          p_c1=p_c1)


# -------------------------------------------------------------------- RNG
def test_philox_known_answer_vectors():
    """Known-answer vectors published with the Philox4x32-10 reference
    implementation (Random123): counters/keys of all zeros, all ones and the
    hexadecimal digits of pi."""
    assert ev.philox4x32_10([0, 0, 0, 0], [0, 0]) == [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]
    assert ev.philox4x32_10([0xffffffff] * 4, [0xffffffff] * 2) == \
        [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]
    assert ev.philox4x32_10([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344],
                            [0xa4093822, 0x299f31d0]) == \
        [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]


def test_draw_addressing_and_uniformity():
    # word j mod 4 of block j div 4
    w = ev.philox4x32_10((1, 5, 3, 0), (0x1234, 0))
    assert [ev.draw(0x1234, 3, 5, j) for j in (4, 5, 6, 7)] == w
    # 40k draws: uniform on 16 buckets (chi-square), distinct children independent
    r = np.array([ev.draw(99, 1, i, j) for i in range(400) for j in range(100)], dtype=np.uint64)
    h = np.bincount((r >> np.uint64(28)).astype(np.int64), minlength=16)
    assert stats.chisquare(h).pvalue > 1e-4


def test_uniform_index_and_parent_threshold():
    assert ev.uniform_index(0, 7) == 0 and ev.uniform_index(2**32 - 1, 7) == 6
    assert ev.parent1_threshold(1.0) == 2**32 and ev.parent1_threshold(0.0) == 0
    assert ev.parent1_threshold(0.5) == 2**31


def test_poisson_table_exact_and_distribution():
    """FP64 table equals 60-digit arithmetic; the clipped law matches scipy's
    Poisson pmf with the tail folded into N_a and P(0) into 1."""
    for mean in (2.0, 0.5, 3.7):
        for n_a in (1, 3, 8):
            assert ev.poisson_thresholds(mean, n_a) == \
                ev.poisson_thresholds_exact(Decimal(repr(mean)), n_a)
    n_a, mean = 5, 2.0
    thr = ev.poisson_thresholds(mean, n_a)
    rng = np.random.default_rng(1)
    r = rng.integers(0, 2**32, size=200000, dtype=np.uint64)
    k = np.array([ev.clipped_poisson(int(x), thr, n_a) for x in r])
    pmf = stats.poisson(mean).pmf(np.arange(n_a + 1))
    want = np.zeros(n_a + 1)
    want[1] = pmf[0] + pmf[1]
    want[2:n_a] = pmf[2:n_a]
    want[n_a] = 1.0 - want[1:n_a].sum()
    got = np.bincount(k, minlength=n_a + 1) / len(k)
    assert got[0] == 0
    assert np.all(np.abs(got[1:] - want[1:]) < 5 * np.sqrt(want[1:] / len(k)) + 1e-4)
    assert ev.clipped_poisson(2**32 - 1, thr, n_a) == n_a and ev.clipped_poisson(0, thr, n_a) == 1
    assert ev.clipped_poisson(123, [], 0) == 0


def test_complement_element_brute_force():
    rng = np.random.default_rng(2)
    for _ in range(200):
        n = int(rng.integers(1, 40))
        k = min(int(rng.integers(0, 6)) * 2, (n + 1) // 2 * 2)
        cut = sorted(rng.choice(np.arange(n + 1), size=k, replace=False))
        ranges = [(int(cut[i]), int(cut[i + 1] - cut[i])) for i in range(0, len(cut), 2)
                  if cut[i + 1] > cut[i]]
        covered = {x for s, ln in ranges for x in range(s, s + ln)}
        comp = [x for x in range(n) if x not in covered]
        rng.shuffle(ranges)
        assert [ev._complement_element(u, list(ranges)) for u in range(len(comp))] == comp


# -------------------------------------------------------------------- Alg. 1
def _feasible(gs, g):
    a, d = g[:gs.n_a], g[gs.n_a:]
    acts = [v for v in a if v != -1]
    disc = [v for v in d if v != -1]
    return (all(0 <= v < gs.n_actions for v in acts) and all(0 <= v < gs.n_disc for v in disc)
            and len({gs.bus(v) for v in acts}) == len(acts) and len(set(disc)) == len(disc))


def _random_genome(gs, rng):
    a = [-1] * gs.n_a
    stations = sorted(gs.count)
    for j, q in enumerate(rng.permutation(stations)[: int(rng.integers(0, gs.n_a + 1))]):
        a[j] = int(gs.station_order[gs.first[int(q)] + int(rng.integers(0, gs.count[int(q)]))])
    d = [-1] * gs.n_d
    k = int(rng.integers(0, gs.n_d + 1))
    d[:k] = [int(x) for x in rng.choice(gs.n_disc, size=k, replace=False)]
    rng.shuffle(a)
    rng.shuffle(d)
    return a + d


def _classify(before, after):
    fb = sum(v != -1 for v in before)
    fa = sum(v != -1 for v in after)
    if fa == fb + 1:
        return ev.ADD
    if fa == fb - 1:
        return ev.REMOVE
    return ev.CHANGE if before != after else ev.IDENTITY


def test_action_step_operation_frequencies_match_paper_weights():
    """Mutation: p_add 0.2, p_remove 0.2, p_change 0.5, p_identity 0.1 when all
    four are feasible; renormalised over the feasible ones otherwise."""
    gs = small_space()
    rng = np.random.default_rng(3)
    a0 = [gs.station_order[gs.first[7]], -1, gs.station_order[gs.first[3]], -1]
    n = 40000
    cnt = Counter()
    for _ in range(n):
        a = list(a0)
        ev.action_step(gs, a, *[int(x) for x in rng.integers(0, 2**32, size=3)])
        cnt[_classify(a0, a)] += 1
    for op, p in ((ev.ADD, .2), (ev.REMOVE, .2), (ev.CHANGE, .5), (ev.IDENTITY, .1)):
        assert abs(cnt[op] / n - p) < 5 * np.sqrt(p * (1 - p) / n)
    # every slot full: Add infeasible -> remove .25, change .625, identity .125
    a1 = [gs.station_order[gs.first[q]] for q in (3, 7, 9, 5)]
    cnt = Counter()
    for _ in range(n):
        a = list(a1)
        ev.action_step(gs, a, *[int(x) for x in rng.integers(0, 2**32, size=3)])
        cnt[_classify(a1, a)] += 1
    for op, p in ((ev.ADD, 0.0), (ev.REMOVE, .25), (ev.CHANGE, .625), (ev.IDENTITY, .125)):
        assert abs(cnt[op] / n - p) < 5 * np.sqrt(p * (1 - p) / n) + 1e-9


def test_action_add_and_change_are_uniform_over_their_sets():
    """Add samples A minus every action of an already split substation;
    Change samples the other actions of already split substations and
    replaces the slot of that substation."""
    gs = small_space()
    a0 = [gs.station_order[gs.first[7]], -1, -1, -1]        # station 7 split (4 actions)
    add_set = sorted(a for a in range(gs.n_actions) if gs.bus(a) != 7)
    chg_set = sorted(a for a in range(gs.n_actions) if gs.bus(a) == 7 and a != a0[0])
    seen_add, seen_chg = Counter(), Counter()
    rng = np.random.default_rng(4)
    for _ in range(30000):
        a = list(a0)
        ev.action_step(gs, a, *[int(x) for x in rng.integers(0, 2**32, size=3)])
        op = _classify(a0, a)
        if op == ev.ADD:
            new = [v for v in a if v != -1 and v != a0[0]]
            assert len(new) == 1 and a[0] == a0[0]
            seen_add[new[0]] += 1
        elif op == ev.CHANGE:
            assert a[1:] == [-1, -1, -1]
            seen_chg[a[0]] += 1
    assert sorted(seen_add) == add_set and sorted(seen_chg) == chg_set
    assert stats.chisquare([seen_add[v] for v in add_set]).pvalue > 1e-4
    assert stats.chisquare([seen_chg[v] for v in chg_set]).pvalue > 1e-4


def test_change_infeasible_when_split_stations_have_one_action():
    gs = small_space()
    a0 = [gs.station_order[gs.first[5]], -1, gs.station_order[gs.first[11]], -1]
    rng = np.random.default_rng(5)
    for _ in range(3000):
        a = list(a0)
        ev.action_step(gs, a, *[int(x) for x in rng.integers(0, 2**32, size=3)])
        assert _classify(a0, a) != ev.CHANGE


def test_disconnection_step_frequencies_and_sets():
    """Disconnection mutation: p_add .25, p_remove .25, p_change .5,
    p_identity 0; Add and Change draw from D minus the current entries."""
    gs = small_space(n_disc=6)
    d0 = [2, -1, 5, -1]
    n = 40000
    cnt = Counter()
    rng = np.random.default_rng(6)
    for _ in range(n):
        d = list(d0)
        ev.disc_step(gs, d, False, *[int(x) for x in rng.integers(0, 2**32, size=3)])
        op = _classify(d0, d)
        cnt[op] += 1
        full = [v for v in d if v != -1]
        assert len(set(full)) == len(full)
        if op == ev.ADD:
            assert set(d0) - {-1} < set(full) and (set(full) - {2, 5}) <= {0, 1, 3, 4}
        if op == ev.CHANGE:
            assert len(full) == 2 and len(set(full) & {2, 5}) == 1
    for op, p in ((ev.ADD, .25), (ev.REMOVE, .25), (ev.CHANGE, .5), (ev.IDENTITY, 0.0)):
        assert abs(cnt[op] / n - p) < 5 * np.sqrt(p * (1 - p) / n) + 1e-9


def test_mutation_of_the_empty_individual_forces_a_disconnection():
    """An individual with neither split nor disconnection gets an Add in the
    disconnection step (the unchanged default topology is not reproduced)."""
    gs = small_space(n_a=0, n_d=3)
    for i in range(500):
        child = ev.mutate(gs, [-1] * 3, lambda j, i=i: ev.draw(7, 0, i, j))
        assert sum(v != -1 for v in child) == 1


def test_mutation_keeps_feasibility_and_n_mut_range():
    gs = small_space()
    rng = np.random.default_rng(8)
    for i in range(3000):
        parent = _random_genome(gs, rng)
        child = ev.mutate(gs, parent, lambda j, i=i: ev.draw(11, 2, i, j))
        assert _feasible(gs, child) and len(child) == gs.n_a + gs.n_d


# -------------------------------------------------------------------- Alg. 2
def test_crossover_bias_reproduces_a_parent():
    """p_c1 = 1 reproduces (a1, d1) and p_c1 = 0 reproduces (a2, d2) (slot
    order aside); identical parents reproduce themselves."""
    rng = np.random.default_rng(9)
    for p_c1, which in ((1.0, 0), (0.0, 1)):
        gs = small_space(p_c1=p_c1)
        for i in range(500):
            g1, g2 = _random_genome(gs, rng), _random_genome(gs, rng)
            child = ev.crossover(gs, g1, g2, lambda j, i=i: ev.draw(13, 0, i, j))
            want = (g1, g2)[which]
            assert sorted(child[:4]) == sorted(want[:4]) and sorted(child[4:]) == sorted(want[4:])
    gs = small_space(p_c1=0.3)
    for i in range(300):
        g = _random_genome(gs, rng)
        child = ev.crossover(gs, g, g, lambda j, i=i: ev.draw(17, 0, i, j))
        assert sorted(child[:4]) == sorted(g[:4]) and sorted(child[4:]) == sorted(g[4:])


def test_crossover_draws_from_the_union_with_bias_p_c1():
    """Children hold only parent entries, stay feasible, and with disjoint
    full parents each child entry comes from parent 1 with probability p_c1."""
    gs = small_space(p_c1=0.75, n_disc=40)
    g1 = [gs.station_order[gs.first[q]] for q in (3, 7)] + [-1, -1] + [0, 1, 2, 3]
    g2 = [gs.station_order[gs.first[q]] for q in (9, 5)] + [-1, -1] + [10, 11, 12, 13]
    from_1 = tot = 0
    for i in range(4000):
        child = ev.crossover(gs, g1, g2, lambda j, i=i: ev.draw(19, 0, i, j))
        assert _feasible(gs, child)
        for v, pool1, pool2 in ((c, g1[:4], g2[:4]) for c in child[:4]):
            assert v in pool1 or v in pool2
        for v in child[4:]:
            assert v in g1[4:] + g2[4:]
            from_1 += v in g1[4:]
            tot += 1
    assert abs(from_1 / tot - 0.75) < 5 * np.sqrt(0.75 * 0.25 / tot)
    # same substation in both parents: the child splits it at most once
    rng = np.random.default_rng(10)
    gs = small_space(p_c1=0.5)
    for i in range(2000):
        g1, g2 = _random_genome(gs, rng), _random_genome(gs, rng)
        assert _feasible(gs, ev.crossover(gs, g1, g2, lambda j, i=i: ev.draw(23, 1, i, j)))


# -------------------------------------------------------------------- Alg. 3
def test_vary_split_and_parent_sampling():
    """b_mc is uniform on 0..b; parents come from occupied cells only; the
    empty repertoire yields mutations of the empty individual."""
    gs = small_space()
    b = 6
    seen = Counter(ev.vary(gs, np.full(4, -1), np.full((4, 8), -1), 31, g, b)[1]
                   for g in range(1400))
    assert sorted(seen) == list(range(b + 1))
    assert stats.chisquare([seen[k] for k in range(b + 1)]).pvalue > 1e-4
    kids, b_mc = ev.vary(gs, np.full(4, -1), np.full((4, 8), -1), 5, 3, 64)
    for i, k in enumerate(kids):
        if i < b_mc:
            assert sum(v != -1 for v in k[4:]) >= 1
        else:
            assert np.all(k == -1)
    rng = np.random.default_rng(12)
    eg = np.array([_random_genome(gs, rng) for _ in range(6)], dtype=np.int32)
    eid = np.array([-1, 4, -1, -1, 9, -1])
    kids, b_mc = ev.vary(ev.GenomeSpace(gs.action_bus, gs.action_moved, gs.disc_branch, 4, 4,
                                        p_c1=1.0), eid, eg, 5, 0, 200)
    for i in range(b_mc, 200):
        assert any(sorted(kids[i][:4]) == sorted(eg[c][:4]) and
                   sorted(kids[i][4:]) == sorted(eg[c][4:]) for c in (1, 4))


def test_expand_maps_ids_and_marks_out_of_range():
    """Ids map to buses / branch ids, out-of-range ids to -2; slots come out
    in canonical order (by bus, by branch id; invalid, then empty last)."""
    gs = small_space()
    g = np.array([[3, -1, 0, 99, 2, -1, 55, 0]], dtype=np.int32)
    opens, sbus, moved = ev.expand(gs, g)
    assert sbus.tolist() == [[7, 9, -2, -1]]
    assert moved == [[0, 100], [3, 103], [], []]
    assert opens.tolist() == [[200, 202, -2, -1]]


def test_expand_is_invariant_under_slot_permutations():
    gs = small_space()
    rng = np.random.default_rng(14)
    for _ in range(200):
        g = np.array(_random_genome(gs, rng), dtype=np.int32)
        perm = np.concatenate([rng.permutation(4), 4 + rng.permutation(4)])
        a, b = ev.expand(gs, g[None]), ev.expand(gs, g[perm][None])
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_archive_with_genomes_matches_sequential_insertion():
    from oracle.metrics import archive_insert_sequential
    rng = np.random.default_rng(13)
    n_cells, G = 16, 5
    fit0 = rng.normal(size=n_cells)
    id0 = np.where(rng.random(n_cells) < .5, -1, np.arange(n_cells))
    gen0 = rng.integers(-1, 9, size=(n_cells, G))
    f = np.round(rng.normal(size=300), 1)            # many ties
    cells = rng.integers(0, n_cells, size=300)
    ok = rng.random(300) < .9
    kids = rng.integers(-1, 9, size=(300, G))
    bf, bi, bg = ev.archive_insert_genomes(fit0, id0, gen0, f, cells, ok, kids, 1000)
    rf, ri = archive_insert_sequential(fit0, id0, f, cells, ok, 1000)
    assert np.array_equal(bf, rf) and np.array_equal(bi, ri)
    for c in range(n_cells):
        if bi[c] >= 1000:
            assert np.array_equal(bg[c], kids[bi[c] - 1000])
        else:
            assert np.array_equal(bg[c], gen0[c])


def test_generation_loop_bookkeeping_on_30_bus_grid():
    """Three generations on the 30-bus grid: every elite's genome, expanded
    and re-evaluated from scratch, gives back its fitness and cell; elites
    only improve; ids name the generation and child that produced them."""
    import gridgen
    from oracle.dcflow import evaluate_candidate
    grid = gridgen.make_grid(30, 41, seed=0x5EED0001)
    P = gridgen.make_injections(grid, 1, seed=0x5EED0001)
    M = C = np.arange(41)
    D = np.flatnonzero(~gridgen.bridges(grid.n_bus, grid.from_bus, grid.to_bus))
    table = gridgen.make_split_table(grid, 24, seed=5)
    gs = ev.GenomeSpace(np.array([b for b, _ in table]), [mv for _, mv in table], D, 2, 2)
    edges = np.geomspace(0.25, 64, 31)
    state, log = ev.run_generations(grid, P, M, C, gs, 77, 3, 16, edges, 1024)
    fit, ids, gen = state
    assert (ids >= 0).sum() >= 3
    first = log[0]      # generation 0 starts from the empty repertoire
    assert np.all((first["children"][: first["b_mc"], 2:] != -1).sum(axis=1) >= 1)
    assert np.all(first["children"][first["b_mc"]:] == -1)
    for c in np.flatnonzero(ids >= 0):
        g, i = divmod(int(ids[c]), 16)
        assert np.array_equal(gen[c], log[g]["children"][i])
        cd = ev.to_candidates(gs, gen[c][None, :])[0]
        r = evaluate_candidate(grid, P, M, C, cd, edges, keep_n1=False)
        assert r.cell == c and r.fitness == fit[c]
        # best of its cell over every generation's valid children
        allf = [rec["fitness"][k] for rec in log for k in range(16)
                if rec["ok"][k] and rec["cell"][k] == c]
        assert fit[c] == max(allf)


def test_feasible_parent_reads_conflicts_as_empty():
    gs = small_space()
    a7, a7b = gs.station_order[gs.first[7]], gs.station_order[gs.first[7] + 1]
    g = [a7, 99, a7b, -5, 3, 3, 40, -1]
    assert ev.feasible_parent(gs, g) == [a7, -1, -1, -1, 3, -1, -1, -1]
