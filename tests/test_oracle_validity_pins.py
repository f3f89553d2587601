"""Pins of the oracle's candidate-validity rules and of its islanding reading.

The expected verdicts are written by hand from the rules (genome of the
Repertoire design section plus the encoding's limits), one rule broken per
invalid row, so a wrong or missing rule in validate_candidate fails a row.
The islanding rows check the reading that a node left without an in-service
branch is an island whatever its injection (the importer's bridge-based
island test, Importer section)."""
import numpy as np
import pytest

import gridgen as gg
import oracle as o
from oracle.dcflow import validate_candidate, post_switch_network, is_connected

import edge_cases as ec


@pytest.mark.parametrize("label,cand,valid", ec.TEN_BUS_TABLE, ids=[r[0] for r in ec.TEN_BUS_TABLE])
def test_validity_table_ten_bus(label, cand, valid):
    g = ec.ten_bus_grid()
    assert validate_candidate(g.n_bus, g.from_bus, g.to_bus, cand) is valid, label


@pytest.mark.parametrize("label,cand,valid", ec.STAR_TABLE, ids=[r[0] for r in ec.STAR_TABLE])
def test_validity_moved_branch_limit(label, cand, valid):
    g = ec.star_grid()
    assert validate_candidate(g.n_bus, g.from_bus, g.to_bus, cand) is valid, label


def test_invalid_candidates_are_not_evaluated():
    g = ec.ten_bus_grid()
    P = np.zeros((g.n_bus, 1))
    for label, cand, valid in ec.TEN_BUS_TABLE:
        r = o.evaluate_candidate(g, P, range(g.n_branch), range(g.n_branch), cand,
                                 gg.default_load_edges(), keep_n1=False)
        assert r.valid is valid, label
        if not valid:
            assert r.cell == -1 and r.fitness == float("-inf") and not r.islanded


def test_table_round_trips_through_the_slot_encoding():
    """The packed batch gives back the same candidates (so GPU tests that use
    the table feed the rows they name)."""
    cands = [c for _, c, _ in ec.TEN_BUS_TABLE]
    b = ec.as_batch(cands, T=1)
    for i, cd in enumerate(cands):
        back = o.candidate_from_batch(b, i)
        assert back.opened == cd.opened
        assert back.splits == cd.splits


def _components(n, fr, to, ins):
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    for e in np.flatnonzero(ins):
        ra, rb = find(int(fr[e])), find(int(to[e]))
        if ra != rb:
            parent[ra] = rb
    return len({find(i) for i in range(n)})


def test_islanding_counts_an_empty_node_without_injection():
    """Opening every branch of a bus with zero injection, or moving every
    branch of a bus away (busbar A left with nothing), leaves a node with no
    branch: islanded, on every path the oracle decides it."""
    g = ec.ten_bus_grid()
    b = 1.0 / g.x_pu
    rng = np.random.default_rng(3)
    P = rng.normal(0, 20, size=(g.n_bus, 2))
    P[3] = 0.0                       # bus 3 carries no injection
    P[0] = 0.0
    P[0] = -P.sum(axis=0)
    cases = [
        ec._c([2, 3, 13, 15], []),                   # all of bus 3's branches opened
        ec._c([], [(3, [2, 3, 13, 15])]),            # all moved to busbar B
    ]
    for cand in cases:
        net = post_switch_network(g.n_bus, g.from_bus, g.to_bus, b, 0, P, cand)
        # an independent union-find count: two components, one of them node 3
        assert _components(net.n_node, net.fr, net.to, net.in_service) == 2
        assert not is_connected(net.n_node, net.fr, net.to, net.in_service)
        r = o.evaluate_candidate(g, P, range(g.n_branch), range(g.n_branch), cand,
                                 gg.default_load_edges(), keep_n1=False)
        assert r.valid and r.islanded and r.cell == -1
    # one branch of bus 3 left in service: connected again
    keep_one = ec._c([2, 3, 13], [])
    r = o.evaluate_candidate(g, P, range(g.n_branch), range(g.n_branch), keep_one,
                             gg.default_load_edges(), keep_n1=False)
    assert r.valid and not r.islanded
    # the injection-free bus 3 hangs on branch 15 alone: it carries nothing
    assert np.abs(r.base_flows[15]).max() < 1e-9


def test_nonfinite_injections_make_candidates_invalid():
    """A NaN or infinite injection (the grid's, or a candidate's moved amount)
    defines no flow: the candidate is invalid and flagged non-finite, after
    the encoding rules and the islanding test have had their say."""
    g = ec.ten_bus_grid()
    rng = np.random.default_rng(4)
    P = rng.normal(0, 20, size=(g.n_bus, 3))
    P[0] = 0.0
    P[0] = -P.sum(axis=0)
    edges = gg.default_load_edges()
    M = C = range(g.n_branch)
    ok = ec._c([0], [(3, [2, 13])])
    bad_code = ec._c([0, 0], [])
    islanded = ec._c([2, 3, 13, 15], [])
    for where in ((4, 1), (0, 0)):
        for v in (np.nan, np.inf, -np.inf):
            Pb = P.copy()
            Pb[where] = v
            r = o.evaluate_candidate(g, Pb, M, C, ok, edges, keep_n1=False)
            assert not r.valid and r.nonfinite and r.cell == -1 and r.fitness == float("-inf")
            r = o.evaluate_candidate(g, Pb, M, C, bad_code, edges, keep_n1=False)
            assert not r.valid and not r.nonfinite
            r = o.evaluate_candidate(g, Pb, M, C, islanded, edges, keep_n1=False)
            assert r.valid and r.islanded and not r.nonfinite
    moved = ec._c([0], [(3, [2, 13])])
    moved.moved_p = [np.array([1.0, np.nan, 2.0])]
    r = o.evaluate_candidate(g, P, M, C, moved, edges, keep_n1=False)
    assert not r.valid and r.nonfinite
    moved.moved_p = [np.array([1.0, -4.0, 2.0])]
    r = o.evaluate_candidate(g, P, M, C, moved, edges, keep_n1=False)
    assert r.valid and not r.islanded and not r.nonfinite


def test_worst_branch_tie_goes_to_the_smaller_position():
    """An exact tie of the maximum loading, resolved by the monitored order:
    on the ten-bus grid with branches 0 (0-1) and 17 (6-8) opened, bus 0 (the
    slack) keeps only branches 9 (9-0) and 10 (0-5), a two-branch cut.  With
    either out, the other carries the slack's whole injection, so both reach
    f^max = |P_0(t)| in exact arithmetic and, with equal 60 MW limits, the same
    loading; rounding alone orders the two computed values (here it puts
    branch 10 ahead), and the tie band must report branch 9.  Closed form:
    rho = max_t |P_0(t)| / 60, t* its timestep."""
    g = ec.ten_bus_grid()
    rng = np.random.default_rng(5)
    P = rng.normal(0, 30, size=(g.n_bus, 3))
    P[0] = 0.0
    P[0] = -P.sum(axis=0)
    cand = ec.TEN_BUS_TABLE[2][1]
    assert sorted(cand.opened) == [0, 17] and not cand.splits
    m = g.n_branch
    r = o.evaluate_candidate(g, P, range(m), range(m), cand, gg.default_load_edges(),
                             keep_n1=False)
    assert r.valid and not r.islanded
    cut = np.abs(P[0])
    np.testing.assert_allclose(r.fmax[9], cut, rtol=1e-12)
    np.testing.assert_allclose(r.fmax[10], cut, rtol=1e-12)
    assert r.metrics["max_loading"] == pytest.approx(cut.max() / 60.0, rel=1e-12)
    assert r.metrics["worst_branch"] == 9
    assert r.metrics["worst_t"] == int(np.argmax(cut))
