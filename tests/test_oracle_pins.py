"""Pins for the FP64 oracle: every check compares it with something that does
not come from the oracle (closed forms, Kirchhoff's laws, independent graph
search, the textbook distribution-factor formulas, hand-worked fixtures)."""
import itertools
import json
import os
from collections import deque

import numpy as np
import pytest

import gridgen as gg
import oracle as o
from oracle.dcflow import Candidate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _flows(grid, P, in_service=None, slack=0):
    b = 1.0 / grid.x_pu
    ins = np.ones(grid.n_branch, bool) if in_service is None else in_service
    return o.solve_flows(grid.n_bus, grid.from_bus, grid.to_bus, b, ins, P, slack)


def _bfs_component(n, fr, to, in_service, start):
    adj = [[] for _ in range(n)]
    for e in range(len(fr)):
        if in_service[e]:
            adj[fr[e]].append(to[e])
            adj[to[e]].append(fr[e])
    seen = {start}
    q = deque([start])
    while q:
        u = q.popleft()
        for v in adj[u]:
            if v not in seen:
                seen.add(v)
                q.append(v)
    return seen


def _balanced(rng, n, T=1, slack=0):
    P = rng.normal(0, 40, size=(n, T))
    P[slack] = 0.0
    P[slack] = -P.sum(axis=0)
    return P


# --------------------------------------------------------------------- flows
def test_radial_flows_equal_downstream_sums():
    """Tree grid: the flow on a branch is the injection sum beyond it (KCL on a cut)."""
    rng = np.random.default_rng(1)
    grid = gg.make_grid(25, 24, seed=11)
    P = _balanced(rng, grid.n_bus, T=3)
    f = _flows(grid, P)
    for e in range(grid.n_branch):
        ins = np.ones(grid.n_branch, bool)
        ins[e] = False
        slack_side = _bfs_component(grid.n_bus, grid.from_bus, grid.to_bus, ins, grid.slack)
        down = [i for i in range(grid.n_bus) if i not in slack_side]
        s = P[down].sum(axis=0)
        expect = -s if grid.to_bus[e] in down else s   # into the downstream side
        np.testing.assert_allclose(f[e], expect, rtol=1e-10, atol=1e-9)


def test_kcl_at_every_bus():
    rng = np.random.default_rng(2)
    grid = gg.make_grid(60, 95, seed=12)
    P = _balanced(rng, grid.n_bus, T=2)
    f = _flows(grid, P)
    net = np.zeros_like(P)
    np.add.at(net, grid.from_bus, f)
    np.add.at(net, grid.to_bus, -f)
    np.testing.assert_allclose(net, P, atol=1e-9)


def test_loop_law_on_every_chord():
    """DC voltage law: sum of x_e f_e around each fundamental cycle is zero."""
    rng = np.random.default_rng(3)
    grid = gg.make_grid(40, 70, seed=13)
    P = _balanced(rng, grid.n_bus)
    f = _flows(grid, P)[:, 0]
    # BFS spanning tree
    adj = [[] for _ in range(grid.n_bus)]
    for e in range(grid.n_branch):
        adj[grid.from_bus[e]].append((grid.to_bus[e], e, +1))
        adj[grid.to_bus[e]].append((grid.from_bus[e], e, -1))
    parent = {0: None}
    q = deque([0])
    tree = set()
    while q:
        u = q.popleft()
        for v, e, sgn in adj[u]:
            if v not in parent:
                parent[v] = (u, e, sgn)
                tree.add(e)
                q.append(v)

    def drop(u):   # angle drop from the root to u as sum of x*f along tree edges
        s = 0.0
        while parent[u] is not None:
            p, e, sgn = parent[u]
            s += sgn * grid.x_pu[e] * f[e]        # theta_p - theta_u
            u = p
        return s

    for e in range(grid.n_branch):
        if e in tree:
            continue
        a, b = grid.from_bus[e], grid.to_bus[e]
        # theta_a - theta_b = drop(b) - drop(a) must equal x_e f_e
        assert abs((drop(b) - drop(a)) - grid.x_pu[e] * f[e]) < 1e-9


def test_parallel_line_current_divider():
    x1, x2 = 0.1, 0.3
    P = np.array([[-100.0], [100.0]])
    f = o.solve_flows(2, [1, 1], [0, 0], [1 / x1, 1 / x2], np.ones(2, bool), P, 0)
    np.testing.assert_allclose(f[:, 0], [100 * x2 / (x1 + x2), 100 * x1 / (x1 + x2)], rtol=1e-12)


def test_superposition_and_slack_invariance():
    rng = np.random.default_rng(4)
    grid = gg.make_grid(50, 80, seed=14)
    P, Q = _balanced(rng, 50), _balanced(rng, 50)
    fa, fb = _flows(grid, P), _flows(grid, Q)
    np.testing.assert_allclose(_flows(grid, 2.5 * P - 0.5 * Q), 2.5 * fa - 0.5 * fb, atol=1e-9)
    # balanced injections: flows do not depend on which bus is the angle reference
    np.testing.assert_allclose(_flows(grid, P, slack=17), fa, atol=1e-9)


# ---------------------------------------------------------------- islanding
def test_islanding_tree_and_cycle():
    tree = gg.make_grid(10, 9, seed=5)
    for e in range(9):
        ins = np.ones(9, bool)
        ins[e] = False
        assert not o.is_connected(10, tree.from_bus, tree.to_bus, ins)
    n = 8
    fr, to = np.arange(n), (np.arange(n) + 1) % n
    for e in range(n):
        ins = np.ones(n, bool)
        ins[e] = False
        assert o.is_connected(n, fr, to, ins)
    for e1, e2 in itertools.combinations(range(n), 2):
        ins = np.ones(n, bool)
        ins[[e1, e2]] = False
        assert not o.is_connected(n, fr, to, ins)


def test_islanding_exhaustive_two_branch_outages_30bus():
    """All C(41,2) + 41 + 1 opening sets on the 30-bus grid versus an independent BFS."""
    grid = gg.make_grid(30, 41, 0x5EED0001)
    P = gg.make_injections(grid, 1, 0x5EED0002)
    m = grid.n_branch
    edges = gg.default_load_edges()
    sets = [()] + [(e,) for e in range(m)] + list(itertools.combinations(range(m), 2))
    for K in sets:
        ins = np.ones(m, bool)
        ins[list(K)] = False
        bfs = len(_bfs_component(30, grid.from_bus, grid.to_bus, ins, 0)) == 30
        cand = Candidate(opened=list(K), splits=[], moved_p=[], n_slots_filled=len(K))
        res = o.evaluate_candidate(grid, P, [0], [0], cand, edges, keep_n1=False)
        assert res.islanded == (not bfs), K


def test_island_contingencies_are_post_switch_bridges():
    """Skipped contingencies are exactly the bridges of the post-switch graph
    (Tarjan's algorithm from the input generator, an independent routine)."""
    w = gg.build_config(2, B=6, move_frac=0.5)
    edges = gg.default_load_edges()
    for c in range(6):
        cand = o.candidate_from_batch(w.batch, c)
        res = o.evaluate_candidate(w.grid, w.P, w.M, w.C, cand, edges, keep_n1=False)
        if res.islanded or not res.valid:
            continue
        net = o.post_switch_network(w.grid.n_bus, w.grid.from_bus, w.grid.to_bus,
                                    1 / w.grid.x_pu, 0, w.P, cand)
        br = gg.bridges(net.n_node, net.fr, net.to, net.in_service)
        expect = br[w.C] & net.in_service[w.C]
        np.testing.assert_array_equal(res.island_cont, expect)


# ------------------------------------------------- outages versus closed form
def _dense_ptdf(grid):
    n, m = grid.n_bus, grid.n_branch
    A = np.zeros((m, n))
    A[np.arange(m), grid.from_bus] = 1.0
    A[np.arange(m), grid.to_bus] = -1.0
    b = 1.0 / grid.x_pu
    L = A.T @ (b[:, None] * A)
    Linv = np.zeros((n, n))
    keep = np.arange(n) != grid.slack
    Linv[np.ix_(keep, keep)] = np.linalg.inv(L[np.ix_(keep, keep)])
    ptdf = b[:, None] * (A @ Linv)
    return ptdf, ptdf @ A.T


def test_lodf_identity_single_outages():
    """Re-solved N-1 flows equal f + H_{:,l} f_l / (1 - H_ll) (line outage
    distribution factors built from a dense inverse)."""
    w = gg.build_config(1)
    grid, P = w.grid, w.P
    _, H = _dense_ptdf(grid)
    f0 = _flows(grid, P)
    nb = gg.bridges(grid.n_bus, grid.from_bus, grid.to_bus)
    edges = gg.default_load_edges()
    cand = Candidate(opened=[], splits=[], moved_p=[], n_slots_filled=0)
    res = o.evaluate_candidate(grid, P, np.arange(grid.n_branch), np.arange(grid.n_branch),
                               cand, edges)
    for l in range(grid.n_branch):
        if nb[l]:
            assert res.island_cont[l]
            continue
        expect = f0[:, 0] + H[:, l] * f0[l, 0] / (1.0 - H[l, l])
        expect[l] = 0.0
        np.testing.assert_allclose(res.n1_flows[l][:, 0], expect, atol=1e-8)


def test_multi_outage_woodbury_identity():
    """Opening a set K: f' = f + H_{:,K} (I - H_KK)^{-1} f_K, zero on K."""
    w = gg.build_config(1)
    grid, P = w.grid, w.P
    _, H = _dense_ptdf(grid)
    f0 = _flows(grid, P)[:, 0]
    edges = gg.default_load_edges()
    rng = np.random.default_rng(9)
    nb = np.flatnonzero(~gg.bridges(grid.n_bus, grid.from_bus, grid.to_bus))
    for _ in range(20):
        K = sorted(rng.choice(nb, size=3, replace=False).tolist())
        cand = Candidate(opened=K, splits=[], moved_p=[], n_slots_filled=3)
        res = o.evaluate_candidate(grid, P, [0], [0], cand, edges, keep_n1=False)
        M_ = np.eye(3) - H[np.ix_(K, K)]
        if abs(np.linalg.det(M_)) < 1e-10:
            assert res.islanded
            continue
        expect = f0 + H[:, K] @ np.linalg.solve(M_, f0[K])
        expect[K] = 0.0
        np.testing.assert_allclose(res.base_flows[:, 0], expect, atol=1e-8)


# -------------------------------------------------------------------- splits
def test_split_moving_one_branch_equals_its_outage():
    w = gg.build_config(2, B=1)
    grid, P = w.grid, w.P
    inc = grid.incident()
    rng = np.random.default_rng(5)
    nb = ~gg.bridges(grid.n_bus, grid.from_bus, grid.to_bus)
    for _ in range(10):
        bus = int(rng.integers(0, grid.n_bus))
        cand_br = [e for e in inc[bus] if nb[e]]
        if len(inc[bus]) < 2 or not cand_br:
            continue
        e = int(rng.choice(cand_br))
        split = Candidate(opened=[], splits=[(bus, [e])], moved_p=[None], n_slots_filled=1)
        net = o.post_switch_network(grid.n_bus, grid.from_bus, grid.to_bus, 1 / grid.x_pu, 0, P, split)
        fs = o.solve_flows(net.n_node, net.fr, net.to, net.b, net.in_service, net.P, 0)
        ins = np.ones(grid.n_branch, bool)
        ins[e] = False
        fo = _flows(grid, P, ins)
        np.testing.assert_allclose(fs, fo, atol=1e-8)


def test_split_moving_everything_is_a_relabel():
    w = gg.build_config(2, B=1)
    grid, P = w.grid, w.P
    inc = grid.incident()
    f0 = _flows(grid, P)
    for bus in [5, 77, 123, 400]:
        cand = Candidate(opened=[], splits=[(bus, list(inc[bus]))], moved_p=[P[bus].copy()],
                         n_slots_filled=1)
        net = o.post_switch_network(grid.n_bus, grid.from_bus, grid.to_bus, 1 / grid.x_pu, 0, P, cand)
        # busbar A is left empty: the graph has an isolated node -> islanded by definition
        assert not o.is_connected(net.n_node, net.fr, net.to, net.in_service)
        keep = np.ones(net.n_node, bool)
        keep[bus] = False
        relabel = -np.ones(net.n_node, int)
        relabel[keep] = np.arange(net.n_node - 1)
        fs = o.solve_flows(net.n_node - 1, relabel[net.fr], relabel[net.to], net.b, net.in_service,
                           net.P[keep], 0)
        np.testing.assert_allclose(fs, f0, atol=1e-8)


def test_split_square_closed_form():
    g = json.load(open(os.path.join(GOLDEN, "split_square.json")))
    grid = gg.Grid(n_bus=g["n_bus"], from_bus=np.array(g["from"], np.int32),
                   to_bus=np.array(g["to"], np.int32), x_pu=np.array(g["x"]),
                   limit_mw=np.full(4, 100.0))
    P = np.array(g["P"])[:, None]
    cand = Candidate(opened=[], splits=[(g["split_bus"], g["moved"])], moved_p=[None],
                     n_slots_filled=1)
    res = o.evaluate_candidate(grid, P, [0, 1, 2, 3], [0, 1, 2, 3], cand,
                               gg.default_load_edges(), keep_n1=True)
    assert res.valid and not res.islanded
    np.testing.assert_allclose(res.base_flows[:, 0], g["expected_flows"], atol=1e-10)
    # the path has only bridges left: every contingency islands except opening
    # branch 3, which already carries nothing (its loss isolates busbar B)
    assert res.island_cont.all()


def test_moved_injection_changes_only_through_kcl():
    """Split with a moved injection: KCL holds at both busbars of the split bus."""
    w = gg.build_config(2, B=20, move_frac=1.0)
    edges = gg.default_load_edges()
    for c in range(20):
        cand = o.candidate_from_batch(w.batch, c)
        if not cand.splits:
            continue
        net = o.post_switch_network(w.grid.n_bus, w.grid.from_bus, w.grid.to_bus,
                                    1 / w.grid.x_pu, 0, w.P, cand)
        if not o.is_connected(net.n_node, net.fr, net.to, net.in_service):
            continue
        f = o.solve_flows(net.n_node, net.fr, net.to, net.b, net.in_service, net.P, 0)
        bal = np.zeros_like(net.P)
        np.add.at(bal, net.fr, f)
        np.add.at(bal, net.to, -f)
        np.testing.assert_allclose(bal, net.P, atol=1e-8)
        return
    pytest.fail("no usable split candidate drawn")


# ------------------------------------------------------ metrics and archive
def test_metrics_hand_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "metrics_example.json")))
    fmax, f0, lim = np.array(g["fmax"]), np.array(g["f0"]), np.array(g["limit"])
    met = o.n1_metrics(fmax, f0, lim)
    ex = g["expected"]
    assert met["overload_mw"] == pytest.approx(ex["overload_mw"], abs=1e-12)
    assert met["n_crit_n1"] == ex["n_crit_n1"]
    assert met["n_crit_n0"] == ex["n_crit_n0"]
    assert met["max_loading"] == pytest.approx(ex["max_loading"], abs=1e-12)
    fit = o.fitness_f1(met["overload_mw"], met["n_crit_n0"], met["n_crit_n1"])
    assert fit == pytest.approx(ex["fitness_f1"], abs=1e-12)
    argl = np.ones(fmax.shape, dtype=int)            # contingency 1 attains fmax
    met2 = o.n1_metrics(fmax, f0, lim, argl)
    assert met2["worst"] == (ex["worst_e"], ex["worst_t"], 1)


def test_descriptor_cell_edges_and_bijection():
    edges = np.array([0.5, 1.0, 1.5])
    assert o.descriptor_cell(0, 0.0, edges, 4) == 0
    assert o.descriptor_cell(0, 0.5, edges, 4) == 1          # on an edge: upper bin
    assert o.descriptor_cell(0, 0.4999, edges, 4) == 0
    assert o.descriptor_cell(1, 9.0, edges, 4) == 1 * 4 + 3   # clamps high
    assert o.descriptor_cell(99, 1.2, edges, 4) == 3 * 4 + 2  # count clamps to n-1
    e32 = gg.default_load_edges()
    seen = set()
    for k in range(32):
        for bi in range(32):
            rho = 0.0 if bi == 0 else e32[bi - 1]
            seen.add(o.descriptor_cell(k, rho, e32, 32))
    assert seen == set(range(1024))


def test_archive_strict_and_order_invariant():
    rng = np.random.default_rng(7)
    B, cells = 300, 16
    fit = rng.integers(-20, 0, size=B).astype(float)   # many exact ties
    cell = rng.integers(0, cells, size=B)
    ok = rng.random(B) > 0.1
    bf0, bi0 = np.full(cells, -np.inf), np.full(cells, -1, np.int64)
    bf, bi = o.archive_insert_sequential(bf0, bi0, fit, cell, ok)
    for c in range(cells):
        sel = np.flatnonzero((cell == c) & ok)
        if len(sel) == 0:
            assert bi[c] == -1
            continue
        best = fit[sel].max()
        assert bf[c] == best and bi[c] == sel[fit[sel] == best][0]   # earliest among ties
    # offering the same batch again never replaces (strict improvement only)
    bf2, bi2 = o.archive_insert_sequential(bf, bi, fit, cell, ok, id_base=1000)
    np.testing.assert_array_equal(bi2, bi)
    # islanded / invalid candidates never enter
    assert not np.isin(bi[bi >= 0], np.flatnonzero(~ok)).any()


def test_worst_contingency_on_a_bridge_follows_list_order():
    """A bridge carries the injection of the side it cuts off, whatever other
    branch is out, so every non-islanding outage ties on it exactly: the
    worst contingency is the first non-islanding entry of C, for any order."""
    from gridgen import Grid
    # ring 0-1-2-3-0 plus bridge 2-4 to a 90 MW load behind a 50 MW limit
    fr = np.array([0, 1, 2, 3, 2]); to = np.array([1, 2, 3, 0, 4])
    grid = Grid(n_bus=5, from_bus=fr, to_bus=to, x_pu=np.array([.1, .2, .15, .12, .1]),
                limit_mw=np.array([300.0, 300, 300, 300, 50]), slack=0)
    P = np.array([[90.0], [0.0], [0.0], [0.0], [-90.0]])
    edges = gg.default_load_edges()
    cand = o.Candidate(opened=[], splits=[], moved_p=[], n_slots_filled=0)
    for C in ([0, 1, 2, 3, 4], [3, 1, 4, 0, 2], [4, 2, 0, 1, 3]):
        for keep in (True, False):
            r = o.evaluate_candidate(grid, P, np.arange(5), np.array(C), cand, edges, keep_n1=keep)
            assert r.metrics["worst_branch"] == 4 and r.metrics["max_loading"] == pytest.approx(1.8)
            first = next(l for l in C if l != 4)          # outage of the bridge islands bus 4
            assert r.metrics["worst_cont"] == first, (C, keep)


def test_worst_contingency_second_pass_matches_stored_tensor():
    w = gg.build_config(2, B=5)
    edges = gg.default_load_edges()
    for c in range(5):
        cand = o.candidate_from_batch(w.batch, c)
        a = o.evaluate_candidate(w.grid, w.P, w.M, w.C, cand, edges, keep_n1=True)
        b = o.evaluate_candidate(w.grid, w.P, w.M, w.C, cand, edges, keep_n1=False)
        assert a.metrics.get("worst_cont") == b.metrics.get("worst_cont")


def test_running_argmax_matches_full_tensor():
    """The worst contingency is the first entry of C whose |flow| in the
    stored N-1 tensor at (e*, t*) is within the tie tolerance of the
    maximum, and f^max is the tensor's maximum."""
    w = gg.build_config(2, B=6, move_frac=0.5)
    edges = gg.default_load_edges()
    for c in range(6):
        cand = o.candidate_from_batch(w.batch, c)
        r = o.evaluate_candidate(w.grid, w.P, w.M, w.C, cand, edges, keep_n1=True)
        if r.islanded or not r.valid:
            continue
        e = int(np.flatnonzero(w.M == r.metrics["worst_branch"])[0])
        t_ = r.metrics["worst_t"]
        col = np.abs(r.n1_flows[:, e, t_])
        col = np.where(np.isnan(col), -np.inf, col)
        tie = o.dcflow.WORST_CONT_TIE_MW
        assert r.metrics["worst_cont"] == int(w.C[int(np.flatnonzero(col >= col.max() - tie)[0])])
        np.testing.assert_allclose(r.fmax, np.nanmax(np.abs(r.n1_flows), axis=0))


def test_contingency_energies_hand_worked():
    """Two monitored branches (limits 100 and 50 MW), two timesteps, three
    contingencies (the second islands):
      l0: |f| = [[120, 90], [40, 70]] -> 20 + 0 + 0 + 20 = 40
      l1: islands -> excluded
      l2: |f| = [[-101, 99], [50, 51]] -> 1 + 0 + 0 + 1 = 2
    and a fourth with no overload (0).  Worst-2: l0, l2; worst-4 pads."""
    n1 = np.array([[[120, 90], [40, -70]], [[np.nan, np.nan], [np.nan, np.nan]],
                   [[-101, 99], [50, 51]], [[10, 20], [30, 40]]], dtype=float)
    lim = np.array([100.0, 50.0])
    E = o.contingency_energies(n1, lim)
    assert E[0] == 40.0 and np.isnan(E[1]) and E[2] == 2.0 and E[3] == 0.0
    ids, en = o.worst_k(E, [11, 12, 13, 14], 2)
    assert ids.tolist() == [11, 13] and en.tolist() == [40.0, 2.0]
    ids, en = o.worst_k(E, [11, 12, 13, 14], 5)
    assert ids.tolist() == [11, 13, 14, -1, -1] and np.isnan(en[3:]).all()
    # ties (all zero) go to the earlier entry of C
    ids, _ = o.worst_k(np.zeros(5), [9, 3, 7, 1, 5], 3)
    assert ids.tolist() == [9, 3, 7]


def test_contingency_energies_bound_the_overload_energy():
    """f^max >= |f^(l)| gives E_l <= lambda_o for every l, and every (e, t)
    maximum is attained by some outage, so lambda_o <= sum_l E_l."""
    w = gg.build_config(2, B=6)
    edges = gg.default_load_edges()
    lim = w.grid.limit_mw[w.M]
    seen = 0
    for c in range(6):
        r = o.evaluate_candidate(w.grid, w.P, w.M, w.C, o.candidate_from_batch(w.batch, c), edges,
                                 keep_n1=True)
        if r.islanded or not r.valid:
            continue
        E = o.contingency_energies(r.n1_flows, lim)
        lam = r.metrics["overload_mw"]
        fin = E[~np.isnan(E)]
        assert fin.max() <= lam + 1e-9 and lam <= fin.sum() + 1e-9
        seen += lam > 0
    assert seen >= 1


# ------------------------------------------------------ busbar outages
def _grid(fr, to, x, lim, n):
    from gridgen import Grid
    return Grid(n_bus=n, from_bus=np.array(fr), to_bus=np.array(to), x_pu=np.array(x, float),
                limit_mw=np.array(lim, float), slack=0)


def _empty():
    return Candidate(opened=[], splits=[], moved_p=[], n_slots_filled=0)


def test_busbar_outage_radial_chain_closed_form():
    """Chain 0-1-2-3 (slack 0), loads 10, 20, 30 MW at buses 1..3: losing
    busbar 3 drops its load (flows 30, 20, 0); losing 1 or 2 islands."""
    g = _grid([0, 1, 2], [1, 2, 3], [.1, .1, .1], [100, 100, 100], 4)
    P = np.array([[60.0], [-10.0], [-20.0], [-30.0]])
    b = 1 / g.x_pu
    net = o.post_switch_network(4, g.from_bus, g.to_bus, b, 0, P, _empty())
    f = o.busbar_outage_flows(net, 3)
    np.testing.assert_allclose(f[:, 0], [30.0, 20.0, 0.0], atol=1e-9)
    assert o.busbar_outage_flows(net, 1) is None and o.busbar_outage_flows(net, 2) is None
    met = o.busbar_metrics(g, P, [0, 1, 2], _empty(), [1, 2, 3])
    assert met["n_island"] == 2 and met["lambda_b"] == 0.0


def test_busbar_outage_ring_closed_form():
    """Ring 0-1-2-3-0, 60 MW load at bus 2: losing busbar 1 leaves the chain
    0-3-2, so branch (3,0) carries -60 and (2,3) carries -60 MW."""
    g = _grid([0, 1, 2, 3], [1, 2, 3, 0], [.1, .1, .1, .1], [100, 100, 50, 50], 4)
    P = np.array([[60.0], [0.0], [-60.0], [0.0]])
    net = o.post_switch_network(4, g.from_bus, g.to_bus, 1 / g.x_pu, 0, P, _empty())
    f = o.busbar_outage_flows(net, 1)
    np.testing.assert_allclose(f[:, 0], [0.0, 0.0, -60.0, -60.0], atol=1e-9)
    met = o.busbar_metrics(g, P, [0, 1, 2, 3], _empty(), [1])
    assert met["lambda_b"] == pytest.approx(20.0)        # 10 MW over on each 50 MW branch


def test_busbar_outage_equals_injection_to_slack_and_all_but_one_branch_open():
    """A busbar outage is the injection moved to the slack plus every branch
    of the bus but one opened: the kept branch then joins a node without
    injection and carries nothing."""
    w = gg.build_config(1)
    g = w.grid
    b = 1 / g.x_pu
    net = o.post_switch_network(g.n_bus, g.from_bus, g.to_bus, b, g.slack, w.P, _empty())
    checked = 0
    for bus in range(1, g.n_bus):
        f = o.busbar_outage_flows(net, bus)
        on = np.flatnonzero((g.from_bus == bus) | (g.to_bus == bus))
        if f is None or len(on) < 2:
            continue
        ins = np.ones(len(g.from_bus), bool)
        ins[on[:-1]] = False
        P2 = w.P.copy()
        P2[g.slack] += P2[bus]
        P2[bus] = 0.0
        f2 = o.solve_flows(g.n_bus, g.from_bus, g.to_bus, b, ins, P2, g.slack)
        np.testing.assert_allclose(f2, f, atol=1e-9)
        assert np.all(np.abs(f2[on[-1]]) < 1e-9)
        checked += 1
    assert checked >= 5


def test_busbar_outage_of_a_split_bus_keeps_busbar_b():
    """Losing busbar A of a split bus keeps the moved branches and the moved
    injection on busbar B (KCL holds at B)."""
    w = gg.build_config(1)
    g = w.grid
    inc = [np.flatnonzero((g.from_bus == i) | (g.to_bus == i)) for i in range(g.n_bus)]
    bus = next(i for i in range(1, g.n_bus) if len(inc[i]) >= 3)
    moved = [int(inc[bus][0])]
    cand = Candidate(opened=[], splits=[(bus, moved)], moved_p=[np.array([5.0])], n_slots_filled=1)
    net = o.post_switch_network(g.n_bus, g.from_bus, g.to_bus, 1 / g.x_pu, g.slack, w.P, cand)
    f = o.busbar_outage_flows(net, bus)
    assert f is not None
    e = moved[0]
    sign = 1.0 if net.fr[e] == g.n_bus else -1.0     # orientation out of busbar B
    assert sign * f[e, 0] == pytest.approx(5.0)       # B's only branch carries its injection
    for x in inc[bus][1:]:
        assert f[x, 0] == 0.0


def test_fitness_f2_clips_at_the_pre_optimisation_penalty():
    assert o.fitness_f2(-100.0, 30.0, 50.0) == -100.0
    assert o.fitness_f2(-100.0, 80.0, 50.0) == -130.0


def test_paper_descriptor_is_a_bijection_of_the_clamped_ranges():
    """lambda_d in 0..2, lambda_s in 0..3, lambda_r in 0..45 map one to one
    onto the 3 x 4 x 46 = 552 cells; larger counts clamp."""
    cells = {o.descriptor_cell_paper(d, s_, r) for d in range(3) for s_ in range(4)
             for r in range(46)}
    assert cells == set(range(552))
    assert o.descriptor_cell_paper(0, 0, 0) == 0
    assert o.descriptor_cell_paper(1, 1, 1) == 1 + 3 * (1 + 4)
    assert o.descriptor_cell_paper(2, 3, 45) == 551
    assert o.descriptor_cell_paper(7, 8, 99) == 551


# ------------------------------------------------------ PTDF and bridges
def test_ptdf_radial_chain_and_divider():
    """Chain 0-1-2 (slack 0): one MW from bus 2 crosses both branches towards
    the slack (PTDF -1 on branches oriented away from it).  Two parallel
    paths 0-1 (x = 0.1) and 0-2-1 (x = 0.1 + 0.3): the direct branch carries
    0.4 / 0.5 of a transfer into bus 1."""
    from oracle.ptdf import ptdf
    P = ptdf(3, [0, 1], [1, 2], [10.0, 10.0], 0)
    np.testing.assert_allclose(P, [[0, -1, -1], [0, 0, -1]], atol=1e-12)
    P = ptdf(3, [0, 0, 2], [1, 2, 1], [10.0, 10.0, 1 / 0.3], 0)
    assert P[0, 1] == pytest.approx(-0.8)
    assert P[1, 1] == pytest.approx(-0.2) and P[2, 1] == pytest.approx(-0.2)


def test_ptdf_kirchhoff_at_every_bus():
    """Every column is a unit transfer from bus j to the slack: the net
    outflow of its flows is +1 at j, -1 at the slack, 0 elsewhere."""
    from oracle.ptdf import ptdf
    w = gg.build_config(1)
    g = w.grid
    P = ptdf(g.n_bus, g.from_bus, g.to_bus, 1 / g.x_pu, g.slack)
    A = np.zeros((len(g.from_bus), g.n_bus))
    A[np.arange(len(g.from_bus)), g.from_bus] = 1
    A[np.arange(len(g.from_bus)), g.to_bus] = -1
    want = np.eye(g.n_bus)
    want[g.slack] -= 1
    want[:, g.slack] = 0
    np.testing.assert_allclose(A.T @ P, want, atol=1e-10)


def test_bridges_brute_force_against_tarjan_generator():
    from oracle.ptdf import bridges
    for cfg in (1, 2):
        g = gg.build_config(cfg, B=1).grid
        assert np.array_equal(bridges(g.n_bus, g.from_bus, g.to_bus),
                              gg.bridges(g.n_bus, g.from_bus, g.to_bus))
