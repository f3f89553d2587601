"""MapElites generation on the GPU (tto_vary, tto_genome_expand,
tto_generation) against oracle/evolve.py: children bit-exact, expanded batches
exact, the repertoire of a multi-generation FP64 loop equal to the oracle's,
graph replays equal to eager generations."""
import numpy as np
import pytest

import gridgen as gg
from oracle import evolve as ev
from parity_util import log, make_session

pytestmark = pytest.mark.gpu


def tables(w, n_actions, seed):
    table = gg.make_split_table(w.grid, n_actions, seed)
    D = np.flatnonzero(~gg.bridges(w.grid.n_bus, w.grid.from_bus, w.grid.to_bus)).astype(np.int32)
    return np.array([b for b, _ in table], dtype=np.int32), [mv for _, mv in table], D


def spaces(sess, w, n_a, n_d, n_actions, seed, p_c1=0.5, **kw):
    from paper_2605_10128_amd import tto
    bus, moved, D = tables(w, n_actions, seed)
    dev = tto.GenomeSpace(sess, bus, moved, D, n_a, n_d, p_c1=p_c1, **kw)
    orc = ev.GenomeSpace(bus, moved, D, n_a, n_d, p_c1=p_c1, **kw)
    return dev, orc


def random_elites(orc, n_cells, occ_frac, rng, garbage=False):
    G = orc.n_a + orc.n_d
    ids = np.where(rng.random(n_cells) < occ_frac, rng.integers(0, 10**6, n_cells), -1)
    gen = np.full((n_cells, max(G, 1)), -1, dtype=np.int32)
    stations = sorted(orc.count)
    for c in range(n_cells):
        if garbage:
            gen[c, :G] = rng.integers(-3, max(orc.n_actions, orc.n_disc) + 3, size=G)
            continue
        k = int(rng.integers(0, min(orc.n_a, len(stations)) + 1))
        for j, q in enumerate(rng.choice(stations, size=k, replace=False)):
            q = int(q)
            gen[c, j] = orc.station_order[orc.first[q] + int(rng.integers(0, orc.count[q]))]
        kd = int(rng.integers(0, min(orc.n_d, orc.n_disc) + 1))
        gen[c, orc.n_a:orc.n_a + kd] = rng.choice(orc.n_disc, size=kd, replace=False)
        gen[c, :orc.n_a] = rng.permutation(gen[c, :orc.n_a])
        gen[c, orc.n_a:G] = rng.permutation(gen[c, orc.n_a:G])
    return ids.astype(np.int64), gen


@pytest.fixture(scope="module")
def w500():
    return gg.build_config(2, B=64)


@pytest.fixture(scope="module")
def s500(w500):
    from paper_2605_10128_amd import tto
    s = make_session(w500, tto.TTO_FLOW_F32, max_batch=4096)
    yield s
    s.close()


# (n_a, n_d, p_c1, |A|, occupied fraction, n_child, generation, garbage elites)
VARY_CASES = [
    (4, 4, 0.5, 600, 0.3, 5000, 7, False),
    (4, 4, 0.5, 600, 0.0, 1000, 0, False),          # empty repertoire
    (8, 0, 0.25, 600, 0.5, 777, 3, False),          # no disconnection slots
    (0, 8, 1.0, 600, 0.5, 300, 2**33 + 5, False),   # no action slots, counter above 2^32
    (3, 2, 0.0, 40, 0.002, 4097, 11, False),        # small table, few occupied cells
    (2, 2, 0.5, 8, 1.0, 1, 1, False),               # one child
    (4, 3, 0.6, 200, 0.5, 2000, 5, True),           # infeasible elites read as feasible
]


@pytest.mark.parametrize("case", VARY_CASES, ids=[str(i) for i in range(len(VARY_CASES))])
def test_vary_matches_oracle_bitwise(s500, w500, case):
    import torch
    n_a, n_d, p_c1, n_act, occ, n_child, gen, garbage = case
    log(f"[vary] n_a={n_a} n_d={n_d} p_c1={p_c1} |A|={n_act} occ={occ} n_child={n_child} gen={gen}")
    dev, orc = spaces(s500, w500, n_a, n_d, n_act, seed=1234 + n_act, p_c1=p_c1)
    rng = np.random.default_rng(n_child)
    ids, genomes = random_elites(orc, 1024, occ, rng, garbage)
    seed = 0x1234_5678_9ABC + gen

    class Rep:
        n_cells = 1024
        id = torch.as_tensor(ids, device=s500.device)
        genome = torch.as_tensor(genomes, device=s500.device)
        generation = torch.tensor([gen], dtype=torch.int64, device=s500.device)

    kids, b_mc = dev.vary(Rep, seed, n_child)
    torch.cuda.synchronize()
    want, want_b = ev.vary(orc, ids, genomes[:, :n_a + n_d], seed, gen, n_child)
    got = kids.cpu().numpy()[:, :n_a + n_d]
    assert int(b_mc.item()) == want_b
    bad = np.flatnonzero(np.any(got != want, axis=1))
    assert bad.size == 0, f"{bad.size} children differ, first {bad[:5]}: {got[bad[:3]]} vs {want[bad[:3]]}"
    log(f"  {n_child} children identical, b_mc={want_b}")


def test_expand_matches_oracle(s500, w500):
    import torch
    dev, orc = spaces(s500, w500, 4, 3, 600, seed=99)
    rng = np.random.default_rng(5)
    n = 3001
    g = np.full((n, 7), -1, dtype=np.int32)
    g[:, :4] = np.where(rng.random((n, 4)) < 0.6, rng.integers(0, 600, (n, 4)), -1)
    g[:, 4:] = np.where(rng.random((n, 3)) < 0.6, rng.integers(0, orc.n_disc, (n, 3)), -1)
    g[::97, 1] = 600 + 5          # out-of-range action id
    g[::89, 5] = -7               # out-of-range disconnection
    db = dev.expand(torch.as_tensor(g, device=s500.device))
    torch.cuda.synchronize()
    opens, sbus, moved = ev.expand(orc, g)
    assert np.array_equal(db.open.cpu().numpy(), opens)
    assert np.array_equal(db.split_bus.cpu().numpy(), sbus)
    off = db.moved_off.cpu().numpy()
    br = db.moved_br.cpu().numpy()
    assert off[0] == 0 and np.all(np.diff(off) >= 0)
    for s in range(n * 4):
        assert br[off[s]:off[s + 1]].tolist() == moved[s], s


def _run_loop(w, flow, n_a, n_d, n_actions, n_child, n_gen, seed, processes, max_batch=None,
              descriptor="count_load"):
    import torch
    from paper_2605_10128_amd import tto
    sess = make_session(w, flow, max_batch=max_batch or n_child)
    if descriptor == "paper":
        sess.set_descriptor(gg.default_load_edges(), kind=tto.TTO_DESC_PAPER)
    dev, orc = spaces(sess, w, n_a, n_d, n_actions, seed=seed)
    rep = tto.Repertoire(sess, dev)
    outs = sess.alloc_outputs(n_child)
    evo = tto.Evolver(sess, dev, rep, n_child, seed, outputs=outs)
    edges = gg.default_load_edges()
    state = None
    for g in range(n_gen):
        evo.step()
        torch.cuda.synchronize()
        state, logs = _oracle_generation(w, orc, seed, g, n_child, edges, state, processes,
                                         descriptor, sess.n_cells)
        kids = evo.children.cpu().numpy()
        assert np.array_equal(kids, logs["children"]), f"generation {g}: children differ"
        st = outs["status"].cpu().numpy()
        assert np.array_equal((st & 2) == 0, logs["valid"]), f"generation {g}: validity differs"
        ok = logs["valid"] & ~logs["islanded"]
        assert np.array_equal((st & 3) == 0, ok), f"generation {g}: islanding differs"
        assert np.array_equal(outs["cell"].cpu().numpy()[ok], logs["cell"][ok]), f"generation {g}: cells differ"
        gfit = outs["fitness"].cpu().numpy()
        np.testing.assert_allclose(gfit[ok], logs["fitness"][ok], rtol=1e-12, atol=1e-6)
        fit, ids, gen = state
        gf, gi, gg_ = rep.fitness.cpu().numpy(), rep.id.cpu().numpy(), rep.genome.cpu().numpy()
        for c in np.flatnonzero(gi != ids):
            log(f"  cell {c}: gpu elite {gi[c]} (fitness {gf[c]!r}), oracle elite {ids[c]} "
                f"(fitness {fit[c]!r})")
            for who, e in (("gpu", gi[c]), ("oracle", ids[c])):
                if e >= g * n_child:
                    k = int(e - g * n_child)
                    log(f"    {who} pick child {k}: genome {kids[k].tolist()} gpu fit "
                        f"{gfit[k]!r} oracle fit {logs['fitness'][k]!r}")
        assert np.array_equal(gi, ids), f"generation {g}: elite ids differ"
        assert np.array_equal(gg_[:, :n_a + n_d], gen), f"generation {g}: elite genomes differ"
        occ = ids >= 0
        np.testing.assert_allclose(gf[occ], fit[occ], rtol=1e-12, atol=1e-6)
        assert int(rep.generation.item()) == g + 1
        log(f"  generation {g}: {int(occ.sum())} cells, b_mc={logs['b_mc']}, "
            f"invalid {int((~logs['valid']).sum())}, islanded {int(logs['islanded'].sum())}")
    sess.close()


def _oracle_generation(w, orc, seed, g, n_child, edges, state, processes,
                       descriptor="count_load", n_cells=1024):
    import oracle
    if state is None:
        G = orc.n_a + orc.n_d
        state = (np.full(n_cells, -np.inf), np.full(n_cells, -1, dtype=np.int64),
                 np.full((n_cells, G), -1, dtype=np.int32))
    fit, ids, gen = state
    kids, b_mc = ev.vary(orc, ids, gen, seed, g, n_child)
    cands = ev.to_candidates(orc, kids)
    jobs = [(w.grid, w.P, w.M, w.C, cd, edges, dict(keep_n1=False, descriptor=descriptor))
            for cd in cands]
    if processes > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(processes) as pool:
            res = pool.map(oracle.dcflow._eval_one, jobs, chunksize=1)
    else:
        res = [oracle.dcflow._eval_one(j) for j in jobs]
    ok = np.array([r.valid and not r.islanded for r in res])
    f = np.array([r.fitness for r in res])
    cells = np.array([r.cell for r in res])
    state = ev.archive_insert_genomes(fit, ids, gen, f, cells, ok, kids, g * n_child)
    return state, dict(children=kids, b_mc=b_mc, valid=np.array([r.valid for r in res]),
                       islanded=np.array([r.islanded for r in res]), fitness=f, cell=cells)


def test_generation_loop_matches_oracle_30_bus_f64():
    from paper_2605_10128_amd import tto
    w = gg.build_config(1)
    log("[loop] 30-bus, FP64, N_a=2, N_d=2, 64 children x 6 generations")
    _run_loop(w, tto.TTO_FLOW_F64, 2, 2, 24, 64, 6, seed=77, processes=1)


def test_generation_loop_paper_descriptor_30_bus_f64():
    """The same loop on the paper's 552-cell (disconnections, splits,
    reassigned assets) map."""
    from paper_2605_10128_amd import tto
    w = gg.build_config(1)
    log("[loop] 30-bus, FP64, paper descriptor, N_a=3, N_d=2, 64 children x 4 generations")
    _run_loop(w, tto.TTO_FLOW_F64, 3, 2, 24, 64, 4, seed=91, processes=1, descriptor="paper")


def test_paper_descriptor_cells_500_bus_f32():
    """Cells of the paper map for a batch with splits: integers from the
    candidate alone, equal to the oracle's for every connected candidate."""
    import torch
    import oracle
    from paper_2605_10128_amd import tto
    w = gg.build_config(2, B=512)
    sess = make_session(w, tto.TTO_FLOW_F32, max_batch=512)
    sess.set_descriptor(gg.default_load_edges(), kind=tto.TTO_DESC_PAPER)
    out = sess.evaluate(tto.device_batch(w.batch))
    torch.cuda.synchronize()
    st, cell = out["status"].cpu().numpy(), out["cell"].cpu().numpy()
    seen = set()
    for c in range(512):
        cd = oracle.candidate_from_batch(w.batch, c)
        if st[c] & 3:
            assert cell[c] == -1
            continue
        want = oracle.descriptor_cell_paper(len(cd.opened), len(cd.splits),
                                            sum(len(mv) for _, mv in cd.splits))
        assert cell[c] == want, c
        seen.add(want)
    assert len(seen) >= 10 and max(seen) < 552
    log(f"[descriptor] paper map: {len(seen)} distinct cells over 512 candidates")
    sess.close()


def test_generation_loop_matches_oracle_500_bus_f64():
    from paper_2605_10128_amd import tto
    w = gg.build_config(2, B=32)
    log("[loop] 500-bus, FP64, N_a=3, N_d=3, 32 children x 3 generations")
    _run_loop(w, tto.TTO_FLOW_F64, 3, 3, 300, 32, 3, seed=5, processes=8)


@pytest.mark.parametrize("flow", ["f64", "f32"])
def test_generation_graph_replays_equal_eager(flow):
    import torch
    from paper_2605_10128_amd import tto
    w = gg.build_config(1) if flow == "f64" else gg.build_config(2, B=512)
    fp = tto.TTO_FLOW_F64 if flow == "f64" else tto.TTO_FLOW_F32
    n_child = 64 if flow == "f64" else 512
    sess = make_session(w, fp, max_batch=n_child)
    dev, _ = spaces(sess, w, 3, 3, 60, seed=3)
    eager = tto.Repertoire(sess, dev)
    evo = tto.Evolver(sess, dev, eager, n_child, seed=9)
    for _ in range(4):
        evo.step()
    torch.cuda.synchronize()
    rep = tto.Repertoire(sess, dev)
    evo2 = tto.Evolver(sess, dev, rep, n_child, seed=9)
    with tto.Graph() as graph:
        evo2.step()
    assert int(rep.generation.item()) == 0
    for k in range(4):
        graph.launch()
        torch.cuda.synchronize()
        _ = rep.fitness.sum().item()        # eager work between replays
    graph.close()
    assert int(rep.generation.item()) == 4
    for a, b in ((eager.fitness, rep.fitness), (eager.id, rep.id), (eager.genome, rep.genome)):
        assert torch.equal(a, b)
    log(f"[graph] {flow}: 4 replays equal 4 eager generations, "
        f"{int((rep.id >= 0).sum().item())} cells filled")
    sess.close()


def test_genome_space_rejects_bad_tables(s500, w500):
    from paper_2605_10128_amd import tto
    bus, moved, D = tables(w500, 20, 7)
    g = w500.grid
    far = next(e for e in range(len(g.from_bus))
               if g.from_bus[e] != bus[0] and g.to_bus[e] != bus[0])
    cases = [
        (dict(action_moved=[[far]] + moved[1:]), tto.TTO_E_GRID),
        (dict(disc_branch=np.array([D[0], D[0]])), tto.TTO_E_GRID),
        (dict(action_bus=np.array([g.n_bus] + list(bus[1:]))), tto.TTO_E_GRID),
        (dict(n_action_slots=9), tto.TTO_E_RANK),
        (dict(p_c1=1.5), tto.TTO_E_INVALID),
        (dict(action_moved=[[]] + moved[1:]), tto.TTO_E_INVALID),
    ]
    for over, code in cases:
        kw = dict(action_bus=bus, action_moved=moved, disc_branch=D, n_action_slots=2,
                  n_disc_slots=2)
        kw.update(over)
        with pytest.raises(tto.TTOError) as ei:
            tto.GenomeSpace(s500, **kw)
        assert ei.value.code == code, (over.keys(), ei.value)
    gs = tto.GenomeSpace(s500, bus, moved, D, 2, 2)
    rep = tto.Repertoire(s500, gs, n_cells=5000)
    with pytest.raises(tto.TTOError):
        gs.vary(rep, 1, 10)
    rep = tto.Repertoire(s500, gs, n_cells=100)          # not the descriptor's 1024 cells
    with pytest.raises(tto.TTOError):
        tto.Evolver(s500, gs, rep, 16, 1).step()


def test_generation_at_benchmarked_size():
    """The benchmarked generation (2000 buses, 16384 children, N_a = N_d = 4,
    the 4096-action table, FP32 flows) after two device generations: the
    third generation's children bit-exact against the oracle's variation from
    the same repertoire, their expansion exact, and the insertion of the
    device's evaluations equal to the oracle's one-at-a-time insertion."""
    import torch
    from paper_2605_10128_amd import tto
    w = gg.build_config(3)
    g = w.grid
    B = w.batch.n_cand
    sess = make_session(w, tto.TTO_FLOW_F32, max_batch=B)
    D = np.flatnonzero(~gg.bridges(g.n_bus, g.from_bus, g.to_bus)).astype(np.int32)
    bus = np.array([b for b, _ in w.split_table], dtype=np.int32)
    moved = [mv for _, mv in w.split_table]
    gs = tto.GenomeSpace(sess, bus, moved, D, 4, 4)
    orc = ev.GenomeSpace(bus, moved, D, 4, 4)
    rep = tto.Repertoire(sess, gs)
    outs = sess.alloc_outputs(B)
    seed = 0xE701
    evo = tto.Evolver(sess, gs, rep, B, seed=seed, outputs=outs)
    evo.step()
    evo.step()
    torch.cuda.synchronize()
    fit0 = rep.fitness.cpu().numpy()
    id0 = rep.id.cpu().numpy()
    gen0 = rep.genome.cpu().numpy()
    g0 = int(rep.generation.item())
    evo.step()
    torch.cuda.synchronize()
    kids = evo.children.cpu().numpy()
    want, want_b = ev.vary(orc, id0, gen0[:, :gs.G], seed, g0, B)
    assert int(evo.b_mc.item()) == want_b
    bad = np.flatnonzero(np.any(kids != want, axis=1))
    assert bad.size == 0, f"{bad.size} children differ, first {bad[:5]}"
    db = gs.expand(torch.as_tensor(kids, device=sess.device))
    torch.cuda.synchronize()
    opens, sbus, mv = ev.expand(orc, kids)
    assert np.array_equal(db.open.cpu().numpy(), opens)
    assert np.array_equal(db.split_bus.cpu().numpy(), sbus)
    off, br = db.moved_off.cpu().numpy(), db.moved_br.cpu().numpy()
    for s_ in range(0, B * gs.n_a, 97):
        assert br[off[s_]:off[s_ + 1]].tolist() == mv[s_], s_
    st = outs["status"].cpu().numpy()
    ok = (st & 3) == 0
    f_, i_, gm = ev.archive_insert_genomes(fit0, id0, gen0, outs["fitness"].cpu().numpy(),
                                           outs["cell"].cpu().numpy(), ok, kids, g0 * B)
    assert int(rep.generation.item()) == g0 + 1
    assert np.array_equal(rep.id.cpu().numpy(), i_)
    assert np.array_equal(rep.fitness.cpu().numpy(), f_)
    assert np.array_equal(rep.genome.cpu().numpy(), gm)
    log(f"[evolve] benchmarked size: generation {g0}, {B} children identical, b_mc={want_b}, "
        f"{int((i_ >= 0).sum())} cells after insertion")
    sess.close()
