"""Boundary and degenerate cases of the method on the device against the
oracle, through the C ABI: the encoding's validity rules on both sides of
each boundary, a split that moves every branch of its bus, a branch moved by
the splits at both of its ends, non-finite injections, and candidates whose
bordered-system LU (candidate set-up and busbar outages) must interchange
rows."""
import numpy as np
import pytest

import gridgen as gg
import oracle
import edge_cases as ec
from parity_util import TOL_F32, TOL_F64, compare, log, make_session, to_numpy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tto():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_10128_amd import tto as t
    return t


def _ten_bus(T=3, seed=5):
    g = ec.ten_bus_grid()
    rng = np.random.default_rng(seed)
    P = rng.normal(0, 30, size=(g.n_bus, T))
    P[0] = 0.0
    P[0] = -P.sum(axis=0)
    return g, P


def _workload(g, P, cands, moved_p=None):
    b = ec.as_batch(cands, T=P.shape[1])
    b.moved_p = moved_p
    m = g.n_branch
    return gg.Workload(cfg=0, grid=g, P=P, M=np.arange(m, dtype=np.int32),
                       C=np.arange(m, dtype=np.int32), batch=b)


def _flow(tto, flow):
    return (tto.TTO_FLOW_F64, TOL_F64) if flow == "f64" else (tto.TTO_FLOW_F32, TOL_F32)


@pytest.mark.parametrize("flow", ["f64", "f32"])
def test_validity_table_on_device(tto, flow):
    """Every row of the ten-bus table: the INVALID bit equals the oracle's
    verdict, and every valid row (islanded or not) matches the oracle's full
    evaluation, N-1 flows included."""
    import torch
    g, P = _ten_bus()
    cands = [c for _, c, _ in ec.TEN_BUS_TABLE]
    w = _workload(g, P, cands)
    fl, tol = _flow(tto, flow)
    s = make_session(w, fl, max_batch=len(cands))
    o = to_numpy(s.evaluate(tto.device_batch(w.batch), fmax=True, base_flows=True, n1=True))
    torch.cuda.synchronize()
    edges = gg.default_load_edges()
    ores = [oracle.evaluate_candidate(g, P, w.M, w.C, cd, edges, keep_n1=True) for cd in cands]
    for i, (label, _, valid) in enumerate(ec.TEN_BUS_TABLE):
        assert ores[i].valid is valid, label
        assert bool(o["status"][i] & tto.TTO_ST_INVALID) == (not valid), (label, o["status"][i])
        assert not (o["status"][i] & tto.TTO_ST_NONFINITE), label
    st = compare(w, o, range(len(cands)), ores, tol, strict_discrete=(flow == "f64"))
    n_isl = sum(1 for r in ores if r.valid and r.islanded)
    log(f"[edge] ten-bus table {flow}: {len(cands)} rows, {st['checked']} evaluated, "
        f"{n_isl} islanded, {sum(1 for r in ores if not r.valid)} invalid")
    # the split that leaves busbar A empty is islanded on both sides
    k = [r[0] for r in ec.TEN_BUS_TABLE].index(
        "split moving every branch of its bus (busbar A left empty)")
    assert ores[k].islanded and o["status"][k] & tto.TTO_ST_ISLANDED
    s.close()


def test_moved_branch_limit_on_device(tto):
    """64 moved branches over a candidate's splits are accepted, 65 are not."""
    import torch
    g = ec.star_grid()
    rng = np.random.default_rng(9)
    P = rng.normal(0, 10, size=(g.n_bus, 1))
    P[0] = 0.0
    P[0] = -P.sum(axis=0)
    cands = [c for _, c, _ in ec.STAR_TABLE]
    w = _workload(g, P, cands)
    s = make_session(w, tto.TTO_FLOW_F64, max_batch=len(cands))
    o = to_numpy(s.evaluate(tto.device_batch(w.batch)))
    torch.cuda.synchronize()
    ores = [oracle.evaluate_candidate(g, P, w.M, w.C, cd, gg.default_load_edges(), keep_n1=False)
            for cd in cands]
    for i, (label, _, valid) in enumerate(ec.STAR_TABLE):
        assert ores[i].valid is valid, label
        assert bool(o["status"][i] & tto.TTO_ST_INVALID) == (not valid), label
    compare(w, o, range(len(cands)), ores, TOL_F64, strict_discrete=True)
    s.close()


@pytest.mark.parametrize("flow", ["f64", "f32"])
def test_nonfinite_injections(tto, flow):
    """A NaN grid injection, an infinite slack injection and a NaN moved
    amount: candidates the oracle cannot evaluate get INVALID | NONFINITE,
    cell -1 and fitness -inf and never enter the repertoire; encoding-invalid
    and islanded candidates keep those verdicts; with finite grid injections
    the other candidates still match the oracle."""
    import torch
    g, P = _ten_bus()
    cands = [c for _, c, _ in ec.TEN_BUS_TABLE]
    fl, tol = _flow(tto, flow)
    edges = gg.default_load_edges()
    w = _workload(g, P, cands)
    s = make_session(w, fl, max_batch=len(cands))
    db = tto.device_batch(w.batch)
    bad_nan = P.copy()
    bad_nan[4, 1] = np.nan
    bad_inf = P.copy()
    bad_inf[0, 0] = np.inf
    for name, Pb in (("nan", bad_nan), ("inf at the slack", bad_inf)):
        s.set_injections(Pb)
        out = s.evaluate(db)
        arch = s.new_archive()
        s.archive_insert(arch, out)
        o = to_numpy(out)
        torch.cuda.synchronize()
        assert (arch[1].cpu().numpy() == -1).all(), name
        n_nf = 0
        for i, cd in enumerate(cands):
            r = oracle.evaluate_candidate(g, Pb, w.M, w.C, cd, edges, keep_n1=False)
            st = int(o["status"][i])
            if not r.valid and not r.nonfinite:
                assert st == tto.TTO_ST_INVALID, (name, i, st)
            elif r.islanded:
                assert st == tto.TTO_ST_ISLANDED, (name, i, st)
            else:
                assert r.nonfinite, (name, i)
                assert st == tto.TTO_ST_INVALID | tto.TTO_ST_NONFINITE, (name, i, st)
                n_nf += 1
            if st:
                assert o["cell"][i] == -1 and o["fitness"][i] == -np.inf, (name, i)
        log(f"[edge] {name} injection {flow}: {n_nf} candidates flagged non-finite")
        assert n_nf >= 10
    # finite grid injections, one candidate with a NaN moved amount
    T = P.shape[1]
    ns = 8
    mp = np.zeros((len(cands) * ns, T))
    base = [r[0] for r in ec.TEN_BUS_TABLE].index("base: one opening, one split")
    other = [r[0] for r in ec.TEN_BUS_TABLE].index("two splits at distinct buses")
    mp[base * ns + 0] = [5.0, np.nan, 5.0]
    mp[other * ns + 1] = [3.0, -2.0, 1.0]
    w2 = _workload(g, P, cands, moved_p=mp)
    s.set_injections(P)
    o = to_numpy(s.evaluate(tto.device_batch(w2.batch), fmax=True, base_flows=True))
    torch.cuda.synchronize()
    ores = [oracle.evaluate_candidate(g, P, w2.M, w2.C, oracle.candidate_from_batch(w2.batch, i),
                                      edges, keep_n1=True) for i in range(len(cands))]
    assert ores[base].nonfinite and o["status"][base] == tto.TTO_ST_INVALID | tto.TTO_ST_NONFINITE
    keep = [i for i in range(len(cands)) if i != base]
    compare(w2, o, keep, [ores[i] for i in keep], tol, strict_discrete=(flow == "f64"))
    s.close()


def _swapping_candidates(w, S, b, need=3):
    """Candidates of the batch whose set-up LU interchanges rows, each chosen
    pivot beating the diagonal by at least 5% (so rounding cannot undo the
    swap) and far from singular."""
    out = []
    for c in range(w.batch.n_cand):
        cd = oracle.candidate_from_batch(w.batch, c)
        if len(cd.opened) + len(cd.splits) < 2:
            continue
        sw, mp, beat = ec.pivot_swaps(ec.bordered_matrix(S, b, w.grid, cd.opened, cd.splits))
        if sw and mp > 1e-6 and beat > 1.05:
            out.append(c)
        if len(out) >= need:
            break
    return out


@pytest.mark.parametrize("flow", ["f64", "f32"])
def test_setup_lu_row_interchanges_against_oracle(tto, flow):
    """500-bus candidates whose bordered system needs row interchanges (two
    splits with strongly coupled moved branches): every output and the N-1
    flows against the oracle."""
    import torch
    w = gg.build_config(2)
    S, b = ec.sensitivity_s(w.grid)
    pick = _swapping_candidates(w, S, b)
    assert len(pick) >= 2, "no swapping candidate found"
    sub = w.batch.subset(pick)
    ws = gg.Workload(cfg=2, grid=w.grid, P=w.P, M=w.M, C=w.C, batch=sub)
    fl, tol = _flow(tto, flow)
    s = make_session(ws, fl, max_batch=len(pick))
    o = to_numpy(s.evaluate(tto.device_batch(sub), fmax=True, base_flows=True, n1=True))
    torch.cuda.synchronize()
    ores = [oracle.evaluate_candidate(w.grid, w.P, w.M, w.C, oracle.candidate_from_batch(sub, i),
                                      gg.default_load_edges(), keep_n1=True)
            for i in range(len(pick))]
    st = compare(ws, o, range(len(pick)), ores, tol, strict_discrete=(flow == "f64"))
    log(f"[edge] LU interchanges {flow}: candidates {pick}, {st['checked']} checked")
    assert st["checked"] == len(pick)
    s.close()


def test_busbar_lu_row_interchanges_against_oracle(tto):
    """Busbar outages of the swapping candidates: their busbar systems (the
    candidate's openings plus all but one branch of the busbar, then the
    splits) interchange rows too; lambda_b and the islanding count against
    the oracle's re-solves, FP64."""
    import torch
    w = gg.build_config(2)
    g = w.grid
    S, b = ec.sensitivity_s(g)
    pick = _swapping_candidates(w, S, b)
    sub = w.batch.subset(pick)
    inc = g.incident()
    deg = np.array([len(x) for x in inc])
    rng = np.random.default_rng(17)
    ok = [x for x in range(g.n_bus) if x != g.slack and 1 <= deg[x] <= 16]
    buses = np.array(sorted(rng.choice(ok, size=40, replace=False).tolist()), np.int32)
    n_swap = 0
    for i in range(len(pick)):
        cd = oracle.candidate_from_batch(sub, i)
        at = {bb: mv for bb, mv in cd.splits}
        for bus in buses.tolist():
            ids = [x for x in sorted(inc[bus]) if x not in cd.opened and x not in at.get(bus, [])]
            gone = set(ids[:max(len(ids) - 1, 0)])
            sp = [(bb, [e for e in mv if e not in gone]) for bb, mv in cd.splits]
            if any(len(mv) == 0 for _, mv in sp):
                continue
            sw, mp, beat = ec.pivot_swaps(ec.bordered_matrix(
                S, b, g, list(cd.opened) + ids[:max(len(ids) - 1, 0)], sp))
            n_swap += int(sw > 0 and mp > 1e-6 and beat > 1.05)
    assert n_swap > 0
    ws = gg.Workload(cfg=2, grid=g, P=w.P, M=w.M, C=w.C, batch=sub)
    s = make_session(ws, tto.TTO_FLOW_F64, max_batch=len(pick))
    ptdf = tto.ptdf_device(g.n_bus, g.from_bus, g.to_bus, 1.0 / g.x_pu, g.slack)
    bset = s.busbar_set(buses, ptdf)
    db = tto.device_batch(sub)
    out = s.evaluate(db)
    lam, nis, _ = s.busbar_evaluate(bset, db)
    torch.cuda.synchronize()
    lam, nis = lam.cpu().numpy(), nis.cpu().numpy()
    lim = g.limit_mw[w.M]
    for i in range(len(pick)):
        r = oracle.busbar_metrics(g, w.P, w.M, oracle.candidate_from_batch(sub, i), buses)
        assert nis[i] == r["n_island"], i
        bound = TOL_F64 * ((r["fmax"] > lim[:, None] - TOL_F64).sum() + 1)
        assert abs(lam[i] - r["lambda_b"]) <= bound, (i, lam[i], r["lambda_b"])
    log(f"[edge] busbar LU interchanges: {n_swap} swapping (candidate, busbar) systems among "
        f"{len(pick)} x {len(buses)}")
    s.close()
