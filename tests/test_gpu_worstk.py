"""Worst-k contingency export (tto_worst_contingencies) against the oracle's
per-contingency overload energies (re-solved N-1 flows)."""
import numpy as np
import pytest

import gridgen as gg
import oracle
from parity_util import TOL_F32, TOL_F64, log, make_session, oracle_results

pytestmark = pytest.mark.gpu


def _tol_energy(n1, lim, tol):
    """Bound of |E_gpu - E| per contingency: tol for every (e, t) whose flow
    is within tol of (or above) its limit."""
    a = np.abs(np.nan_to_num(n1, nan=0.0))
    return tol * (a > lim[None, :, None] - tol).sum(axis=(1, 2)) + 1e-9


def _check(w, ids, en, idx, ores, K, tol):
    lim = w.grid.limit_mw[w.M]
    C = np.asarray(w.C)
    stats = dict(exact=0, ambiguous=0, island=0)
    for j, c in enumerate(idx):
        r = ores[j]
        gi, ge = ids[c], en[c]
        if not r.valid or r.islanded:
            assert np.all(gi == -1) and np.all(np.isnan(ge)), c
            stats["island"] += 1
            continue
        E = oracle.contingency_energies(r.n1_flows, lim)
        tE = _tol_energy(r.n1_flows, lim, tol)
        want_ids, _ = oracle.worst_k(E, C, K)
        n_ok = int((~np.isnan(E)).sum())
        n_list = min(K, n_ok)
        assert np.all(gi[n_list:] == -1) and np.all(np.isnan(ge[n_list:])), c
        pos = np.array([int(np.flatnonzero(C == v)[0]) for v in gi[:n_list]])
        assert len(set(pos.tolist())) == n_list and not np.isnan(E[pos]).any(), c
        assert np.all(np.abs(ge[:n_list] - E[pos]) <= tE[pos]), (c, ge[:n_list], E[pos])
        assert np.all(np.diff(ge[:n_list]) <= 0), c
        # a valid top-k: nothing left out beats the smallest listed energy
        rest = np.setdiff1d(np.flatnonzero(~np.isnan(E)), pos)
        if rest.size:
            m = int(pos[np.argmin(E[pos])])
            assert np.all(E[rest] <= E[m] + tE[rest] + tE[m]), c
        # unique answer unless two energies near the top lie within tolerance
        srt = sorted(np.flatnonzero(~np.isnan(E)), key=lambda li: (-E[li], li))[: K + 1]
        amb = any(abs(E[a] - E[b]) <= tE[a] + tE[b] and (E[a] > 0 or E[b] > 0)
                  for x, a in enumerate(srt) for b in srt[x + 1:])
        if amb:
            stats["ambiguous"] += 1
        else:
            assert np.array_equal(gi[:n_list], want_ids[:n_list]), (c, gi, want_ids)
            stats["exact"] += 1
    return stats


@pytest.mark.parametrize("cfg,flow,B,K", [(1, "f64", 64, 20), (1, "f64", 64, 64),
                                          (2, "f32", 48, 20), (2, "f64", 24, 20)])
def test_worst_k_matches_oracle(cfg, flow, B, K):
    import torch
    from paper_2605_10128_amd import tto
    w = gg.build_config(cfg, B=B)
    fp = tto.TTO_FLOW_F64 if flow == "f64" else tto.TTO_FLOW_F32
    log(f"[worst-k] cfg{cfg} {flow} B={B} k={K}")
    sess = make_session(w, fp, max_batch=B)
    ids, en = sess.worst_contingencies(tto.device_batch(w.batch), K)
    torch.cuda.synchronize()
    ids, en = ids.cpu().numpy(), en.cpu().numpy()
    idx = list(range(B))
    ores = oracle_results(w, idx, keep_n1=True)
    st = _check(w, ids, en, idx, ores, K, TOL_F64 if flow == "f64" else TOL_F32)
    log(f"  {st}")
    assert st["exact"] >= 1
    sess.close()


def test_worst_k_consistent_with_evaluate():
    """The largest per-contingency energy never exceeds the candidate's N-1
    overload energy, and an opened-branch contingency ranks as the N-0 state."""
    import torch
    from paper_2605_10128_amd import tto
    w = gg.build_config(2, B=256)
    sess = make_session(w, tto.TTO_FLOW_F32, max_batch=256)
    db = tto.device_batch(w.batch)
    out = sess.evaluate(db)
    ids, en = sess.worst_contingencies(db, 8)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    lam = out["overload_mw"].cpu().numpy()
    e0 = en.cpu().numpy()[:, 0]
    ok = (st & 3) == 0
    assert np.all(e0[ok] <= lam[ok] * (1 + 1e-5) + 1e-3)
    assert np.all(np.isnan(e0[~ok]))
    log(f"[worst-k] 256 candidates: max E_l / lambda_o median {np.median(e0[ok & (lam > 0)] / lam[ok & (lam > 0)]):.3f}")
    sess.close()


def test_worst_k_benchmarked_size_sampled():
    """The benchmarked export (2000 buses, T = 24, 1024 candidates, k = 20,
    FP32): for sampled candidates the oracle re-solves the 20 listed
    contingencies and 8 others; the listed energies equal the oracle's
    within tolerance and descend, no listed contingency islands, and no
    unlisted sampled contingency exceeds the 20th energy."""
    import torch
    import oracle
    from paper_2605_10128_amd import tto
    w = gg.build_config(3, B=1024)
    K = 20
    sess = make_session(w, tto.TTO_FLOW_F32, max_batch=1024)
    db = tto.device_batch(w.batch)
    out = sess.evaluate(db)
    ids, en = sess.worst_contingencies(db, K)
    torch.cuda.synchronize()
    ids, en = ids.cpu().numpy(), en.cpu().numpy()
    st = out["status"].cpu().numpy()
    lim = w.grid.limit_mw[w.M]
    edges = gg.default_load_edges()
    rng = np.random.default_rng(20)
    ok = np.flatnonzero((st & 3) == 0)
    checked = 0
    for c in rng.choice(ok, size=4, replace=False):
        c = int(c)
        listed = [int(np.flatnonzero(w.C == i)[0]) for i in ids[c] if i >= 0]
        others = [p for p in rng.choice(len(w.C), size=12, replace=False).tolist()
                  if p not in listed][:8]
        cand = oracle.candidate_from_batch(w.batch, c)
        r = oracle.evaluate_candidate(w.grid, w.P, w.M, w.C, cand, edges, keep_n1=True,
                                      cont_subset=sorted(listed + others))
        assert r.valid and not r.islanded
        E = oracle.contingency_energies(r.n1_flows, lim)
        assert np.all(np.diff(en[c][: len(listed)]) <= 0), c
        for j, p in enumerate(listed):
            assert not np.isnan(E[p]), (c, p)
            n_over = int((np.abs(r.n1_flows[p]) > lim[:, None] - TOL_F32).sum())
            assert abs(en[c][j] - E[p]) <= TOL_F32 * (n_over + 1), (c, p, en[c][j], E[p])
        kth = en[c][len(listed) - 1] if listed else -np.inf
        for p in others:
            if np.isnan(E[p]):
                continue
            n_over = int((np.abs(r.n1_flows[p]) > lim[:, None] - TOL_F32).sum())
            assert E[p] <= kth + TOL_F32 * (n_over + 1), (c, p, E[p], kth)
        checked += 1
    log(f"[worst-k] benchmarked size: 1024 candidates, k = {K}, {checked} sampled candidates "
        f"checked against the oracle")
    sess.close()
