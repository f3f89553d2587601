"""Throughput of the batched DC N-1 topology screen on one MI355X.

One step = one tto_evaluate over the whole candidate batch (set-up, N-1 sweep
with fused reductions, finalize, FP64 refinement) plus the archive update,
inputs resident in HBM.  The K timed steps are launched eagerly with the
library's stage events on the launch stream; the same step replayed as one
captured graph is timed afterwards and reported beside it.  Default workload:
2000-bus / 3200-branch grid, 24 timesteps, 16384 candidates of rank 0..8,
1200 monitored x 1600 contingencies, FP32 flows.

A second leg measures the learned pre-screen inside the MapElites loop on the
same grid: the network is trained on exact evaluations of evolved children
under 8 injection scenarios; on an unseen scenario a screened generation
(65536 children varied, scored, the best-predicted 10% evaluated exactly and
inserted) runs as one captured graph; it reports the screened rate next to
the exact one, the network's error and recall on evolved children, and the
repertoires reached by screened and exact-only generations at an equal
exact-evaluation budget.

Prints one JSON line.  `python bench.py --copy-calibration` instead runs a
plain 1 GiB device copy, the reference for scaling HBM byte counters.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "N-1-evaluated topologies/sec, 2000-bus grid; surrogate-screened vs exact"
# MI355X: 256 CUs x 64 VALU lanes x 2.4 GHz (non-packed issue rate)
VALU_PEAK_T = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sweep_alg_ops(T, n_mon, n_act, rank):
    """Minimal VALU lane-instructions of the N-1 sweep for one candidate:
    per (e, l, t) one FMA and half of a 3-input max (two flows per max), per
    (e, l) one FMA per rank for H'_el."""
    return n_mon * n_act * (1.5 * T + rank)


def kernel_hash():
    h = hashlib.sha256()
    for f in ("k_eval.hip", "tto_common.h"):
        h.update(open(os.path.join(ROOT, "paper_2605_10128_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def cpu_baseline(w):
    """Time the oracle as it stands on a bounded sample of the same workload:
    one whole candidate (N-0 plus every contingency re-solved from scratch)
    per host core, one single-threaded worker process per core.  Runs before
    the process touches the GPU, so that the workers fork from a plain host
    process."""
    import gridgen as gg
    import oracle
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cores = max(1, min(16, avail))
    nC = len(w.C)
    idx = list(range(cores))
    t0 = time.perf_counter()
    oracle.evaluate_batch(w.grid, w.P, w.M, w.C, w.batch, gg.default_load_edges(), idx=idx,
                          processes=cores, keep_n1=False)
    dt = time.perf_counter() - t0
    solves = cores * (nC + 1)
    return {"value": cores / dt, "unit": "topologies/s", "cores": cores, "kind": "oracle",
            "sample": f"candidates 0..{cores - 1} of the workload, each with N-0 and all {nC} "
                      f"contingencies re-solved (sparse LU, {w.P.shape[1]} right-hand sides), "
                      f"{cores} single-threaded processes, {dt:.1f} s wall, "
                      f"{dt * cores / solves * 1e3:.1f} ms per re-solve per core"}


def copy_calibration():
    """A plain 1 GiB device-to-device copy (reference for HBM byte counters)."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] copied {a.numel() * 4} bytes")


def surrogate_leg(s, w, args, exact_rate):
    """The learned pre-screen inside the MapElites loop (Alg. 3).

    Training data are exact evaluations of evolved children that the DC
    evaluator itself produces: exact-only generations (16384 children each)
    under 8 injection scenarios.  On an unseen scenario, one screened
    generation (65536 children varied on the device, scored by the network,
    the best-predicted tenth evaluated exactly and inserted) is captured as a
    graph and timed; then screened and exact-only generations run from empty
    repertoires at an equal exact-evaluation budget (6554 children evaluated
    exactly per generation), and the repertoires they reach are compared.
    Finally the 65536 children of one screened generation are all evaluated
    exactly to measure the network's error and the screen's recall."""
    import numpy as np
    import torch
    import gridgen as gg
    from paper_2605_10128_amd import tto, screen
    grid, T, B = w.grid, w.P.shape[1], s.max_batch
    n_scen = 8
    n_gen = args.screen
    keep = max(1, int(round(args.keep_frac * n_gen)))
    if keep > B:
        raise SystemExit(f"keep {keep} exceeds the evaluation batch {B}")
    D = np.flatnonzero(~gg.bridges(grid.n_bus, grid.from_bus, grid.to_bus))
    bus = np.array([b_ for b_, _ in w.split_table])
    moved = [mv for _, mv in w.split_table]
    gs = tto.GenomeSpace(s, bus, moved, D, args.evo_slots, args.evo_slots)
    n_disc, n_act = len(D), len(bus)
    d_bits = n_disc + n_act
    scen = [gg.make_injections(grid, T, 0x7000 + i) for i in range(n_scen + 1)]
    scale = screen.FeatureScale.fit([screen.injection_summary(P) for P in scen[:n_scen]])
    gens_per_scen = max(1, args.train_samples // (n_scen * B))
    out = s.alloc_outputs(B)
    parts, t_eval, t0 = [], 0.0, time.perf_counter()
    for i in range(n_scen):
        s.set_injections(scen[i])
        ref = screen.unswitched_reference(s)
        rep = tto.Repertoire(s, gs)
        evo = tto.Evolver(s, gs, rep, B, seed=0x5C00 + i, outputs=out)
        for _ in range(gens_per_scen):
            torch.cuda.synchronize()
            te = time.perf_counter()
            evo.step()
            torch.cuda.synchronize()
            t_eval += time.perf_counter() - te
            off, ids = screen.genome_bits(evo.children.cpu().numpy(), gs.n_a, n_disc, n_act)
            t_, ok_ = screen.targets_from_outputs(out, ref)
            parts.append([off, ids, scale.apply(screen.injection_summary(scen[i])), t_, ok_])
    n_train = n_scen * gens_per_scen * B
    tscale = screen.TargetScale.fit(np.concatenate([q[3] for q in parts]),
                                    np.concatenate([q[4] for q in parts]))
    for q in parts:
        q[3] = tscale.apply(q[3])
    data = screen.Dataset.assemble(parts, seed=1)
    log(f"[bench] surrogate data: {n_train} exact evaluations of evolved children "
        f"({data.n} usable) in {time.perf_counter() - t0:.1f} s ({t_eval:.1f} s on the GPU)")
    sc = screen.Screener(s, d_bits, T, width=512, max_screen=n_gen, max_keep=keep)
    t0 = time.perf_counter()
    losses = sc.train(data, epochs=args.epochs, batch=4096, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"[bench] surrogate trained: losses {['%.4f' % x for x in losses]} in {t_train:.1f} s")

    # unseen scenario: the screened generation as one captured graph
    P = scen[-1]
    s.set_injections(P)
    ref_h = screen.unswitched_reference(s)
    row = scale.apply(screen.injection_summary(P))
    stream = torch.cuda.current_stream()
    so = s.alloc_outputs(keep)
    rep_t = tto.Repertoire(s, gs)
    gain = dict(rule=tto.TTO_SCREEN_GAIN, y_mu=tuple(tscale.mu), y_sd=tuple(tscale.sd),
                ref=tuple(ref_h), overload_scale_mw=screen.OVERLOAD_SCALE_MW)
    sev = tto.ScreenedEvolver(s, gs, rep_t, sc.net, n_gen, keep, seed=0xC0DE, dense_row=row,
                              outputs=so, **gain)
    for _ in range(2):
        sev.step()
    with tto.Graph() as graph:
        sev.step()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.screen_steps):
        graph.launch()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_gen = e0.elapsed_time(e1) / args.screen_steps
    graph.close()
    # the same generation without the screen, evaluating as many children exactly
    rep_x = tto.Repertoire(s, gs)
    xev = tto.Evolver(s, gs, rep_x, keep, seed=0xC0DE)
    for _ in range(2):
        xev.step()
    with tto.Graph() as graph:
        xev.step()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.screen_steps):
        graph.launch()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_exact_keep = e0.elapsed_time(e1) / args.screen_steps
    graph.close()

    # equal exact budget from empty repertoires: exact-only generations of
    # `keep` children against screened generations of n_gen children under
    # both screen rules
    G = args.loop_generations
    runs = {"exact_only": None, "screened_gain": gain, "screened_overload": {}}
    reps, evs = {}, {}
    for name, rule in runs.items():
        reps[name] = tto.Repertoire(s, gs)
        if rule is None:
            evs[name] = tto.Evolver(s, gs, reps[name], keep, seed=0xA11)
        else:
            evs[name] = tto.ScreenedEvolver(s, gs, reps[name], sc.net, n_gen, keep, seed=0xA11,
                                            dense_row=row, **rule)
    curve = []
    for g in range(G):
        for name in runs:
            evs[name].step()
        if (g + 1) % max(1, G // 4) == 0 or g + 1 == G:
            torch.cuda.synchronize()
            curve.append([g + 1] + [int((reps[n].id >= 0).sum().item()) for n in runs])
    torch.cuda.synchronize()
    fit_of = {n: reps[n].fitness.cpu().numpy() for n in runs}
    occ_of = {n: reps[n].id.cpu().numpy() >= 0 for n in runs}
    loop = {"generations": G, "exact_evaluations_each": G * keep,
            "cells_curve_columns": ["generation"] + list(runs), "cells_curve": curve}
    fe, oe = fit_of["exact_only"], occ_of["exact_only"]
    for n in runs:
        f, o = fit_of[n], occ_of[n]
        both = o & oe
        loop[n] = {"cells_filled": int(o.sum()), "best_fitness": float(f[o].max()),
                   "mean_elite_fitness": float(f[o].mean())}
        if n != "exact_only":
            loop[n].update({
                "cells_both_with_exact_only": int(both.sum()),
                "elite_better_than_exact_only": int((f[both] > fe[both]).sum()),
                "elite_worse_than_exact_only": int((f[both] < fe[both]).sum()),
                "mean_fitness_gain_common_cells":
                    float((f[both] - fe[both]).mean()) if both.any() else None})
    log("[bench] screened loop: " + ", ".join(
        f"{n} {loop[n]['cells_filled']} cells best {loop[n]['best_fitness']:.0f}" for n in runs)
        + f" ({G} generations, {G * keep} exact evaluations each)")

    # the network on one generation of evolved children, all evaluated exactly
    rep_m = tto.Repertoire(s, gs)
    ev_m = tto.ScreenedEvolver(s, gs, rep_m, sc.net, n_gen, keep, seed=0xA11, dense_row=row,
                               **gain)
    for _ in range(G):
        ev_m.step()
    kids, _ = gs.vary(rep_m, 0xA11, n_gen)
    torch.cuda.synchronize()
    kids_h = kids.cpu().numpy()
    exact = {}
    for c0 in range(0, n_gen, B):
        n = min(B, n_gen - c0)
        o = s.evaluate(gs.expand(kids[c0:c0 + n].contiguous()))
        for k, v in o.items():
            exact.setdefault(k, []).append(v.cpu().numpy())
    exact = {k: np.concatenate(v) for k, v in exact.items()}
    off, ids = screen.genome_bits(kids_h, gs.n_a, n_disc, n_act)
    dev = s.device
    dense_d = sc.dense_rows(scale, P, n_gen)
    sc.predict(torch.as_tensor(off, device=dev), torch.as_tensor(ids, device=dev), dense_d, n_gen)
    idx = np.sort(sc.select(n_gen, keep).cpu().numpy())
    y = tscale.invert(sc.y[:n_gen].cpu().numpy()) + ref_h[None, :]
    valid = (exact["status"] & 3) == 0
    truth = screen.raw_targets(exact["max_loading"], exact["overload_mw"])
    fit = np.where(valid, exact["fitness"], -np.inf)
    best = np.argsort(-fit, kind="stable")[:keep]
    recall = len(np.intersect1d(best, idx)) / keep
    lam = np.where(valid, exact["overload_mw"], np.inf)
    m_all, m_scr = exact["overload_mw"][valid].mean(), exact["overload_mw"][idx][valid[idx]].mean()
    m_best = lam[np.argsort(lam, kind="stable")[:keep]].mean()
    scr_rate = n_gen / (ms_gen / 1e3)
    res = {
        "value": scr_rate,
        "unit": "screened topologies/s",
        "ms_per_generation": ms_gen,
        "launch": "hipGraph replay of one screened generation (vary 65536, features, forward, "
                  "the 10% with the largest predicted gain over their predicted cells' elites, "
                  "expand, exact evaluation, insertion)",
        "generation": n_gen,
        "exactly_evaluated": keep,
        "vs_exact_only": scr_rate / exact_rate,
        "exact_only_generation_of_kept_size_ms": ms_exact_keep,
        "screen_overhead_ms": ms_gen - ms_exact_keep,
        "train": {"exact_evaluations": n_train, "usable": int(data.n),
                  "source": f"exact-only MapElites generations of {B} children, "
                            f"{gens_per_scen} per scenario",
                  "scenarios": n_scen, "epochs": args.epochs, "final_loss": losses[-1],
                  "train_s": t_train, "gpu_eval_s": t_eval, "width": 512,
                  "bits": d_bits, "dense": T},
        "error_unseen_scenario": {
            "children": "one generation of evolved children of a screened run",
            "max_loading_mae": float(np.abs(y[valid, 0] - truth[valid, 0]).mean()),
            "log_overload_mae": float(np.abs(y[valid, 1] - truth[valid, 1]).mean()),
            "log_overload_corr": float(np.corrcoef(y[valid, 1], truth[valid, 1])[0, 1]),
        },
        "recall_top10pct_fitness": recall,
        "overload_mw": {"screened_tenth": float(m_scr), "all": float(m_all),
                        "best_tenth": float(m_best),
                        "screen_efficiency": float((m_all - m_scr) / max(m_all - m_best, 1e-9))},
        "loop_equal_exact_budget": loop,
    }
    log(f"[bench] screened: {scr_rate:,.0f} topologies/s ({ms_gen:.2f} ms per {n_gen}; exact-only "
        f"generation of {keep}: {ms_exact_keep:.2f} ms), recall {recall:.3f}")
    gs.close()
    return res


def busbar_leg(s, w, ptdf, n_busbars=128, reps=3):
    """Busbar outages (lambda_b, lambda_f2) over the whole batch for a seeded
    busbar set: set-up, one FP64 bordered system per (candidate, busbar) and
    the busbar-outage sweep."""
    import numpy as np
    import torch
    import gridgen as gg
    from paper_2605_10128_amd import tto
    g = w.grid
    buses = gg.select_busbars(g, n_busbars, seed=0xBB00 + w.cfg)
    bset = s.busbar_set(buses, ptdf)
    db = tto.device_batch(w.batch)
    out = s.evaluate(db)
    empty = tto.device_batch(w.batch.subset(np.zeros(1, dtype=np.int64)))
    empty.open.fill_(-1)
    empty.split_bus.fill_(-1)
    pre_l, _, _ = s.busbar_evaluate(bset, empty)
    torch.cuda.synchronize()
    pre = float(pre_l.item())
    s.busbar_evaluate(bset, db, pre, out["fitness"])
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        lam, nis, f2 = s.busbar_evaluate(bset, db, pre, out["fitness"])
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    B = w.batch.n_cand
    lam, nis, f2 = lam.cpu().numpy(), nis.cpu().numpy(), f2.cpu().numpy()
    f1 = out["fitness"].cpu().numpy()
    ok = np.isfinite(lam)
    log(f"[bench] busbar outages: {len(buses)} busbars x {B} candidates in {ms:.2f} ms "
        f"({B / (ms / 1e3):,.0f} topologies/s), lambda_b_pre {pre:.1f} MW")
    bset.close()
    return {"busbars": int(len(buses)), "candidates": B, "ms": ms,
            "value": B / (ms / 1e3), "unit": "topologies/s (lambda_b of every candidate)",
            "lambda_b_pre_mw": pre,
            "lambda_b_median_mw": float(np.median(lam[ok])) if ok.any() else None,
            "islanding_outages_mean": float(nis[ok].mean()) if ok.any() else None,
            "f2_below_f1": int((f2[ok] < f1[ok]).sum()),
            "note": "set-up, an FP64 bordered system per (candidate, busbar), FP32 busbar sweep"}


def worst_k_leg(s, w, n=1024, k=20, reps=3):
    """Worst-k export (tto_worst_contingencies) for n candidates of the
    workload: set-up plus one energy per (candidate, contingency)."""
    import numpy as np
    import torch
    from paper_2605_10128_amd import tto
    n = min(n, w.batch.n_cand)
    db = tto.device_batch(w.batch.subset(np.arange(n)))
    s.worst_contingencies(db, k)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        ids, en = s.worst_contingencies(db, k)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    e = en.cpu().numpy()
    log(f"[bench] worst-{k} export of {n} candidates: {ms:.2f} ms")
    return {"candidates": n, "k": k, "ms": ms,
            "median_top_energy_mw": float(np.nanmedian(e[:, 0])),
            "note": "set-up plus the overload energy of every (candidate, contingency)"}


def evolution_leg(s, w, args):
    """MapElites generations on the device (Alg. 3 with Alg. 1 and 2): one
    generation (vary, expand, evaluate, insert) captured as a graph and
    replayed for an epoch; the variation kernels are also timed alone."""
    import numpy as np
    import torch
    import gridgen as gg
    from paper_2605_10128_amd import tto

    g = w.grid
    B = w.batch.n_cand
    s.set_injections(w.P)          # the screened leg leaves another scenario installed
    D = np.flatnonzero(~gg.bridges(g.n_bus, g.from_bus, g.to_bus))
    bus = np.array([b for b, _ in w.split_table])
    moved = [mv for _, mv in w.split_table]
    gs = tto.GenomeSpace(s, bus, moved, D, args.evo_slots, args.evo_slots)
    rep = tto.Repertoire(s, gs)
    outs = s.alloc_outputs(B)
    evo = tto.Evolver(s, gs, rep, B, seed=0xE701, outputs=outs)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        evo.step()
    torch.cuda.synchronize()
    # variation alone: tto_vary + tto_genome_expand on the generation's buffers
    kids = torch.empty((B, gs.G), dtype=torch.int32, device=s.device)
    bmc = torch.empty(1, dtype=torch.int32, device=s.device)
    op = torch.empty((B, gs.n_d), dtype=torch.int32, device=s.device)
    sb = torch.empty((B, gs.n_a), dtype=torch.int32, device=s.device)
    mo = torch.empty(B * gs.n_a + 1, dtype=torch.int32, device=s.device)
    cap = max(1, B * gs.max_moved)
    mb = torch.empty(cap, dtype=torch.int32, device=s.device)
    v0, v1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    v0.record(stream)
    for _ in range(reps):
        tto.tto_vary(gs.handle, rep.id.data_ptr(), rep.genome.data_ptr(), rep.n_cells, 0xE701,
                     rep.generation.data_ptr(), B, kids.data_ptr(), bmc.data_ptr(), s.stream)
        tto.tto_genome_expand(gs.handle, kids.data_ptr(), B, op.data_ptr(), sb.data_ptr(),
                              mo.data_ptr(), mb.data_ptr(), cap, s.stream)
    v1.record(stream)
    torch.cuda.synchronize()
    vary_ms = v0.elapsed_time(v1) / reps
    with tto.Graph() as graph:
        evo.step()
    K = args.evo_generations
    gen0 = int(rep.generation.item())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(K):
        graph.launch()
    e1.record(stream)
    torch.cuda.synchronize()
    graph.close()
    ms_gen = e0.elapsed_time(e1) / K
    ids = rep.id.cpu().numpy()
    fit = rep.fitness.cpu().numpy()
    occ = ids >= 0
    st = outs["status"].cpu().numpy()
    ch = evo.children.cpu().numpy()
    # end of an epoch: the elites' worst-20 contingencies for the AC validator
    elites = rep.genome[torch.as_tensor(np.flatnonzero(occ), device=s.device)].contiguous()
    w0, w1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0.record(stream)
    edb = gs.expand(elites)
    wk_ids, wk_en = s.worst_contingencies(edb, 20)
    w1.record(stream)
    torch.cuda.synchronize()
    export_ms = w0.elapsed_time(w1)
    res = {
        "value": B / (ms_gen / 1e3),
        "unit": "evaluated children/s",
        "ms_per_generation": ms_gen,
        "children_per_generation": B,
        "generations_replayed": K,
        "launch": "hipGraph replay of one generation (vary, expand, evaluate, insert)",
        "slots": {"actions": gs.n_a, "disconnections": gs.n_d, "|A|": len(bus), "|D|": len(D)},
        "variation_ms": vary_ms,
        "variation_frac": vary_ms / ms_gen,
        "generation_counter": int(rep.generation.item()),
        "counter_advanced": int(rep.generation.item()) - gen0,
        "cells_filled": int(occ.sum()),
        "best_fitness": float(fit[occ].max()) if occ.any() else None,
        "mean_elite_fitness": float(fit[occ].mean()) if occ.any() else None,
        "elite_worst20_export_ms": export_ms,
        "elite_worst20_top_energy_mw": float(np.nanmax(wk_en[:, 0].cpu().numpy())) if occ.any() else None,
        "last_generation": {
            "mutated": int(evo.b_mc.item()),
            "mean_filled_slots": float((ch != -1).sum(1).mean()),
            "invalid": int(((st & 2) != 0).sum()),
            "islanded": int(((st & 3) == 1).sum()),
        },
    }
    log(f"[bench] evolution: {ms_gen:.2f} ms per generation of {B} ({res['value']:,.0f} children/s), "
        f"variation {vary_ms:.3f} ms, {res['cells_filled']} cells after {res['generation_counter']} generations")
    # the same loop on the paper's (disconnections, splits, reassigned assets) map
    s.set_descriptor(gg.default_load_edges(), kind=tto.TTO_DESC_PAPER)
    rep2 = tto.Repertoire(s, gs)
    evo2 = tto.Evolver(s, gs, rep2, B, seed=0xE702)
    for _ in range(K):
        evo2.step()
    torch.cuda.synchronize()
    ids2, fit2 = rep2.id.cpu().numpy(), rep2.fitness.cpu().numpy()
    occ2 = ids2 >= 0
    res["paper_map"] = {"cells": tto.TTO_PAPER_CELLS, "generations": K,
                        "cells_filled": int(occ2.sum()),
                        "best_fitness": float(fit2[occ2].max()) if occ2.any() else None}
    log(f"[bench] evolution on the paper map: {int(occ2.sum())} of {tto.TTO_PAPER_CELLS} cells after {K} generations")
    s.set_descriptor(gg.default_load_edges())
    gs.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--flow", choices=["f32", "f64"], default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plan", default="auto",
                    help="sweep plan 'auto' (autotune) or 'lanes,branches_per_lane,order,persistent', "
                         "e.g. 256,2,1,0")
    ap.add_argument("--sweep-plans", action="store_true",
                    help="also report the sweep time of every plan (stderr)")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay check")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the screened leg")
    ap.add_argument("--train-samples", type=int, default=1 << 20)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--loop-generations", type=int, default=24,
                    help="generations of the screened vs exact-only comparison")
    ap.add_argument("--screen", type=int, default=65536)
    ap.add_argument("--keep-frac", type=float, default=0.1)
    ap.add_argument("--screen-steps", type=int, default=10)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-evolution", action="store_true", help="skip the MapElites leg")
    ap.add_argument("--no-busbar", action="store_true", help="skip the busbar-outage leg")
    ap.add_argument("--evo-generations", type=int, default=20)
    ap.add_argument("--evo-slots", type=int, default=4)
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU only; --gpus must be 1 (candidates would "
                                   "shard along the batch across GPUs, not implemented)"}))
        sys.exit(2)

    import numpy as np
    import torch
    import gridgen as gg
    from paper_2605_10128_amd import tto

    spec = gg.CONFIGS[args.config]
    t0 = time.perf_counter()
    w = gg.build_config(args.config, B=args.batch)
    B = w.batch.n_cand
    log(f"[bench] workload cfg{args.config} B={B} built in {time.perf_counter() - t0:.1f}s")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle sample), before the first GPU call")
        cpu = cpu_baseline(w)
        log(f"[bench] cpu baseline {cpu['value']:.4f} topologies/s: {cpu['sample']}")
    torch.cuda.set_device(0)
    g = w.grid
    b = 1.0 / g.x_pu
    # importer on the GPU; the first build also loads the library's code objects,
    # so the reported build time is that of a second build
    ptdf = tto.ptdf_device(g.n_bus, g.from_bus, g.to_bus, b, g.slack)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ptdf = tto.ptdf_device(g.n_bus, g.from_bus, g.to_bus, b, g.slack)
    torch.cuda.synchronize()
    ptdf_ms = (time.perf_counter() - t0) * 1e3
    flow = tto.TTO_FLOW_F32 if args.flow == "f32" else tto.TTO_FLOW_F64
    gemm = tto.TTO_GEMM_F32 if args.flow == "f32" else tto.TTO_GEMM_F64
    s = tto.Session(g.n_bus, g.from_bus, g.to_bus, b, g.limit_mw, ptdf, w.M, w.C, w.P.shape[1],
                    flow_precision=flow, gemm_precision=gemm, max_batch=B)
    s.set_injections(w.P)
    s.set_descriptor(gg.default_load_edges())
    db = tto.device_batch(w.batch)
    out = s.alloc_outputs(B)
    arch = s.new_archive()
    stream = torch.cuda.current_stream()
    log(f"[bench] grid ready; ws grid {s.grid_bytes/2**30:.2f} GiB batch {s.batch_bytes/2**30:.2f} GiB")
    if args.sweep_plans:
        tto.tto_profile_enable(s.handle, True)
        for npl in (1, 2):
            for order in (0, 1, 2):
                s.set_sweep_plan(256, npl, order, False)
                ts = []
                for _ in range(3):
                    s.evaluate(db, out)
                    ts.append(tto.tto_profile_read(s.handle)[1])
                log(f"[bench] plan npl={npl} order={order}: sweep {sorted(ts)[1]:.3f} ms")
        tto.tto_profile_enable(s.handle, False)
    if args.plan == "auto":
        chosen = s.autotune(db, out)   # untimed: picks the sweep launch shape
    else:
        lanes, npl, order, p = (int(v) for v in args.plan.split(","))
        s.set_sweep_plan(lanes, npl, order, bool(p))
        chosen = {"lanes": lanes, "branches_per_lane": npl, "order": order, "persistent": bool(p),
                  "from_cache": False}
    log(f"[bench] sweep plan {chosen}")

    for i in range(args.warmup):
        s.evaluate(db, out)
        s.archive_insert(arch, out, id_base=i * B)
    torch.cuda.synchronize()
    log("[bench] warmup done")

    # timed region: K eager steps, each with the library's stage events on
    # the launch stream (the sweep's duration for the roofline)
    tto.tto_profile_enable(s.handle, True)
    sweep_ms, setup_ms, fin_ms, ref_ms = [], [], [], []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for i in range(args.steps):
        s.evaluate(db, out)
        s.archive_insert(arch, out, id_base=(args.warmup + i) * B)
        ms = tto.tto_profile_read(s.handle)   # waits for this step's events only
        setup_ms.append(ms[0]); sweep_ms.append(ms[1]); fin_ms.append(ms[2]); ref_ms.append(ms[3])
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    tto.tto_profile_enable(s.handle, False)
    # the same step replayed as one captured graph (evaluate + archive)
    graph_ms = None
    if not args.no_graph:
        try:
            graph = s.capture_evaluate(db, out, arch, id_base=(args.warmup + args.steps) * B)
            graph.launch()
            torch.cuda.synchronize()
            g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            g0.record(stream)
            for _ in range(args.steps):
                graph.launch()
            g1.record(stream)
            torch.cuda.synchronize()
            graph_ms = g0.elapsed_time(g1) / args.steps
            graph.close()
        except tto.TTOError as e:
            log(f"[bench] graph capture unavailable ({e})")
    ms_step = total_ms / args.steps
    value = B * args.steps / (total_ms / 1e3)
    log(f"[bench] {ms_step:.3f} ms/step, {value:,.0f} topologies/s; stage ms "
        f"setup {np.mean(setup_ms):.3f} sweep {np.mean(sweep_ms):.3f} fin {np.mean(fin_ms):.3f} "
        f"refine {np.mean(ref_ms):.3f}")

    o = {k: v.cpu().numpy() for k, v in out.items()}
    ok = (o["status"] & 3) == 0
    r = (w.batch.open != -1).sum(1) + (w.batch.split_bus != -1).sum(1)
    n_act = len(w.C) - o["n_island_cont"]
    T = w.P.shape[1]
    ops = float(sum(sweep_alg_ops(T, len(w.M), int(n_act[c]), int(r[c]))
                    for c in range(B) if ok[c]))
    sweep_s = float(np.mean(sweep_ms)) / 1e3
    achieved = ops / sweep_s / 1e12
    traffic = None
    cpath = os.path.join(ROOT, "profiles", f"sweep_cfg{args.config}_{args.flow}_counters.json")
    if os.path.exists(cpath):
        cj = json.load(open(cpath))
        if cj.get("kernel_hash") == kernel_hash():
            traffic = cj.get("hbm_bytes_per_launch")
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "topologies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.flow == "f32" else "f64",
        "data": "synthetic",
        "config": {
            "ptdf_build_ms": ptdf_ms,
            "workload": f"{spec['name']}: n={g.n_bus}, m={g.n_branch}, T={T}, B={B}, "
                        f"|M|={len(w.M)}, |C|={len(w.C)}, rank 0..8 (exact evaluation)",
            "flow_precision": args.flow,
            "candidates_ok": int(ok.sum()),
            "sweep_plan": {k: chosen[k] for k in ("lanes", "branches_per_lane", "order",
                                                  "persistent")},
            "launch": "eager (timed), graph replay checked",
            "graph_replay_ms_per_step": graph_ms,
            "islanded": int(((o["status"] & 1) != 0).sum()),
            "refined_fp64": int(((o["status"] & 4) != 0).sum()),
            "refine_skipped": int(((o["status"] & 8) != 0).sum()),
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_sweep",
            "achieved": achieved,
            "peak": VALU_PEAK_T,
            "unit": "T VALU-instr/s",
            "frac": achieved / VALU_PEAK_T,
            "traffic": traffic,
            "sweep_ms": float(np.mean(sweep_ms)),
            "setup_ms": float(np.mean(setup_ms)),
            "finalize_ms": float(np.mean(fin_ms)),
            "refine_ms": float(np.mean(ref_ms)),
        },
        "cpu_baseline": None,
        "surrogate_screened": None,
        "evolution": None,
        "worst_k": None,
        "busbar": None,
    }
    if not args.no_surrogate:
        result["surrogate_screened"] = surrogate_leg(s, w, args, value)
    if not args.no_evolution and w.split_table:
        result["evolution"] = evolution_leg(s, w, args)
    if not args.no_evolution:
        result["worst_k"] = worst_k_leg(s, w)
    if not args.no_busbar:
        s.set_injections(w.P)
        result["busbar"] = busbar_leg(s, w, ptdf)
    result["cpu_baseline"] = cpu
    print(json.dumps(result))


if __name__ == "__main__":
    main()
