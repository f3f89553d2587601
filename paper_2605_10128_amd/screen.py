"""Learned pre-screen of a MapElites generation (argument marshalling only).

A generation of candidates is scored by the surrogate network
(tto_mlp_forward), the k most promising are picked on the device
(tto_topk_smallest over the predicted overload), compacted into a batch
(tto_batch_gather) and only those are evaluated exactly (tto_evaluate) and
offered to the archive.  The network is trained on exact evaluations the DC
evaluator itself produces.  The network's forward and backward passes, the
optimiser, the selection, the gather and the evaluation run in the library's
kernels; the data preparation around them (the injection summary, the
training targets taken from exact outputs and their standardisation) is host
NumPy in this module.

The paper scores every mutated candidate exactly (DC-Optimizer section);
the screen is an addition for large generations.  Feature encoding: one bit
per base non-bridge opening and one per split action of the action table
(the paper's reconfiguration action set, Importer section), plus the
per-timestep total positive injection, standardised.  Targets: maximum
loading (it places a candidate in its descriptor cell) and log1p(overload
energy / 100 MW) (the dominant term of the fitness), each taken relative to
the unswitched grid under the same injections (what the actions change,
which is all a screen within one generation needs) and standardised over the
training set.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import tto

OVERLOAD_SCALE_MW = 100.0


def injection_summary(P) -> np.ndarray:
    """Per-timestep total positive injection [T] (MW) of one scenario."""
    P = np.asarray(P, dtype=np.float64)
    return np.clip(P, 0.0, None).sum(axis=0)


@dataclass
class FeatureScale:
    mu: float
    sd: float

    @staticmethod
    def fit(summaries) -> "FeatureScale":
        a = np.concatenate([np.ravel(s) for s in summaries])
        return FeatureScale(float(a.mean()), float(max(a.std(), 1e-9)))

    def apply(self, summary) -> np.ndarray:
        return ((np.asarray(summary, dtype=np.float64) - self.mu) / self.sd).astype(np.float32)


def raw_targets(rho, overload_mw):
    """(maximum loading, log1p(overload / 100 MW)) as float64 columns."""
    rho = np.asarray(rho, dtype=np.float64)
    lam = np.maximum(np.asarray(overload_mw, dtype=np.float64), 0.0)
    return np.stack([rho, np.log1p(lam / OVERLOAD_SCALE_MW)], axis=-1)


def unswitched_reference(session: tto.Session):
    """Raw targets of the unswitched grid under the session's current
    injections (one exact evaluation of the empty candidate)."""
    torch = session.torch
    d = session.device
    empty = tto.DeviceBatch(1, torch.full((1, 1), -1, dtype=torch.int32, device=d),
                            torch.full((1, 1), -1, dtype=torch.int32, device=d),
                            torch.zeros(2, dtype=torch.int32, device=d),
                            torch.zeros(1, dtype=torch.int32, device=d), None)
    o = session.evaluate(empty)
    if int(o["status"][0].item()) & 3:
        raise RuntimeError("the unswitched grid is islanded or invalid")
    return raw_targets(o["max_loading"].cpu().numpy(), o["overload_mw"].cpu().numpy())[0]


def targets_from_outputs(out: dict, reference=None):
    """(targets [B][2] float32, usable mask) from tto_evaluate outputs,
    relative to `reference` (raw targets of the unswitched grid) if given."""
    st = out["status"].cpu().numpy()
    t = raw_targets(out["max_loading"].cpu().numpy(), out["overload_mw"].cpu().numpy())
    if reference is not None:
        t = t - np.asarray(reference, dtype=np.float64)[None, :]
    ok = (st & 3) == 0
    return np.where(ok[:, None], t, 0.0).astype(np.float32), ok


@dataclass
class TargetScale:
    """Per-column mean and deviation of the training targets."""
    mu: np.ndarray
    sd: np.ndarray

    @staticmethod
    def fit(targets, mask) -> "TargetScale":
        t = np.asarray(targets, dtype=np.float64)[np.asarray(mask, bool)]
        return TargetScale(t.mean(axis=0), np.maximum(t.std(axis=0), 1e-9))

    def apply(self, t) -> np.ndarray:
        return ((np.asarray(t, dtype=np.float64) - self.mu) / self.sd).astype(np.float32)

    def invert(self, y) -> np.ndarray:
        return np.asarray(y, dtype=np.float64) * self.sd + self.mu


def genome_bits(genomes, n_a: int, n_disc: int, n_actions: int):
    """Feature rows of genomes [n][n_a + n_d] as CSR (offsets, ids), the
    vocabulary of the device's screened generation: action a -> bit
    n_disc + a, disconnection d (an index into D) -> bit d; empty and
    out-of-range slots give no bit."""
    g = np.asarray(genomes, dtype=np.int64)
    a, d = g[:, :n_a], g[:, n_a:]
    ids = np.concatenate([np.where((a >= 0) & (a < n_actions), n_disc + a, -1),
                          np.where((d >= 0) & (d < n_disc), d, -1)], axis=1)
    big = np.iinfo(np.int64).max
    ids = np.sort(np.where(ids >= 0, ids, big), axis=1)
    ok = ids != big
    # repeated entries of a row give one bit (the network reads a set)
    ok[:, 1:] &= ids[:, 1:] != ids[:, :-1]
    off = np.concatenate([[0], np.cumsum(ok.sum(axis=1))]).astype(np.int32)
    return off, ids[ok].astype(np.int32)


class Dataset:
    """Training samples on the device: CSR bits, dense rows, targets."""

    def __init__(self, off, ids, dense, target, device="cuda"):
        import torch
        self.n = int(len(off) - 1)
        self.off = torch.as_tensor(np.ascontiguousarray(off, dtype=np.int32), device=device)
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        self.ids = torch.as_tensor(ids if ids.size else np.zeros(1, np.int32), device=device)
        self.dense = torch.as_tensor(np.ascontiguousarray(dense, dtype=np.float32), device=device)
        self.target = torch.as_tensor(np.ascontiguousarray(target, dtype=np.float32),
                                      device=device)

    @staticmethod
    def assemble(parts, seed=0, device="cuda") -> "Dataset":
        """parts: list of (off, ids, dense_row [d], targets [B][2], mask [B]).
        Concatenates the usable rows of every part in a seeded random order."""
        rows_off, rows_ids, rows_dense, rows_t = [], [], [], []
        for off, ids, drow, t, ok in parts:
            sel = np.flatnonzero(ok)
            lens = (off[1:] - off[:-1])[sel]
            starts = off[:-1][sel]
            rep = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
            flat = ids[np.arange(int(lens.sum())) + rep] if lens.sum() else np.zeros(0, np.int32)
            rows_off.append(lens)
            rows_ids.append((flat, lens))
            rows_dense.append(np.repeat(np.asarray(drow, np.float32)[None, :], len(sel), axis=0))
            rows_t.append(t[sel])
        lens = np.concatenate(rows_off)
        flat = np.concatenate([f for f, _ in rows_ids])
        dense = np.concatenate(rows_dense)
        tg = np.concatenate(rows_t)
        start = np.concatenate([[0], np.cumsum(lens)[:-1]])
        perm = np.random.default_rng(seed).permutation(len(lens))
        lens_p = lens[perm]
        off = np.concatenate([[0], np.cumsum(lens_p)]).astype(np.int32)
        rep = np.repeat(start[perm] - off[:-1], lens_p)
        ids_p = flat[np.arange(int(off[-1])) + rep] if off[-1] else np.zeros(0, np.int32)
        return Dataset(off, ids_p, dense[perm], tg[perm], device=device)


class Screener:
    """Surrogate + top-k + gather + exact evaluation around one Session."""

    def __init__(self, session: tto.Session, d_bits: int, d_dense: int, width: int = 512,
                 max_screen: int = 65536, max_keep: int = 8192, max_train_batch: int = 4096,
                 moved_cap: Optional[int] = None, seed: int = 0):
        import torch
        self.torch = torch
        self.sess = session
        self.dev = session.device
        self.net = tto.Surrogate(d_bits, d_dense, width=width, max_batch=max_screen,
                                 max_train_batch=max_train_batch, device=self.dev)
        self.net.set_params(tto.he_init(d_bits, d_dense, width, seed=seed))
        self.max_keep = int(max_keep)
        self.moved_cap = int(moved_cap if moved_cap is not None else max_keep * 8 * 16)
        self.y = torch.empty((max_screen, 2), dtype=torch.float32, device=self.dev)
        self.idx = torch.empty(self.max_keep, dtype=torch.int32, device=self.dev)
        self.g_open = torch.empty((self.max_keep, 8), dtype=torch.int32, device=self.dev)
        self.g_split = torch.empty((self.max_keep, 8), dtype=torch.int32, device=self.dev)
        self.g_moff = torch.empty(self.max_keep * 8 + 1, dtype=torch.int32, device=self.dev)
        self.g_mbr = torch.empty(max(self.moved_cap, 1), dtype=torch.int32, device=self.dev)
        self.g_mp = None

    # ---- training
    def train(self, data: Dataset, epochs: int = 4, batch: int = 4096, lr: float = 1e-3,
              log_every: int = 0):
        """Adam over contiguous slices of the (pre-shuffled) data set.
        Returns the list of per-epoch mean losses (read back once per epoch)."""
        torch = self.torch
        n = data.n
        losses = []
        for ep in range(epochs):
            acc = torch.zeros(1, dtype=torch.float32, device=self.dev)
            steps = 0
            for s0 in range(0, n - batch + 1 if n >= batch else 1, batch):
                nb = min(batch, n - s0)
                self.net.train_step(data.off[s0:], data.ids, data.dense[s0:], data.target[s0:],
                                    nb, lr)
                acc += self.net.loss
                steps += 1
            losses.append(float(acc.item()) / max(steps, 1))
            if log_every and (ep + 1) % log_every == 0:
                print(f"epoch {ep + 1}: loss {losses[-1]:.5f}", flush=True)
        return losses

    # ---- one generation
    def dense_rows(self, scale: FeatureScale, P, n):
        """The scenario's standardised summary repeated for n candidates."""
        row = self.torch.as_tensor(scale.apply(injection_summary(P)), device=self.dev)
        return row[None, :].expand(n, row.shape[0]).contiguous()

    def predict(self, off_d, ids_d, dense_d, n):
        return self.net.forward(off_d, ids_d, dense_d, n, y=self.y)

    def select(self, n, k):
        """Indices (device int32 [k]) of the k lowest predicted overloads."""
        if k > self.max_keep:
            raise ValueError(f"k={k} exceeds max_keep={self.max_keep}")
        y1 = int(self.y.data_ptr()) + 4   # column 1, stride 2 floats
        tto.tto_topk_smallest(y1, n, 2, k, int(self.idx.data_ptr()), self.sess.stream)
        return self.idx[:k]

    def gather(self, dbatch: tto.DeviceBatch, k) -> tto.DeviceBatch:
        torch = self.torch
        no, ns = dbatch.n_open_slots, dbatch.n_split_slots
        if no > 8 or ns > 8:
            raise ValueError("at most 8 open and 8 split slots")
        if dbatch.moved_p is not None and (self.g_mp is None or self.g_mp.shape[1] != self.sess.T):
            self.g_mp = torch.empty((self.max_keep * 8, self.sess.T), dtype=torch.float64,
                                    device=self.dev)
        go = self.g_open.view(-1)[:k * no].view(k, no)
        gs = self.g_split.view(-1)[:k * ns].view(k, ns)
        tto.tto_batch_gather(dbatch.struct(), int(self.idx.data_ptr()), k, self.sess.T,
                             tto._ptr(go) if no else 0, tto._ptr(gs) if ns else 0,
                             tto._ptr(self.g_moff), tto._ptr(self.g_mbr), self.moved_cap,
                             tto._ptr(self.g_mp) if dbatch.moved_p is not None else 0,
                             self.sess.stream)
        return tto.DeviceBatch(k, go, gs, self.g_moff, self.g_mbr,
                               self.g_mp if dbatch.moved_p is not None else None)

    def screen_and_evaluate(self, dbatch, off_d, ids_d, dense_d, k, outputs=None):
        """Forward, top-k, gather and exact evaluation of the k survivors."""
        n = dbatch.n_cand
        self.predict(off_d, ids_d, dense_d, n)
        self.select(n, k)
        gb = self.gather(dbatch, k)
        return gb, self.sess.evaluate(gb, outputs)
