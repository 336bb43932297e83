"""Train and evaluate the learned peak filter on the device (ht_cnn_*).

Labels: truth matching of the peak cell against the event generator,
independent of the refinement.  A threshold peak (i, j, k) is positive when
a generated track in acceptance (q/pT and d0 inside the grid, at least
min_layers hits after its perigee) has its true parameters in a cell within
one bin of it in q/pT and in d0 and within two bins in phi0 (periodic); the
phi0 tolerance is wider because the vote samples each column at its centre,
which moves the track's votes by up to about a bin.  Every other peak is
negative.  The peaks are those of hough_vote and hough_peaks on the device,
which equal the oracle's bit for bit (the parity tests), so these are the
oracle Hough's peaks labelled by truth.  The training set keeps every
positive and a stated number of random negatives per event.  Training: SGD
with momentum on the device (ht_cnn_train_step), positives weighted by the
negative/positive ratio.  The threshold keeps a stated fraction of the
validation positives.  Evaluation on other events: track efficiency and fake
rate of assoc_cluster (the refinement and its truth matching of tracks, the
judge of the filter) on all peaks and on the kept peaks, the peaks kept, and
the time of assoc_cluster with and without the filter (scoring with
ht_cnn_score and compaction included).

Seeds: training events 5 000 000 + e, validation 5 500 000 + e, test
5 900 000 + e, all of the 3D displaced-jet composition.

    python -m paper_1309_6275_amd.peakfilter [--train-events 60] [--epochs 6]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import configs as CF
from . import eventgen as G
from . import metrics as M


class Pipeline:
    def __init__(self, torch, H, W, peak_cap=1 << 19):
        self.torch, self.H, self.W = torch, H, W
        g, cl = W["grid"], W["cluster"]
        self.plan = H.Plan(g, max_hits=65535, max_peaks=peak_cap,
                           max_member_cap=cl["member_cap"], max_tracks=1 << 13)
        self.acc = torch.empty(self.plan.acc_shape, dtype=torch.int32, device="cuda")
        self.peaks = torch.empty((peak_cap, 2), dtype=torch.int32, device="cuda")
        self.kept = torch.empty((peak_cap, 2), dtype=torch.int32, device="cuda")
        self.nf = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.nk = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.win = torch.empty((peak_cap, H.CNN_WINDOW), dtype=torch.bfloat16, device="cuda")
        self.logits = torch.empty(peak_cap, dtype=torch.float32, device="cuda")
        self.ws = H.cnn_workspace(peak_cap)
        self.bufs = H.ClusterBuffers(65535, 1 << 13, 256, 1 << 14, cl["n_rho"], cl["n_theta"])
        self.cap = peak_cap

    def upload(self, ev):
        t = self.torch
        return dict(r=t.from_numpy(ev.r).cuda(), phi=t.from_numpy(ev.phi).cuda(),
                    layer=t.from_numpy(ev.layer).cuda())

    def peaks_of(self, d):
        H = self.H
        H.hough_vote(self.plan, d["r"], d["phi"], self.acc)
        H.hough_peaks(self.plan, self.acc, self.W["min_votes"], self.peaks, self.nf)

    def assoc(self, d, peaks, n):
        self.H.assoc_cluster(self.plan, d["r"], d["phi"], d["layer"], peaks, n, self.W["cluster"],
                             self.bufs, with_vacc=False)

    def filter(self, params, thr):
        H = self.H
        H.cnn_score(self.plan, params, self.acc, self.peaks, self.nf, self.logits, self.ws)
        H.cnn_keep(self.plan, self.logits, self.peaks, self.nf, thr, self.kept, self.nk)


def truth_labels(ev, grid, min_layers, lins, dphi=2, dq=1, dd=1):
    """1 for the peak cells within (dphi, dq, dd) bins of the true cell of a
    generated track in acceptance (phi0 periodic, the others clipped to the
    grid), else 0.  The cells near the truth are listed once per track and
    offset, then looked up: linear in tracks plus peaks."""
    nphi, nq, nd = grid["n_phi"], grid["n_qpt"], grid["n_d0"]
    lins = np.asarray(lins, np.int64)
    acc = M.in_acceptance(ev, grid, min_layers)
    t = np.flatnonzero(acc)
    qw = (grid["qpt_hi"] - grid["qpt_lo"]) / nq
    it = np.floor((np.asarray(ev.trk_phi0)[t] + np.pi) * nphi / (2 * np.pi)).astype(np.int64) % nphi
    jt = np.clip(np.floor((np.asarray(ev.trk_qpt)[t] - grid["qpt_lo"]) / qw).astype(np.int64),
                 0, nq - 1)
    if nd > 1:
        dw = (grid["d0_hi"] - grid["d0_lo"]) / nd
        kt = np.clip(np.floor((np.asarray(ev.trk_d0)[t] - grid["d0_lo"]) / dw).astype(np.int64),
                     0, nd - 1)
    else:
        kt = np.zeros(t.size, np.int64)
    di, dj, dk = np.meshgrid(np.arange(-dphi, dphi + 1), np.arange(-dq, dq + 1),
                             np.arange(-dd, dd + 1), indexing="ij")
    ii = (it[:, None] + di.reshape(-1)[None, :]) % nphi
    jj = jt[:, None] + dj.reshape(-1)[None, :]
    kk = kt[:, None] + dk.reshape(-1)[None, :]
    ok = (jj >= 0) & (jj < nq) & (kk >= 0) & (kk < nd)
    near = np.unique(((kk * nq + jj) * nphi + ii)[ok])
    return np.isin(lins, near).astype(np.float32)


def training_set(pl, events, cl, rng, neg_per_event):
    """Windows (device bfloat16) and truth labels of every positive peak and
    up to neg_per_event random negative peaks of each event."""
    t, H = pl.torch, pl.H
    xs, ys = [], []
    for ev in events:
        d = pl.upload(ev)
        pl.peaks_of(d)
        H.cnn_windows(pl.plan, pl.acc, pl.peaks, pl.nf, pl.win)
        t.cuda.synchronize()
        n = min(int(pl.nf.item()), pl.cap)
        y = truth_labels(ev, pl.W["grid"], cl["min_layers"], pl.peaks[:n, 0].cpu().numpy())
        pos = np.flatnonzero(y > 0.5)
        neg = np.flatnonzero(y < 0.5)
        neg = rng.choice(neg, min(neg_per_event, neg.size), replace=False)
        sel = np.concatenate([pos, neg])
        xs.append(pl.win[t.from_numpy(sel).cuda()].clone())
        ys.append(y[sel])
    return t.cat(xs), np.concatenate(ys).astype(np.float32)


def train(pl, X, Y, rng, epochs=6, batch=4096, lr=0.05, seed=7):
    """SGD with momentum on the device, positives weighted by the
    negative/positive ratio.  Returns the device parameters and the mean
    loss of each epoch."""
    t, H = pl.torch, pl.H
    n_pos = int(Y.sum())
    pos_weight = (Y.size - n_pos) / max(n_pos, 1)
    params = t.from_numpy(init_params(seed)).cuda()
    mom = t.zeros_like(params)
    loss = t.zeros(1, dtype=t.float32, device="cuda")
    Yd = t.from_numpy(Y).cuda()
    ws = H.cnn_workspace(batch, training=True)
    losses = []
    for ep in range(epochs):
        perm = t.from_numpy(rng.permutation(Y.size)).cuda()
        ep_loss = []
        for b in range(0, Y.size - batch + 1, batch):
            idx = perm[b:b + batch]
            H.cnn_train_step(params, mom, X[idx].contiguous(), Yd[idx].contiguous(), lr, 0.9,
                             pos_weight, loss, ws)
            ep_loss.append(loss.clone())
        t.cuda.synchronize()
        losses.append(float(t.cat(ep_loss).mean().item()) if ep_loss else float("nan"))
    return params, losses, pos_weight


def threshold(pl, params, events, cl, keep):
    """The logit threshold that keeps the fraction keep of the truth-positive
    peaks of the events (scored with ht_cnn_score)."""
    t, H = pl.torch, pl.H
    pos_logits = []
    for ev in events:
        d = pl.upload(ev)
        pl.peaks_of(d)
        H.cnn_score(pl.plan, params, pl.acc, pl.peaks, pl.nf, pl.logits, pl.ws)
        t.cuda.synchronize()
        n = min(int(pl.nf.item()), pl.cap)
        y = truth_labels(ev, pl.W["grid"], cl["min_layers"], pl.peaks[:n, 0].cpu().numpy())
        pos_logits.append(pl.logits[:n].cpu().numpy()[y > 0.5])
    pos_logits = np.concatenate(pos_logits)
    return float(np.quantile(pos_logits, 1.0 - keep)) if pos_logits.size else 0.0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-events", type=int, default=60)
    ap.add_argument("--val-events", type=int, default=10)
    ap.add_argument("--test-events", type=int, default=10)
    ap.add_argument("--neg-per-event", type=int, default=3000)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=0.05)
    ap.add_argument("--keep", type=float, default=0.995,
                    help="fraction of validation positives the threshold keeps")
    args = ap.parse_args(argv)
    import torch
    from . import houghtrig as H
    W = CF.WORKLOADS[2]
    cl = W["cluster"]
    pl = Pipeline(torch, H, W)
    rng = np.random.default_rng(5_000_000)

    t0 = time.perf_counter()
    X, Y = training_set(pl, (G.make_event(2, 5_000_000 + e) for e in range(args.train_events)),
                        cl, rng, args.neg_per_event)
    n_pos = int(Y.sum())
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    params, losses, pos_weight = train(pl, X, Y, rng, args.epochs, args.batch, args.lr)
    t_train = time.perf_counter() - t0
    steps = args.epochs * (Y.size // args.batch)
    thr = threshold(pl, params, (G.make_event(2, 5_500_000 + e) for e in range(args.val_events)),
                    cl, args.keep)

    # evaluation: the same events with all peaks and with the kept peaks
    rows = []
    ev_s, ev_e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for e in range(args.test_events):
        ev = G.make_event(2, 5_900_000 + e)
        d = pl.upload(ev)
        res = {}
        for mode in ("all", "filtered"):
            pl.peaks_of(d)
            torch.cuda.synchronize()
            ev_s.record()
            if mode == "all":
                pl.assoc(d, pl.peaks, pl.nf)
            else:
                pl.filter(params, thr)
                pl.assoc(d, pl.kept, pl.nk)
            ev_e.record()
            torch.cuda.synchronize()
            out = pl.bufs.to_host(ev.n_hits)
            tm = M.track_metrics(ev, W["grid"], cl["min_layers"], out["tracks"]["hits"])
            res[mode] = dict(ms=ev_s.elapsed_time(ev_e), eff=tm["efficiency"],
                             fake=tm["fake_rate"], n_found=tm["n_found"], n_acc=tm["n_truth_acc"],
                             n_fake=tm["n_fake"], n_tracks=tm["n_tracks"])
        res["peaks"] = int(pl.nf.item())
        res["kept"] = int(pl.nk.item())
        rows.append(res)

    def agg(mode, key):
        return float(np.mean([r[mode][key] for r in rows]))

    def ratio(mode, a, b):
        return sum(r[mode][a] for r in rows) / max(1, sum(r[mode][b] for r in rows))

    line = {
        "train_windows": int(Y.size), "train_positives": n_pos, "pos_weight": pos_weight,
        "data_seconds": t_data, "train_steps": steps, "train_seconds": t_train,
        "epoch_loss": losses, "threshold": thr, "keep_target": args.keep,
        "peaks_per_event": float(np.mean([r["peaks"] for r in rows])),
        "kept_fraction": sum(r["kept"] for r in rows) / max(1, sum(r["peaks"] for r in rows)),
        "assoc_ms_all": agg("all", "ms"), "filter_plus_assoc_ms": agg("filtered", "ms"),
        "efficiency_all": ratio("all", "n_found", "n_acc"),
        "efficiency_filtered": ratio("filtered", "n_found", "n_acc"),
        "fake_rate_all": ratio("all", "n_fake", "n_tracks"),
        "fake_rate_filtered": ratio("filtered", "n_fake", "n_tracks"),
    }
    print(json.dumps(line), flush=True)
    return line, params


def init_params(seed):
    """He-style normal weights (fan-in scaled), zero biases, in the flat
    layout of the device parameters."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape, fan_in in (((16, 27), 27), ((16,), 0), ((16, 16, 27), 432), ((16,), 0),
                          ((64, 16), 16), ((64,), 0), ((64,), 64), ((1,), 0)):
        if fan_in:
            parts.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), shape).reshape(-1))
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts).astype(np.float32)


if __name__ == "__main__":
    main(sys.argv[1:])
