"""Throughput of the Hough trigger path on one MI355X.

A step is one pass of the whole path -- hough_vote, hough_peaks and
assoc_cluster (refinement, ownership, refit, vertex transform) -- over a batch
of synthetic events on the 512 phi0 x 256 q/pT x 64 d0 accumulator, inputs
resident in HBM before the timed region.  By default the batch is 4
high-pileup events (~55k hits each, the largest single-GPU workload); the
displaced-jet workload (~3.6k hits, 16 events per step) is measured after it
and reported under its own key.  Prints one JSON line: whole-job Hough
votes/s (value), events/s, p50/p99 event latency, track efficiency and fake
rate of the outputs, the roofline of the dominant kernel and of the vote
kernel (the operations each kernel actually executed, against the published
MI355X vector peak of its precision; the library's HIP-event stage timers on
the launch stream give the kernel times), and the CPU oracle timed on a
bounded sample on the host cores.

    python bench.py [--steps K] [--warmup W] [--batch B] [--workload 1|2|3]
                    [--second-workload 0|1|2|3]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Hough votes/s + events/s at >=95% track eff; p50/p99 event latency (ms)"
# fp32 operations of the canonical vote formula per (hit, column) evaluation:
# u = ((KAP*r2 + Q)*ir)*T (4), |u| <= 1 (1); then for a vote: 1 - |u|, sqrt,
# 7 multiplies + 7 adds of the polynomial, s*p, pi/2 - sp (18), phi - asin,
# - PHI_LO, * INVW, floor (4)
OPS_PER_EVAL = 5
OPS_PER_VOTE = 22
# float64 operations of one road test of the seed search, the distance of a
# member from a seed circle: f = A q + B x + C y + D (3 multiplies, 3 adds),
# s = 1 + 4 A f (2, 1), sqrt, 1 + sqrt, 2 f, the division
OPS_PER_TEST = 13
# MI355X published vector peaks (a fused multiply-add counts two flops):
# fp32 157.3 TFLOP/s, fp64 78.6 TFLOP/s
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
# single-issue rate of plain (not fused, not packed) vector operations:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, reported beside the published peaks
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# events per step and CPU-oracle events per workload
DEFAULT_BATCH = {1: 64, 2: 16, 3: 4}
DEFAULT_CPU_EVENTS = {1: 64, 2: 16, 3: 2}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=0,
                    help="events per step (0: 4 for workload 3, 16 for 2, 64 for 1)")
    ap.add_argument("--workload", type=int, default=3,
                    help="1: 2D prompt event; 2: displaced-jet event (~3.6k hits); "
                         "3: high-pileup event (~55k hits), the largest single-GPU workload")
    ap.add_argument("--second-workload", type=int, default=2,
                    help="also measure this workload and report it under workload_<n> "
                         "(0 skips it)")
    ap.add_argument("--streams", type=int, default=1,
                    help="HIP streams, each with its own plan and scratch; events are "
                         "assigned round-robin and run concurrently.  The per-launch kernel "
                         "times of the roofline are meaningful with one stream only")
    ap.add_argument("--concurrent", type=int, default=2,
                    help="after the timed region, also time the same steps on this many "
                         "concurrent streams (0 skips it); reported as concurrent_streams")
    ap.add_argument("--cpu-sample", type=int, default=-1,
                    help="events of the CPU oracle baseline (0 skips it; -1: 2 events of "
                         "workload 3, 16 of workload 2)")
    ap.add_argument("--serving-probe", type=int, default=1,
                    help="1: also replay the mixed trigger stream at 1 kHz through the plain "
                         "server and report arrival-to-result latency as serving_1kHz")
    ap.add_argument("--serve", action="store_true",
                    help="benchmark the trigger serving loop instead: Poisson arrivals of a mixed "
                         "2D/3D event stream, p50/p99 latency, shedding, closed-loop throughput")
    ap.add_argument("--work-budget", type=float, default=None,
                    help="--serve: hit-columns in flight at most, as a fraction of the "
                         "largest event (max_hits x the most q/pT x d0 columns); 0: no limit")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="seconds of arrivals per Poisson rate in --serve")
    ap.add_argument("--serve-batch-hits", type=int, default=SERVE_BATCH_HITS,
                    help="--serve: events of at most this many hits may share a batch in the "
                         "learned + batched configuration")
    ap.add_argument("--two-pass", action="store_true",
                    help="benchmark iterative hit removal instead: prompt pass on the 2D grid, "
                         "removal of its hits, displaced pass on the 3D grid, against the "
                         "single pass on the same events")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (read + write) 5 times, the "
                         "reference for scaling HBM byte counters")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = 64 << 20  # 64 Mi float32 = 256 MiB
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))


# the sources a kernel's code comes from (plan and launch code excluded)
KERNEL_SOURCES = {"vote": ("vote.hip", "ht_device.h"),
                  "refine": ("assoc.hip", "ht_device.h"),
                  "members": ("assoc.hip", "ht_device.h")}


def kernel_source_sha(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1309_6275_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current source of that kernel."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_cfg{workload}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"```json\n(.*?)\n```", txt, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_source_sha") != kernel_source_sha(kernel):
        return None
    return float(d["hbm_bytes_per_launch"])


def cpu_baseline(W, events, workload):
    """The oracle (plain C, OpenMP over independent loops) on the host cores.
    Workloads 1 and 2: the full path on each sample event.  Workload 3 (about
    40 s of oracle time per event on 8 cores): the vote and peaks of each
    sample event, and the refinement on every 8th peak of its list (still in
    cell order), scaled by 8 -- its time is linear in the candidates."""
    from oracle import oracle as O
    stride = 8 if workload == 3 else 1
    t_total = 0.0
    total_votes = 0
    t_wall0 = time.perf_counter()
    for ev in events:
        t0 = time.perf_counter()
        acc, nv = O.hough_vote(W["grid"], ev.r, ev.phi)
        pk, n = O.hough_peaks(W["grid"], acc, W["min_votes"])
        t1 = time.perf_counter()
        O.assoc_cluster(W["grid"], ev.r, ev.phi, ev.layer, pk[::stride].copy(), W["cluster"])
        t2 = time.perf_counter()
        t_total += (t1 - t0) + stride * (t2 - t1)
        total_votes += nv
    wall = time.perf_counter() - t_wall0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    sample = (f"{len(events)} events of the same workload, full path (vote, peaks, refinement, "
              f"vertex transform), {wall:.1f} s, {len(events) / t_total:.3f} events/s")
    if stride > 1:
        sample = (f"{len(events)} events of the same workload: vote and peaks of each, and the "
                  f"refinement and vertex transform on every {stride}th peak, its time scaled "
                  f"by {stride}; {wall:.1f} s of CPU work, {t_total:.1f} s per "
                  f"{len(events)} events extrapolated, {len(events) / t_total:.3f} events/s")
    return {"value": total_votes / t_total, "unit": "votes/s", "cores": min(cores, threads),
            "kind": "oracle", "sample": sample}


# hit-columns in flight at most in the serving loop, as a fraction of the
# largest event
SERVE_WORK_BUDGET = 0.0
SERVE_METRIC = ("trigger serving loop: highest Poisson rate with p99 latency < 10 ms "
                "(events/s); p50/p99 ms; shed at 20 kHz; closed-loop events/s")


def serve_kinds():
    from paper_1309_6275_amd import configs as CF
    return [dict(grid=CF.GRID_2D, cluster=CF.CLUSTER_2D, min_votes=CF.WORKLOADS[1]["min_votes"],
                 peak_cap=1 << 16),
            dict(grid=CF.GRID_3D, cluster=dict(CF.CLUSTER_3D, member_cap=256),
                 min_votes=CF.WORKLOADS[2]["min_votes"], peak_cap=1 << 21)]


# events of at most this many hits may share a batch in the learned + batched
# serving configuration
SERVE_BATCH_HITS = 16384
SERVE_RATES = (50, 100, 200, 300, 400, 600, 800, 1000, 1200, 1400, 1600, 2000, 2500, 3000)


def serve_filter(torch, H, n_train, n_val, keep=0.995):
    """The 3D kind's learned peak filter, trained on the device on events of
    the serving stream's 3D kind (seeds apart from the replayed pool's),
    threshold keeping the fraction keep of the validation events' truth
    positives."""
    from paper_1309_6275_amd import configs as CF
    from paper_1309_6275_amd import eventgen as G
    from paper_1309_6275_amd import peakfilter as PF
    W = CF.WORKLOADS[2]
    t0 = time.perf_counter()
    pl = PF.Pipeline(torch, H, W, peak_cap=1 << 21)
    rng = np.random.default_rng(4_200_000)
    X, Y = PF.training_set(pl, (G.make_serving_event(1, 4_200_001 + 2 * e) for e in range(n_train)),
                           W["cluster"], rng, 3000)
    params, losses, _ = PF.train(pl, X, Y, rng)
    thr = PF.threshold(pl, params, (G.make_serving_event(1, 4_300_001 + 2 * e)
                                    for e in range(n_val)), W["cluster"], keep)
    out = params.cpu().numpy()
    info = dict(train_events=n_train, val_events=n_val, train_windows=int(Y.size),
                train_positives=int(Y.sum()), epoch_loss=losses, threshold=thr, keep_target=keep,
                seconds=time.perf_counter() - t0)
    del pl, X, params
    torch.cuda.empty_cache()
    return out, thr, info


def serve_replay(srv, rate, seconds, events, tags, min_events=1):
    """Real-time replay of Poisson arrivals (seeded by the rate, so every
    server configuration sees the same sequence at a given rate) through a
    server; latency = result seen by poll - arrival (host clock)."""
    arng = np.random.default_rng(4_100_000 + int(rate))
    n = max(min_events, int(rate * seconds))
    arrivals = np.cumsum(arng.exponential(1.0 / rate, n))
    picks = arng.integers(0, len(events), n)
    lat, shed, batched = [], 0, 0

    def take(done):
        nonlocal batched
        for d in done:
            lat.append(d["t_done"] - d["t_submit"])
            batched += d["batch"] > 1
    t0 = time.perf_counter()
    for a, p in zip(arrivals, picks):
        while time.perf_counter() - t0 < a:
            take(srv.poll(wait=False))
        k, ev = events[p]
        if not srv.submit(k, ev.r, ev.phi, ev.layer, next(tags), want_outputs=False):
            shed += 1
    take(srv.drain())
    wall = time.perf_counter() - t0
    lat = np.array(lat) * 1e3
    return dict(rate=rate, offered=n, done=int(lat.size), shed=shed, wall_s=wall,
                batched_fraction=batched / max(1, lat.size),
                p50_ms=float(np.percentile(lat, 50)) if lat.size else None,
                p99_ms=float(np.percentile(lat, 99)) if lat.size else None)


def serve_closed_loop(srv, events, n, tags):
    """n events back to back, the queue kept full; events/s."""
    t0 = time.perf_counter()
    sent = done = 0
    while done < n:
        while sent < n:
            k, ev = events[sent % len(events)]
            if not srv.submit(k, ev.r, ev.phi, ev.layer, next(tags), want_outputs=False):
                break
            sent += 1
        done += len(srv.poll(wait=True))
    return n / (time.perf_counter() - t0)


def serving_probe():
    """Arrival-to-result latency for the default line: the plain server (4
    slots) on the mixed trigger stream at 1 kHz for 2 s, and its closed-loop
    rate (the full comparison is bench.py --serve)."""
    from paper_1309_6275_amd import eventgen as G
    from paper_1309_6275_amd import houghtrig as H
    pool = [(k, G.make_serving_event(k, 4_000_001 + 2 * i + k)) for i in range(16) for k in (0, 1)]
    tags = iter(range(1 << 62))
    srv = H.Server(serve_kinds(), max_hits=65535, track_cap=4096, object_cap=256,
                   member_cap=4096, hbm_budget=96 << 30, max_slots=4, queue_cap=64)
    serve_closed_loop(srv, pool, 2 * len(pool), tags)  # warm every slot and kind
    r = serve_replay(srv, 1000, 2.0, pool, tags)
    r["closed_loop_events_per_s"] = serve_closed_loop(srv, pool, 4 * len(pool), tags)
    srv.close()
    r["stream"] = ("50% 2D (256x256) / 50% 3D (512x256x64) events, hits ~ U[2k, 60k], "
                   "Poisson arrivals replayed in real time, plain server with 4 slots")
    return r


def serve_bench(args):
    """Real-time replay of Poisson arrivals through the server (host clock:
    latency = result seen by poll - arrival), several rates, for three
    configurations: the plain serial baseline (one slot: events one after
    another, no filter), plain (four slots), and learned + batched (four
    slots, waiting events batched four to a launch, the 3D kind's peaks
    filtered by the learned filter).  Then the 20 kHz stream with a bounded
    queue, closed-loop throughput of each configuration and of the two
    ingredients alone, and the track efficiency and fake rate of each
    configuration's results on the replayed pool."""
    import torch
    from paper_1309_6275_amd import configs as CF
    from paper_1309_6275_amd import eventgen as G
    from paper_1309_6275_amd import houghtrig as H
    from paper_1309_6275_amd import metrics as M
    torch.cuda.set_device(0)
    pool = [(k, G.make_serving_event(k, 4_000_001 + 2 * i + k)) for i in range(16) for k in (0, 1)]
    kinds = serve_kinds()
    params, thr, filt_info = serve_filter(torch, H, n_train=16, n_val=4)
    print(json.dumps({"filter": filt_info}), file=sys.stderr, flush=True)
    learned_kinds = [kinds[0], dict(kinds[1], cnn_params=params, cnn_threshold=thr)]

    largest = 65535 * max(k["grid"]["n_qpt"] * k["grid"]["n_d0"] for k in kinds)
    frac = SERVE_WORK_BUDGET if args.work_budget is None else args.work_budget
    work_budget = int(frac * largest)

    def make(kinds=kinds, use_graphs=True, slots=4, queue=64, budget=work_budget, batch=0):
        return H.Server(kinds, max_hits=65535, track_cap=4096, object_cap=256, member_cap=4096,
                        hbm_budget=128 << 30, max_slots=slots, queue_cap=queue,
                        use_graphs=use_graphs, work_budget=budget, batch_max=batch,
                        batch_max_hits=args.serve_batch_hits if batch > 1 else 0)

    tags = iter(range(1 << 62))

    def replay(srv, rate, seconds, events, min_events=1):
        return serve_replay(srv, rate, seconds, events, tags, min_events)

    def closed_loop(srv, events, n):
        return serve_closed_loop(srv, events, n, tags)

    def sweep(srv, name):
        """Poisson rates in increasing order until the p99 passes 50 ms; the
        highest rate with nothing shed and a p99 under 10 ms."""
        out = []
        for rate in SERVE_RATES:
            r = replay(srv, rate, args.serve_seconds, pool, min_events=400)
            out.append(r)
            print(json.dumps(dict(r, config=name)), file=sys.stderr, flush=True)
            if r["p99_ms"] is not None and r["p99_ms"] > 50:
                break
        ok = [r["rate"] for r in out
              if r["shed"] == 0 and r["p99_ms"] is not None and r["p99_ms"] < 10]
        return out, (max(ok) if ok else None)

    def physics(srv):
        """Track efficiency and fake rate over the pool's events (truth
        matching of the served tracks), per kind and overall, and the peaks
        handed to assoc_cluster as a fraction of the threshold peaks."""
        for i, (k, ev) in enumerate(pool):
            assert srv.submit(k, ev.r, ev.phi, ev.layer, (1 << 61) + i)
        got = {d["tag"] - (1 << 61): d for d in srv.drain()}
        tot = {0: np.zeros(4), 1: np.zeros(4)}
        peaks = np.zeros(2)
        for i, (k, ev) in enumerate(pool):
            d = got[i]
            K = kinds[k]
            tm = M.track_metrics(ev, K["grid"], K["cluster"]["min_layers"], d["tracks"]["hits"])
            tot[k] += [tm["n_found"], tm["n_truth_acc"], tm["n_fake"], tm["n_tracks"]]
            if k == 1:
                peaks += [d["n_kept"], d["n_peaks"]]
        out = {}
        for k, name in ((0, "2d"), (1, "3d")):
            f, a, fk, nt = tot[k]
            out[name] = dict(track_efficiency=f / max(a, 1), fake_rate=fk / max(nt, 1))
        f, a, fk, nt = tot[0] + tot[1]
        out.update(track_efficiency=f / max(a, 1), fake_rate=fk / max(nt, 1),
                   kept_fraction_3d=peaks[0] / max(peaks[1], 1))
        return out

    def run_config(name, srv, do_sweep=True):
        closed_loop(srv, pool, 2 * len(pool))  # warm every slot, kind and batch size
        res = dict(slots=srv.n_slots, slot_bytes=srv.slot_bytes)
        if do_sweep:
            res["rates"], res["value"] = sweep(srv, name)
            best = next((r for r in res["rates"] if r["rate"] == res["value"]), None)
            res["p50_ms"] = best["p50_ms"] if best else None
            res["p99_ms"] = best["p99_ms"] if best else None
            res["at_20kHz"] = replay(srv, 20000, 1.0, pool)
        res["closed_loop_events_per_s"] = closed_loop(srv, pool, 4 * len(pool))
        res["physics"] = physics(srv)
        srv.close()
        print(json.dumps({name: {k: v for k, v in res.items() if k != "rates"}}), file=sys.stderr,
              flush=True)
        return res

    learned = run_config("learned_batched", make(learned_kinds, batch=4))
    plain = run_config("plain", make())
    serial = run_config("plain_serial", make(slots=1))
    batched_only = run_config("batched_no_filter", make(batch=4), do_sweep=False)
    filter_only = run_config("filter_no_batching", make(learned_kinds), do_sweep=False)
    direct = make(learned_kinds, use_graphs=False, batch=4)
    closed_loop(direct, pool, len(pool))
    tput_direct = closed_loop(direct, pool, 4 * len(pool))
    direct.close()
    two_d = [e for e in pool if e[0] == 0]
    srv2 = make(learned_kinds, batch=4)
    closed_loop(srv2, two_d, len(two_d))
    tput_2d = closed_loop(srv2, two_d, 8 * len(two_d))
    srv2.close()
    line = {
        "metric": SERVE_METRIC, "value": learned["value"], "unit": "events/s", "n_gpus": 1,
        "higher_is_better": True, "data": "synthetic", "dtype": "f32+f64+bf16",
        "config": {"workload": "mixed trigger stream: 50% 2D (256x256) / 50% 3D (512x256x64) "
                               "events, hits ~ U[2k, 60k], pool of 32 seeded events",
                   "form": "learned + batched: 4 slots, up to 4 waiting events of a kind with "
                           f"<= {args.serve_batch_hits} hits per launch, learned peak filter on the "
                           "3D kind (keeps 99.5% of validation truth positives)",
                   "slots": learned["slots"], "slot_bytes": learned["slot_bytes"],
                   "queue_cap": 64, "graphs": True, "work_budget": work_budget,
                   "work_budget_fraction_of_largest_event": frac},
        "p50_ms": learned["p50_ms"], "p99_ms": learned["p99_ms"],
        "track_efficiency": learned["physics"]["track_efficiency"],
        "fake_rate": learned["physics"]["fake_rate"],
        "physics": learned["physics"],
        "rates": learned["rates"],
        "at_20kHz": learned["at_20kHz"],
        "closed_loop_events_per_s": learned["closed_loop_events_per_s"],
        "closed_loop_events_per_s_direct_launches": tput_direct,
        "closed_loop_2d_only_events_per_s": tput_2d,
        "filter": filt_info,
        "plain_serial": serial,
        "plain": plain,
        "batched_no_filter": batched_only,
        "filter_no_batching": filter_only,
        "vs_plain_serial": (learned["value"] / serial["value"]
                            if learned["value"] and serial["value"] else None),
        "vs_plain": (learned["value"] / plain["value"]
                     if learned["value"] and plain["value"] else None),
    }
    print(json.dumps(line), flush=True)


def two_pass_bench(args):
    """Events/s and physics of iterative hit removal on the displaced-jet
    workload, beside the single pass over the same events."""
    import torch
    from paper_1309_6275_amd import configs as CF
    from paper_1309_6275_amd import eventgen as G
    from paper_1309_6275_amd import houghtrig as H
    from paper_1309_6275_amd import iterative
    from paper_1309_6275_amd import metrics as M

    W = CF.WORKLOADS[2]
    D = CF.TWO_PASS["displaced"]
    B = args.batch or 16
    events = [G.make_event(2, W["seed0"] + 100 + e) for e in range(B)]
    dev = [dict(r=torch.from_numpy(ev.r).cuda(), phi=torch.from_numpy(ev.phi).cuda(),
                layer=torch.from_numpy(ev.layer).cuda()) for ev in events]
    tp = iterative.TwoPass(max_hits=65535, track_cap=1 << 13)
    plan = H.Plan(W["grid"], max_hits=65535, max_peaks=1 << 19,
                  max_member_cap=W["cluster"]["member_cap"], max_tracks=1 << 13)
    acc = torch.empty(plan.acc_shape, dtype=torch.int32, device="cuda")
    peaks = torch.empty((1 << 19, 2), dtype=torch.int32, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    bufs = H.ClusterBuffers(65535, 1 << 13, 1024, 1 << 15, W["cluster"]["n_rho"],
                            W["cluster"]["n_theta"])
    cl = W["cluster"]
    rho_bin = (cl["rho_hi"] - cl["rho_lo"]) / cl["n_rho"]
    theta_bin = 2 * np.pi / cl["n_theta"]

    def single(d):
        H.hough_vote(plan, d["r"], d["phi"], acc)
        H.hough_peaks(plan, acc, W["min_votes"], peaks, nf)
        H.assoc_cluster(plan, d["r"], d["phi"], d["layer"], peaks, nf, cl, bufs)

    def timed(fn):
        for _ in range(args.warmup):
            for d in dev:
                fn(d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for d in dev:
                fn(d)
        torch.cuda.synchronize()
        return args.steps * B / (time.perf_counter() - t0)

    rate_two = timed(lambda d: tp.run(d["r"], d["phi"], d["layer"]))
    rate_one = timed(single)

    def physics(run_one):
        found = truth = fake = ntrk = vfound = vfind = nv = kept = 0
        for ev, d in zip(events, dev):
            hits, objects, members, k = run_one(ev, d)
            kept += k
            hit_rows = np.concatenate(hits) if len(hits) > 1 else hits[0]
            tm = M.track_metrics(ev, W["grid"], cl["min_layers"], hit_rows)
            found += tm["n_found"]
            truth += tm["n_truth_acc"]
            fake += tm["n_fake"]
            ntrk += tm["n_tracks"]
            match = M.match_tracks(hits[-1], ev.hit_track, cl["min_layers"])
            vm = M.vertex_metrics(ev, objects, members, match, rho_bin, theta_bin, min_tracks=2)
            vfound += vm["n_found"]
            vfind += vm["n_findable"]
            nv += vm["n_vertices"]
        return dict(track_efficiency=found / max(truth, 1), fake_rate=fake / max(ntrk, 1),
                    tracks_per_event=ntrk / B, vertices_found=vfound, vertices_findable=vfind,
                    vertices=nv, hits_in_displaced_pass=kept / B)

    def run_two(ev, d):
        tp.run(d["r"], d["phi"], d["layer"])
        first, keep, second = tp.to_host(ev.n_hits)
        return ([first["tracks"]["hits"], second["tracks"]["hits"]], second["objects"],
                second["members"], keep.size)

    def run_single(ev, d):
        single(d)
        torch.cuda.synchronize()
        out = bufs.to_host(ev.n_hits)
        return [out["tracks"]["hits"]], out["objects"], out["members"], ev.n_hits

    line = {
        "metric": "events_per_s",
        "value": rate_two,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "higher_is_better": True,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": W["name"] + ", iterative hit removal",
                   "passes": CF.TWO_PASS["name"], "events_per_step": B,
                   "parallelism": "single GPU, events back to back on one stream"},
        "two_pass": physics(run_two),
        "single_pass_events_per_s": rate_one,
        "single_pass": physics(run_single),
        "note": "both passes asynchronous on one stream; the displaced pass reads the kept-hit "
                "count on the device",
    }
    tp.close()
    print(json.dumps(line), flush=True)


def measure(args, workload, B, steps, warmup, cpu_events, concurrent):
    """Times `steps` steps of the whole path over B events of one workload
    (inputs resident in HBM) and returns the figures of one bench line."""
    import torch
    from paper_1309_6275_amd import configs as CF
    from paper_1309_6275_amd import eventgen as G
    from paper_1309_6275_amd import houghtrig as H
    from paper_1309_6275_amd import metrics as M

    W = CF.WORKLOADS[workload]
    g, cl = W["grid"], W["cluster"]
    events = [G.make_event(workload, W["seed0"] + 100 + e) for e in range(B)]
    peak_cap = 1 << 19 if workload < 3 else 1 << 21
    S = max(1, args.streams)
    plans = [H.Plan(g, max_hits=65535, max_peaks=peak_cap, max_member_cap=cl["member_cap"],
                    max_tracks=1 << 14) for _ in range(S)]
    plan = plans[0]
    dev = []
    for ev in events:
        dev.append(dict(r=torch.from_numpy(ev.r).cuda(), phi=torch.from_numpy(ev.phi).cuda(),
                        layer=torch.from_numpy(ev.layer).cuda(), n=ev.n_hits))
    ctx = [dict(acc=torch.empty(plan.acc_shape, dtype=torch.int32, device="cuda"),
                peaks=torch.empty((peak_cap, 2), dtype=torch.int32, device="cuda"),
                nf=torch.zeros(1, dtype=torch.int32, device="cuda")) for _ in range(S)]
    acc = ctx[0]["acc"]
    nv = torch.zeros(1, dtype=torch.int64, device="cuda")
    bufs = [H.ClusterBuffers(ev.n_hits, 1 << 14, 1024, 1 << 16, cl["n_rho"], cl["n_theta"])
            for ev in events]

    # per-event vote counts, evaluations and distinct hit radii (deterministic),
    # outside timing
    votes, evals, radii = [], [], []
    ncol = g["n_qpt"] * g["n_d0"]
    for d, ev in zip(dev, events):
        H.hough_vote(plan, d["r"], d["phi"], acc, nv)
        torch.cuda.synchronize()
        votes.append(int(nv.item()))
        ok = (ev.r > 0) & (ev.r < 1e4) & (np.abs(ev.phi) <= 4)
        evals.append(int(ok.sum()) * ncol)
        radii.append(int(np.unique(ev.r[ok]).size))

    # default-priority streams, one plan (tables and scratch) per stream
    streams = [torch.cuda.Stream() for _ in range(S)]
    torch.cuda.synchronize()
    ev_a = [torch.cuda.Event(enable_timing=True) for _ in range(B)]
    ev_c = [torch.cuda.Event(enable_timing=True) for _ in range(B)]

    def step(record):
        for e, d in enumerate(dev):
            c, st, pl = ctx[e % S], streams[e % S], plans[e % S]
            with torch.cuda.stream(st):
                if record:
                    ev_a[e].record(st)
                H.hough_vote(pl, d["r"], d["phi"], c["acc"])
                H.hough_peaks(pl, c["acc"], W["min_votes"], c["peaks"], c["nf"])
                H.assoc_cluster(pl, d["r"], d["phi"], d["layer"], c["peaks"], c["nf"], cl,
                                bufs[e], with_vacc=False)
                if record:
                    ev_c[e].record(st)

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    # stage timers: HIP events the library records around its kernels on each
    # plan's launch stream, read after each step
    for pl in plans:
        H.profile_begin(pl, depth=2 * B)
    stages = {}
    lat_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
        torch.cuda.synchronize()  # per-step sync so the events of this step can be read
        for e in range(B):
            lat_ms.append(ev_a[e].elapsed_time(ev_c[e]))
        for pl in plans:
            H.profile_read(pl, stages)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for pl in plans:
        H.profile_end(pl)

    # the same steps on concurrent streams, each with its own plan: throughput
    # when kernels of several events overlap (not the headline value, whose
    # per-launch kernel times the roofline needs)
    conc = None
    if concurrent > 1 and S == 1:
        C = concurrent
        cplans = [plan] + [H.Plan(g, max_hits=65535, max_peaks=peak_cap,
                                  max_member_cap=cl["member_cap"], max_tracks=1 << 14)
                           for _ in range(C - 1)]
        cctx = [ctx[0]] + [dict(acc=torch.empty(plan.acc_shape, dtype=torch.int32, device="cuda"),
                                peaks=torch.empty((peak_cap, 2), dtype=torch.int32, device="cuda"),
                                nf=torch.zeros(1, dtype=torch.int32, device="cuda"))
                           for _ in range(C - 1)]
        cstreams = [torch.cuda.Stream() for _ in range(C)]

        def cstep():
            for e, d in enumerate(dev):
                c, st, pl = cctx[e % C], cstreams[e % C], cplans[e % C]
                with torch.cuda.stream(st):
                    H.hough_vote(pl, d["r"], d["phi"], c["acc"])
                    H.hough_peaks(pl, c["acc"], W["min_votes"], c["peaks"], c["nf"])
                    H.assoc_cluster(pl, d["r"], d["phi"], d["layer"], c["peaks"], c["nf"], cl,
                                    bufs[e], with_vacc=False)

        for _ in range(warmup):
            cstep()
        torch.cuda.synchronize()
        tc = time.perf_counter()
        for _ in range(steps):
            cstep()
        torch.cuda.synchronize()
        cw = time.perf_counter() - tc
        conc = {"streams": C, "events_per_s": steps * B / cw,
                "votes_per_s": steps * sum(votes) / cw,
                "note": "same steps after the timed region, events round-robin over streams "
                        "with one plan each"}
        for pl in cplans[1:]:
            pl.close()

    n_events = steps * B
    total_votes = steps * sum(votes)
    lat_ms = np.array(lat_ms)
    avg_ms = {k: (v[0] / v[1] if v[1] else float("nan")) for k, v in stages.items()}

    # physics of the outputs (last step) and the seed search's work totals,
    # outside the timed region
    effs, fakes, n_trk, defined, executed, cnts = [], [], 0, [], [], []
    for ev, b in zip(events, bufs):
        out = b.to_host(ev.n_hits)
        cnts.append(out["counts"].astype(np.int64))
        tm = M.track_metrics(ev, g, cl["min_layers"], out["tracks"]["hits"])
        effs.append((tm["n_found"], tm["n_truth_acc"]))
        fakes.append((tm["n_fake"], tm["n_tracks"]))
        n_trk += tm["n_tracks"]
        defined.append(int(out["work"][0]))
        executed.append(int(out["work"][1]))
    eff = sum(a for a, _ in effs) / max(1, sum(b for _, b in effs))
    fake = sum(a for a, _ in fakes) / max(1, sum(b for _, b in fakes))

    # Work actually executed per launch.
    #  vote: the per-radius table path (every hit here lies on one of at most
    #  16 distinct radii of its workgroup) computes u, the |u| test and the
    #  arcsine once per (radius, column), 27 fp32 operations, and per vote
    #  x = ((phi - s) - PHI_LO) * INVW and the floor, 4 operations.
    #  refine: 13 fp64 operations per float64 circle distance the kernel
    #  computed (work[1]); the float32 pre-filter is not counted.
    table_path = all(n <= 16 for n in radii)
    vote_exec = np.mean([(OPS_PER_EVAL + OPS_PER_VOTE) * n * ncol + 4 * V if table_path
                         else OPS_PER_EVAL * E + OPS_PER_VOTE * V
                         for n, E, V in zip(radii, evals, votes)])
    vote_method = np.mean([OPS_PER_EVAL * E + OPS_PER_VOTE * V for E, V in zip(evals, votes)])
    refine_exec = OPS_PER_TEST * float(np.mean(executed))
    refine_method = OPS_PER_TEST * float(np.mean(defined))

    def roofline(kernel, executed_ops, method_ops, peak, dtype):
        t = avg_ms[kernel] / 1e3
        achieved = executed_ops / t / 1e12
        return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic_from_profile(kernel, workload),
                "kernel": f"{kernel}_kernel", "avg_launch_ms": avg_ms[kernel], "dtype": dtype,
                "executed_ops_per_launch": executed_ops,
                "method_ops_per_launch": method_ops,
                "method_ops_frac": method_ops / t / 1e12 / peak,
                "single_issue_peak": ALU_PEAK_TOPS,
                "frac_single_issue": achieved / ALU_PEAK_TOPS}

    rl = {"vote": roofline("vote", vote_exec, vote_method, FP32_PEAK_TFLOPS, "f32"),
          "refine": roofline("refine", refine_exec, refine_method, FP64_PEAK_TFLOPS, "f64")}
    # the dominant kernel by measured time among the timed kernels with an
    # operation count (the member sweep has none of its own)
    dominant = max(("vote", "refine"), key=lambda k: avg_ms.get(k, 0.0))

    cpu = None
    if cpu_events > 0:
        cpu = cpu_baseline(W, events[:cpu_events], workload)

    res = {
        "workload": W["name"],
        "events_per_step": B,
        "mean_hits": float(np.mean([ev.n_hits for ev in events])),
        "votes_per_s": total_votes / wall,
        "events_per_s": n_events / wall,
        "ms_per_step": wall * 1e3 / steps,
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "track_efficiency": eff,
        "fake_rate": fake,
        "tracks_per_event": n_trk / B,
        # per event: peaks handed to assoc_cluster, refined candidates,
        # candidates over member_cap, (candidate, member) pairs within it
        "assoc_counts": {"refined": float(np.mean([c[0] for c in cnts])),
                         "over_member_cap": float(np.mean([c[4] for c in cnts])),
                         "member_pairs": float(np.mean([c[5] for c in cnts])),
                         "objects": float(np.mean([c[2] for c in cnts])),
                         "object_members": float(np.mean([c[3] for c in cnts]))},
        "vote_kernel_votes_per_s": float(np.mean(votes)) / (avg_ms["vote"] / 1e3),
        "stage_ms": {k: avg_ms[k] for k in ("vote", "peaks", "members", "refine", "assoc")},
        "roofline": rl[dominant],
        "roofline_vote": rl["vote"],
        "roofline_refine": rl["refine"],
        "cpu_baseline": cpu,
        "concurrent_streams": conc,
        "grid": f"{g['n_phi']}x{g['n_qpt']}x{g['n_d0']}",
        "parallelism": ("single GPU, events back to back on one stream" if S == 1
                        else f"single GPU, {S} streams with one plan each, events "
                             "round-robin and concurrent"),
    }
    for pl in plans:
        pl.close()
    return res


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(events are independent: scale by running one process per GPU)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    from paper_1309_6275_amd import build as hip_build
    if not os.path.exists(hip_build.LIB):
        hip_build.build()
    if args.serve:
        serve_bench(args)
        return
    if args.two_pass:
        two_pass_bench(args)
        return
    torch.cuda.set_device(0)
    wl = args.workload
    B = args.batch if args.batch else DEFAULT_BATCH[wl]
    cpu_events = args.cpu_sample if args.cpu_sample >= 0 else DEFAULT_CPU_EVENTS[wl]
    r = measure(args, wl, B, args.steps, args.warmup, cpu_events, args.concurrent)
    line = {
        "metric": METRIC,
        "value": r["votes_per_s"],
        "unit": "votes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": r["workload"], "events_per_step": B, "grid": r["grid"],
                   "mean_hits": r["mean_hits"], "parallelism": r["parallelism"]},
    }
    for k in ("events_per_s", "p50_ms", "p99_ms", "track_efficiency", "fake_rate",
              "tracks_per_event", "assoc_counts", "vote_kernel_votes_per_s", "stage_ms", "roofline",
              "roofline_vote", "roofline_refine", "cpu_baseline", "concurrent_streams"):
        line[k] = r[k]
    # the displaced-jet workload beside it, where the method reaches its
    # efficiency; same figures, its own timed region after the first
    if args.second_workload and args.second_workload != wl:
        w2 = args.second_workload
        r2 = measure(args, w2, DEFAULT_BATCH[w2], args.steps, args.warmup, 0, 0)
        line[f"workload_{w2}"] = {k: r2[k] for k in (
            "workload", "events_per_step", "mean_hits", "votes_per_s", "events_per_s",
            "ms_per_step", "p50_ms", "p99_ms", "track_efficiency", "fake_rate",
            "tracks_per_event", "stage_ms", "roofline", "roofline_vote", "roofline_refine")}
    if args.serving_probe:
        line["serving_1kHz"] = serving_probe()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
