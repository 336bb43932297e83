"""Efficiency studies of the paper (section "Preliminary Results") on its toy
detector, run through the gfx950 path: the fraction of simulated displaced
jets found as vertex objects,

  fig8  one jet per event, varying tracks per jet (10 hits per track);
  fig9  varying jets per event, 10 tracks each, half-angles U[15, 60] deg;
  fig10 3000 tracks of 10 hits per event, of which 10 per jet belong to a
        varying number of jets (vertices inside the 3.0 cm pipe filtered).

The paper shows these as curves without numbers; only their shapes can be
compared.  A jet counts as found when a vertex object lies within 2 rho and
2 theta bins of it and at least half of the object's members are tracks of
that jet (metrics.vertex_metrics); the paper's efficiency divides by all
simulated jets.

    python -m paper_1309_6275_amd.studies [--events N] [--figs 8,9,10]
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

SCANS = {
    8: ("tracks per jet", [2, 3, 4, 5, 6, 8, 10, 15, 20],
        lambda x: dict(n_prompt=0, n_jets=1, jet_ntrk=x)),
    9: ("jets per event", [1, 2, 3, 4, 5, 6],
        lambda x: dict(n_prompt=0, n_jets=x, jet_ntrk=10)),
    10: ("jets per event among 3000 tracks", [1, 2, 3, 4, 5],
         lambda x: dict(n_prompt=3000 - 10 * x, n_jets=x, jet_ntrk=10)),
}


def run_event(H, torch, plan, W, cl, ev, bufs, acc, peaks, nf):
    d = dict(r=torch.from_numpy(ev.r).cuda(), phi=torch.from_numpy(ev.phi).cuda(),
             layer=torch.from_numpy(ev.layer).cuda())
    H.hough_vote(plan, d["r"], d["phi"], acc)
    H.hough_peaks(plan, acc, W["min_votes"], peaks, nf)
    H.assoc_cluster(plan, d["r"], d["phi"], d["layer"], peaks, nf, cl, bufs,
                    with_vacc=False)
    return bufs.to_host(ev.n_hits)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--events", type=int, default=40, help="events per scan point")
    ap.add_argument("--figs", default="8,9,10")
    args = ap.parse_args(argv)
    import torch
    from . import houghtrig as H
    W = CF.PAPER_WORKLOAD
    g, cl = W["grid"], W["cluster"]
    # 3000 tracks put several hundred hits in a cell's member window
    dense = dict(cl, member_cap=1024)
    plan = H.Plan(g, max_hits=65535, max_peaks=1 << 21, max_member_cap=dense["member_cap"],
                  max_tracks=1 << 13)
    acc = torch.empty(plan.acc_shape, dtype=torch.int32, device="cuda")
    peaks = torch.empty((1 << 21, 2), dtype=torch.int32, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    bufs = H.ClusterBuffers(65535, 1 << 13, 256, 1 << 14, cl["n_rho"], cl["n_theta"])
    rho_bin = (cl["rho_hi"] - cl["rho_lo"]) / cl["n_rho"]
    theta_bin = 2 * np.pi / cl["n_theta"]
    out = []
    for fig in [int(f) for f in args.figs.split(",")]:
        label, xs, kw = SCANS[fig]
        n_ev = args.events if fig != 10 else max(1, args.events // 2)
        for x in xs:
            found = findable = total = 0
            t0 = time.perf_counter()
            for e in range(n_ev):
                ev = G.make_paper_event(W["seed0"] + 100_000 * fig + 1000 * x + e, **kw(x))
                res = run_event(H, torch, plan, W, dense if fig == 10 else cl, ev, bufs, acc,
                                peaks, nf)
                tm = M.match_tracks(res["tracks"]["hits"], ev.hit_track, cl["min_layers"])
                vm = M.vertex_metrics(ev, res["objects"], res["members"], tm, rho_bin, theta_bin,
                                      min_tracks=2)
                found += vm["n_found"]
                findable += vm["n_findable"]
                total += vm["n_vertices"]
            row = dict(fig=fig, scan=label, x=x, events=n_ev, jets=total, found=found,
                       efficiency=found / max(total, 1),
                       efficiency_findable=found / max(findable, 1),
                       seconds=time.perf_counter() - t0)
            out.append(row)
            print(json.dumps(row), flush=True)
    return out


if __name__ == "__main__":
    main(sys.argv[1:])
