"""Iterative hit removal on the device (the paper's tracker practice,
section "Current Tracker and Tracking Algorithm": an earlier pass finds the
easier, prompt tracks, their hits are removed, and a later pass searches
the rest for displaced tracks among far fewer combinations).

Pass 1 runs hough_vote, hough_peaks and assoc_cluster on the prompt grid
(one d0 column, beam-line seeds); ht_compact_hits keeps the hits it left;
pass 2 runs the displaced-jet path (3D grid, vertex transform) on those;
ht_remap_track_hits makes pass-2 tracks name event hits.  The displaced
pass takes the kept-hit count from device memory (hough_vote_n,
assoc_cluster_n), so the whole chain is asynchronous on one stream.

    tp = TwoPass(max_hits=65535)
    tp.run(r, phi, layer)                      # device tensors in
    first, keep, second = tp.to_host(n_hits)   # synchronises
"""
from __future__ import annotations

from . import configs as CF
from . import houghtrig as H


class TwoPass:
    def __init__(self, max_hits=65535, spec=None, track_cap=8192, object_cap=1024,
                 member_cap=1 << 15, prompt_peaks=1 << 16, displaced_peaks=1 << 21):
        import torch
        self.torch = torch
        self.spec = spec or CF.TWO_PASS
        P, D = self.spec["prompt"], self.spec["displaced"]
        self.plan_p = H.Plan(P["grid"], max_hits=max_hits, max_peaks=prompt_peaks,
                             max_member_cap=P["cluster"]["member_cap"], max_tracks=track_cap)
        self.plan_d = H.Plan(D["grid"], max_hits=max_hits, max_peaks=displaced_peaks,
                             max_member_cap=D["cluster"]["member_cap"], max_tracks=track_cap)
        dev = "cuda"
        self.acc_p = torch.empty(self.plan_p.acc_shape, dtype=torch.int32, device=dev)
        self.acc_d = torch.empty(self.plan_d.acc_shape, dtype=torch.int32, device=dev)
        self.pk_p = torch.empty((prompt_peaks, 2), dtype=torch.int32, device=dev)
        self.pk_d = torch.empty((displaced_peaks, 2), dtype=torch.int32, device=dev)
        self.nf = torch.zeros(2, dtype=torch.int32, device=dev)
        cp, cd = P["cluster"], D["cluster"]
        self.bufs_p = H.ClusterBuffers(max_hits, track_cap, 1, 1, cp["n_rho"], cp["n_theta"])
        self.bufs_d = H.ClusterBuffers(max_hits, track_cap, object_cap, member_cap, cd["n_rho"],
                                       cd["n_theta"])
        self.r2 = torch.empty(max_hits, dtype=torch.float32, device=dev)
        self.phi2 = torch.empty(max_hits, dtype=torch.float32, device=dev)
        self.layer2 = torch.empty(max_hits, dtype=torch.uint8, device=dev)
        self.keep = torch.empty(max_hits, dtype=torch.int32, device=dev)
        self.n_keep = torch.zeros(1, dtype=torch.int32, device=dev)

    def run(self, r, phi, layer, with_vacc=True):
        """Both passes on one event, asynchronous on the current stream (the
        outputs stay in bufs_p, keep, n_keep and bufs_d)."""
        P, D = self.spec["prompt"], self.spec["displaced"]
        n = int(r.numel())
        H.hough_vote(self.plan_p, r, phi, self.acc_p)
        H.hough_peaks(self.plan_p, self.acc_p, P["min_votes"], self.pk_p, self.nf[0:1])
        H.assoc_cluster(self.plan_p, r, phi, layer, self.pk_p, self.nf[0:1], P["cluster"],
                        self.bufs_p, with_vacc=False)
        H.compact_hits(r, phi, layer, self.bufs_p.hit_owner[:n], self.r2[:n], self.phi2[:n],
                       self.layer2[:n], self.keep[:n], self.n_keep)
        # the displaced pass reads the kept-hit count on the device
        H.hough_vote_n(self.plan_d, self.r2[:n], self.phi2[:n], self.n_keep, self.acc_d)
        H.hough_peaks(self.plan_d, self.acc_d, D["min_votes"], self.pk_d, self.nf[1:2])
        H.assoc_cluster_n(self.plan_d, self.r2[:n], self.phi2[:n], self.layer2[:n], self.n_keep,
                          self.pk_d, self.nf[1:2], D["cluster"], self.bufs_d,
                          with_vacc=with_vacc, acc=self.acc_d)
        H.remap_track_hits(self.bufs_d, self.keep[:n])

    def to_host(self, n_hits):
        m = int(self.n_keep.item())
        return (self.bufs_p.to_host(n_hits), self.keep[:m].cpu().numpy(),
                self.bufs_d.to_host(m))

    def close(self):
        self.plan_p.close()
        self.plan_d.close()
