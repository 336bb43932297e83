"""The seeded generator's paper-geometry and mixed-stream events (inputs
only: no arithmetic of the method is involved)."""
import numpy as np

from paper_1309_6275_amd import eventgen as G


def test_paper_geometry_events():
    ev = G.make_paper_event(5_000_123, n_prompt=20, n_jets=2, jet_ntrk=10)
    # ten hits per track: prompt tracks reach 110 cm, jet vertices lie inside the first layer
    assert np.all(ev.trk_nhits == 10)
    assert len(ev.vtx_rho) == 2 and np.all((ev.vtx_rho >= 4.0) & (ev.vtx_rho <= 10.0))
    # hits sit within a few resolutions of their layer radius (0.4 mm in x and y)
    dr = ev.r - np.array(G.PAPER_RADII, np.float32)[ev.layer]
    assert np.all(np.abs(dr) < 0.3) and 0.02 < np.std(dr) < 0.06
    assert ev.n_hits == 10 * (20 + 2 * 10)


def test_serving_events_sizes():
    for kind in (0, 1):
        n = [G.make_serving_event(kind, 900 + i).n_hits for i in range(6)]
        assert all(1500 <= x <= 65535 for x in n), n
