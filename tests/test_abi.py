"""The C-ABI library builds, loads and exports every entry point its header
declares (no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "houghtrig.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libpath():
    from paper_1309_6275_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return build.LIB


def test_header_declares_the_path():
    names = declared_functions()
    for f in ("hough_vote", "hough_peaks", "assoc_cluster", "ht_plan_create",
              "ht_plan_destroy", "ht_strerror"):
        assert f in names, names


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_1309_6275_amd import houghtrig
    assert sorted(houghtrig.EXPORTS) == declared_functions()


def test_struct_sizes_match_header_layout():
    from paper_1309_6275_amd import houghtrig as H
    assert ctypes.sizeof(H.Grid) == 32
    assert ctypes.sizeof(H.ClusterCfg) == 18 * 4
    assert H.TRACK_DTYPE.itemsize == 13 * 4 + 16 * 4
    assert H.OBJECT_DTYPE.itemsize == 8 * 4
    # serving loop structs (static_asserts on the C side hold the same sizes)
    assert ctypes.sizeof(H.ServerKind) == 128
    assert ctypes.sizeof(H.ServerCfg) == 576
    assert ctypes.sizeof(H.ServerOut) == 56
    assert ctypes.sizeof(H.ServerResult) == 96


def test_strerror_without_gpu(libpath):
    lib = ctypes.CDLL(libpath)
    lib.ht_strerror.restype = ctypes.c_char_p
    assert lib.ht_strerror(0) == b"ok"
    assert lib.ht_strerror(-1) == b"invalid argument"


def test_no_cpu_fallback_in_binding():
    """The binding never imports the oracle."""
    src = open(os.path.join(ROOT, "paper_1309_6275_amd", "houghtrig.py")).read()
    assert "oracle" not in src.replace("never imports", "")


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU and exits with status 2 for --gpus above 1,
    before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr and res.stdout == ""


def test_server_rejects_bad_configuration_before_the_device(libpath):
    """ht_server_create checks its configuration before any device call:
    each broken field alone gives HT_EINVAL, here without a GPU."""
    from paper_1309_6275_amd import configs as CF
    from paper_1309_6275_amd import houghtrig as H
    lib = ctypes.CDLL(libpath)
    lib.ht_server_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.ht_server_create.restype = ctypes.c_int
    params = (ctypes.c_float * H.CNN_PARAMS)()

    def base():
        c = H.ServerCfg()
        c.n_kinds = 1
        k = c.kinds[0]
        k.grid = H.grid_struct(CF.WORKLOADS[1]["grid"])
        k.cluster = H.cluster_struct(CF.WORKLOADS[1]["cluster"])
        k.min_votes, k.peak_cap = 7, 1024
        k.cnn_params = ctypes.cast(params, ctypes.c_void_p)
        k.cnn_threshold = 0.5
        c.max_hits, c.track_cap, c.object_cap, c.member_cap = 4096, 64, 8, 64
        c.hbm_budget, c.max_slots, c.queue_cap = 1 << 30, 1, 4
        c.batch_max, c.batch_max_hits = 4, 1000
        return c

    breaks = [("batch_max", 5), ("batch_max", -1), ("batch_max_hits", 0),
              ("batch_max_hits", 4097), ("reserved", 1), ("max_hits", 65536),
              ("work_budget", -1), ("n_kinds", 0)]
    for field, value in breaks:
        c = base()
        setattr(c, field, value)
        h = ctypes.c_void_p()
        assert lib.ht_server_create(ctypes.byref(c), ctypes.byref(h)) == H.HT_EINVAL, field
        assert not h.value
    for field, value in [("reserved", 2), ("cnn_threshold", float("nan")), ("peak_cap", 0)]:
        c = base()
        setattr(c.kinds[0], field, value)
        h = ctypes.c_void_p()
        assert lib.ht_server_create(ctypes.byref(c), ctypes.byref(h)) == H.HT_EINVAL, field
