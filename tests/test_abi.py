"""CPU-side checks of the C ABI: the library loads, exports every entry point
that include/*.h declares, rejects invalid arguments before touching a device,
and reports HG_ERR_DEVICE (never a CPU result) when no GPU is usable."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1907_02900_amd", "libhashgraph.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(hg_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1907_02900_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["hg_build", "hg_probe", "hg_probe_pairs", "hg_intersect", "hg_table_view",
                     "hg_table_free", "hg_status_string", "hg_hash", "hg_histogram",
                     "hg_exclusive_scan"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    lib.hg_status_string.restype = ctypes.c_char_p
    for s in range(8):
        assert lib.hg_status_string(s)
    assert lib.hg_status_string(0) == b"ok"


def test_invalid_arguments_rejected_on_host(lib):
    vp = ctypes.c_void_p
    lib.hg_hash.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                            vp, vp]
    dummy = vp(0x1000)
    assert lib.hg_hash(dummy, 10, 16, 100, 0, dummy, None) == 1      # key_bits
    assert lib.hg_hash(dummy, 10, 32, 0, 0, dummy, None) == 1        # V = 0
    assert lib.hg_hash(dummy, 10, 32, 1 << 32, 0, dummy, None) == 1  # V >= 2^32
    assert lib.hg_hash(dummy, 1 << 32, 32, 7, 0, dummy, None) == 1   # n >= 2^32
    assert lib.hg_hash(None, 10, 32, 7, 0, dummy, None) == 1         # NULL input
    lib.hg_build.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                             vp, vp, ctypes.POINTER(vp)]
    out = vp()
    assert lib.hg_build(dummy, 10, 64, 0, 0, None, None, ctypes.byref(out)) == 1
    assert lib.hg_build(dummy, 10, 32, 5, 0, None, None, None) == 1
    lib.hg_probe.argtypes = [vp, vp, ctypes.c_uint64, vp, vp, vp]
    assert lib.hg_probe(None, dummy, 5, dummy, None, None) == 1
    lib.hg_intersect.argtypes = [vp, vp, vp, vp, vp, ctypes.c_uint64, vp, vp]
    assert lib.hg_intersect(None, None, None, None, None, 0, None, None) == 1
    lib.hg_intersect_edges.argtypes = [vp, vp, vp, vp, vp]
    assert lib.hg_intersect_edges(None, None, dummy, None, None) == 1
    assert lib.hg_intersect_edges(dummy, dummy, None, None, None) == 1  # nothing asked for
    lib.hg_collection_build.argtypes = [vp, vp, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint64,
                                        ctypes.c_int32, ctypes.POINTER(vp), vp]
    assert lib.hg_collection_build(dummy, dummy, 4, 32, 0, 0, None, None) == 1   # no out
    assert lib.hg_collection_build(dummy, None, 4, 32, 0, 0, ctypes.byref(out), None) == 1
    assert lib.hg_collection_build(dummy, dummy, 4, 16, 0, 0, ctypes.byref(out), None) == 1
    assert lib.hg_collection_build(dummy, dummy, 4, 32, 0, 32, ctypes.byref(out), None) == 1
    assert lib.hg_collection_build(dummy, dummy, 0xFFFFFFFE, 32, 0, 0, ctypes.byref(out),
                                   None) == 1
    lib.hg_collection_intersect.argtypes = [vp, vp, vp, ctypes.c_uint64, vp, vp, vp]
    assert lib.hg_collection_intersect(None, None, dummy, 1, dummy, None, None) == 1
    lib.hg_collection_view.argtypes = [vp, vp]
    assert lib.hg_collection_view(None, dummy) == 1
    lib.hg_random_access_rate.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, vp, vp]
    ms = ctypes.c_double(0)
    assert lib.hg_random_access_rate(1, 3 << 20, 1000, ctypes.byref(ms), None) == 1  # not 2^k
    assert lib.hg_random_access_rate(1, 1024, 1000, ctypes.byref(ms), None) == 1     # < 4096
    assert lib.hg_random_access_rate(7, 1 << 20, 1000, ctypes.byref(ms), None) == 1  # kind
    assert lib.hg_random_access_rate(1, 1 << 20, 0, ctypes.byref(ms), None) == 1     # none
    assert lib.hg_random_access_rate(1, 1 << 20, 1000, None, None) == 1


def test_probe_orders_match_the_header():
    # the binding's probing orders are the header's defines
    import re
    from paper_1907_02900_amd import hg
    with open(os.path.join(ROOT, "include", "hashgraph.h")) as f:
        text = f.read()
    got = dict(re.findall(r"#define (HG_PROBE_[A-Z_]+) (\d+)", text))
    assert "hg_probe_ordered" in declared_functions()
    assert {k: int(v) for k, v in got.items()} == {
        "HG_PROBE_AUTO": hg.PROBE_AUTO, "HG_PROBE_INPUT_ORDER": hg.PROBE_INPUT_ORDER,
        "HG_PROBE_GROUPED": hg.PROBE_GROUPED,
        "HG_PROBE_GROUPED_UNLESS_SKEWED": hg.PROBE_GROUPED_UNLESS_SKEWED}


def test_bench_grouping_matrix_matches_the_documented_workspace():
    # 2 KiB of tile x range matrix per 4096 queries once V has 2^9 buckets
    # (512 ranges), fewer ranges (at least 2) below
    import bench
    assert bench.group_matrix_bytes(1 << 28, 1 << 28) == (1 << 16) * 2048
    assert bench.group_matrix_bytes(4097, 1 << 20) == 2 * 2048
    assert bench.group_matrix_bytes(4096, 100) == 128 * 4
    assert bench.group_matrix_bytes(10, 1) == 2 * 4


def test_no_cpu_fallback_without_gpu(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    vp = ctypes.c_void_p
    lib.hg_hash.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                            vp, vp]
    dummy = vp(0x1000)
    assert lib.hg_hash(dummy, 10, 32, 100, 0, dummy, None) == 3  # HG_ERR_DEVICE
    lib.hg_collection_build.argtypes = [vp, vp, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint64,
                                        ctypes.c_int32, ctypes.POINTER(vp), vp]
    out = vp()
    assert lib.hg_collection_build(dummy, dummy, 4, 32, 0, 0, ctypes.byref(out), None) == 3
    assert not out.value


def test_build_plan_is_host_only_and_consistent(lib):
    """hg_build_plan needs no device.  The plan's bins cover the range with
    power-of-two bucket ranges, the digits of its passes address every bin,
    a bin holds about 4096 32-bit (2048 64-bit) keys on average, and one pass
    suffices up to 512 bins."""
    from paper_1907_02900_amd import hg
    for kb, target in ((32, 4096), (64, 2048)):
        for n, V in ((1 << 28, 1 << 28), (1 << 28, 1 << 26), (1 << 28, 1 << 30), (1 << 27, 1 << 27),
                     (1 << 20, 1 << 20), (1000, 7), (5, (1 << 32) - 1), (0, 100), (300007, 300007)):
            p = hg.build_plan(n, V, kb)
            k = p["bucket_bits"]
            assert k <= 12 and p["bins"] == -(-V // (1 << k))
            bits = sum(p["digit_bits"][:p["passes"]])
            assert (1 << bits) >= p["bins"] and (bits == 0 or (1 << (bits - 1)) < p["bins"])
            assert p["passes"] == (1 if bits <= 9 else 2)
            assert p["tiles"][0] == -(-n // p["tile_keys"])
            if n and k < 12 and (1 << k) < V:
                per_bin = n * (1 << k) / V
                assert target / 2 <= per_bin <= target
            assert p["workspace_bytes"] >= n * (kb // 8 + 4)
    p = hg.build_plan(1 << 28, 1 << 28, 32)
    assert (p["bucket_bits"], p["bins"], p["passes"], p["digit_bits"]) == (12, 1 << 16, 2, [8, 8])
    assert hg.build_plan(1 << 16, 1 << 16, 32, bins=64)["bins"] == 64
    # a bin spans at most 2^12 buckets, so fewer bins than V / 2^12 are not planned
    assert hg.build_plan(1 << 20, 1 << 20, 32, bins=64)["bins"] == 256
    for bad in ((10, 0, 32, 0), (10, 1 << 32, 32, 0), (1 << 32, 7, 32, 0), (10, 7, 16, 0),
                (10, 7, 32, 8)):
        with pytest.raises(hg.HGError):
            hg.build_plan(*bad)


def test_set_allocator_validates_and_needs_no_device(lib):
    """hg_set_allocator takes both functions or neither (restoring
    hipMallocAsync); it is host state only and needs no device."""
    from paper_1907_02900_amd import hg
    L = hg.lib()
    L.hg_set_allocator.argtypes = [hg.ALLOC_FN, hg.FREE_FN, ctypes.c_void_p]
    L.hg_set_allocator.restype = ctypes.c_int
    a = hg.ALLOC_FN(lambda n, s, c: None)
    f = hg.FREE_FN(lambda p, s, c: None)
    assert L.hg_set_allocator(a, hg.FREE_FN(), None) == 1
    assert L.hg_set_allocator(hg.ALLOC_FN(), f, None) == 1
    assert L.hg_set_allocator(a, f, None) == 0
    assert L.hg_set_allocator(hg.ALLOC_FN(), hg.FREE_FN(), None) == 0
    with pytest.raises(ValueError):
        hg.set_allocator(alloc=lambda n, s: 0)
    hg.set_allocator()


def test_batch_options_validated_on_host(lib):
    """Unsupported launch shapes are rejected before any device work."""
    from paper_1907_02900_amd import hg
    L = hg._batch_sig()
    for part, th, it in ((12, 0, 0), (16, 256, 0), (16, 0, 4), (16, 64, 4), (8, 512, 8)):
        o = hg.BatchOpts()
        o.autotune, o.part_items, o.probe_threads, o.probe_items = 0, part, th, it
        out = ctypes.c_void_p()
        assert L.hg_batch_create(None, 0, 32, ctypes.byref(o), ctypes.byref(out)) == 1
        assert not out.value


def test_build_tune_rejects_bad_arguments_on_host(lib):
    from paper_1907_02900_amd import hg
    L = hg.lib()
    vp = ctypes.c_void_p
    L.hg_build_tune.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                                ctypes.c_uint64, ctypes.POINTER(hg.BuildOpts), vp,
                                ctypes.POINTER(hg.BuildOpts), ctypes.POINTER(hg.TuneInfo)]
    out = hg.BuildOpts()
    dummy = vp(0x1000)
    assert L.hg_build_tune(dummy, 10, 32, 100, 0, None, None, None, None) == 1      # no out
    assert L.hg_build_tune(dummy, 10, 16, 100, 0, None, None, ctypes.byref(out), None) == 1
    assert L.hg_build_tune(dummy, 10, 32, 0, 0, None, None, ctypes.byref(out), None) == 1
    bad = hg._opts(variant=hg.VARIANT_V1, stable=1)
    assert L.hg_build_tune(dummy, 10, 32, 100, 0, ctypes.byref(bad), None,
                           ctypes.byref(out), None) == 1
