"""Thin ctypes binding over libhashgraph.so (include/hashgraph.h).

Only argument marshalling lives here: device buffers are torch tensors on the
current ROCm device, the stream is torch's current stream, and every step of
the HashGraph path runs in the library's HIP kernels.  Unsigned key and id
arrays are carried in signed torch dtypes of the same width (uint32 <-> int32,
uint64 <-> int64); ``to_device`` / ``to_numpy`` convert bit-for-bit.

If the shared library is missing the import fails loudly: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HG_LIB", os.path.join(_PKG, "libhashgraph.so"))

HG_OK, HG_ERR_INVALID_ARG, HG_ERR_OOM, HG_ERR_DEVICE = 0, 1, 2, 3
HG_ERR_CAPACITY, HG_ERR_MISMATCH, HG_ERR_BUDGET, HG_ERR_NOT_FOUND = 4, 5, 6, 7
HG_ERR_TOO_LARGE = 8
NOALLOC_MAX_QUERIES = 1 << 22
VARIANT_AUTO, VARIANT_V1, VARIANT_V2 = 0, 1, 2


# Releases that arrived while the current stream was being captured into a
# graph.  Freeing device memory synchronises, which would invalidate the
# capture (a Table dropped by the garbage collector in the middle of someone's
# torch.cuda.graph block), so such releases wait for the next release made
# outside a capture.
_deferred = []


def _capturing() -> bool:
    try:
        return torch.cuda.is_available() and torch.cuda.is_current_stream_capturing()
    except Exception:
        return False


def _release(fn, handle):
    """Run fn(handle) now, or later if a stream capture is in progress."""
    if _capturing():
        _deferred.append((fn, handle))
        return
    while _deferred:
        f, h = _deferred.pop()
        f(h)
    fn(handle)


def flush_deferred_releases():
    """Free the objects whose release was deferred during a stream capture
    (no-op while capturing)."""
    if not _capturing():
        while _deferred:
            f, h = _deferred.pop()
            f(h)


class HGError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = int(status)
        super().__init__("%s: %s (status %d)" % (where, status_string(status), status))


class BuildOpts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("stable", ctypes.c_int32),
                ("bins", ctypes.c_uint32), ("block", ctypes.c_uint32),
                ("no_index", ctypes.c_int32), ("any_order", ctypes.c_int32),
                ("v1_plain", ctypes.c_int32), ("reserved", ctypes.c_uint32)]


class TableInfo(ctypes.Structure):
    _fields_ = [("d_offsets", ctypes.c_void_p), ("d_ids", ctypes.c_void_p),
                ("d_keys", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("hash_range", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("key_bits", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("device_bytes", ctypes.c_uint64)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("bucket_bits", ctypes.c_uint32), ("bins", ctypes.c_uint32),
                ("passes", ctypes.c_uint32), ("digit_bits", ctypes.c_uint32 * 2),
                ("tiles", ctypes.c_uint32 * 2), ("tile_keys", ctypes.c_uint32),
                ("workspace_bytes", ctypes.c_uint64)]


_lib = None


def lib():
    """Load libhashgraph.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhashgraph.so not built at %s; run `python -m "
                          "paper_1907_02900_amd.build` (there is no CPU fallback)" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    pu64 = ctypes.POINTER(ctypes.c_uint64)
    sig = {
        "hg_status_string": ([i32], ctypes.c_char_p),
        "hg_version": ([], u32),
        "hg_hash": ([vp, u64, i32, u64, u64, vp, vp], i32),
        "hg_histogram": ([vp, u64, i32, u64, u64, vp, vp], i32),
        "hg_exclusive_scan": ([vp, u64, vp, vp], i32),
        "hg_build": ([vp, u64, i32, u64, u64, ctypes.POINTER(BuildOpts), vp,
                      ctypes.POINTER(vp)], i32),
        "hg_table_create": ([u64, u64, i32, ctypes.POINTER(vp)], i32),
        "hg_build_plan": ([u64, u64, i32, u32, ctypes.POINTER(PlanInfo)], i32),
        "hg_table_build": ([vp, vp, u64, u64, u64, ctypes.POINTER(BuildOpts), vp], i32),
        "hg_table_view": ([vp, ctypes.POINTER(TableInfo)], i32),
        "hg_table_export": ([vp, vp, vp, vp, vp], i32),
        "hg_table_free": ([vp], None),
        "hg_probe": ([vp, vp, u64, vp, pu64, vp], i32),
        "hg_probe_ordered": ([vp, vp, u64, vp, pu64, i32, vp], i32),
        "hg_probe_pairs": ([vp, vp, u64, vp, vp, u64, pu64, vp], i32),
        "hg_probe_pairs_noalloc": ([vp, vp, u64, vp, vp, u64, pu64, vp], i32),
        "hg_intersect": ([vp, vp, vp, vp, vp, u64, pu64, vp], i32),
        "hg_intersect_edges": ([vp, vp, vp, pu64, vp], i32),
        "hg_table_erase": ([vp, vp, u64, pu64, vp], i32),
        "hg_table_lengths": ([vp, ctypes.POINTER(vp), pu64], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def status_string(s: int) -> str:
    return lib().hg_status_string(int(s)).decode()


def _check(rc: int, where: str):
    if rc != HG_OK:
        raise HGError(rc, where)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


# ---------------------------------------------------------------- arrays ---

# ------------------------------------------------------- workspace hook ---

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_hook = None  # the installed callbacks, kept alive while the library may call them


def set_allocator(alloc=None, free=None):
    """hg_set_allocator: alloc(bytes, stream_handle) -> device address (0 on
    failure) and free(address, stream_handle) back the library's temporary
    workspace; both None restores hipMallocAsync.  The functions are kept
    referenced here until replaced."""
    global _hook
    L = lib()
    if not hasattr(L, "_alloc_sig"):
        L.hg_set_allocator.argtypes = [ALLOC_FN, FREE_FN, ctypes.c_void_p]
        L.hg_set_allocator.restype = ctypes.c_int
        L._alloc_sig = True
    if alloc is None and free is None:
        _check(L.hg_set_allocator(ALLOC_FN(), FREE_FN(), None), "hg_set_allocator")
        _hook = None
        return
    if alloc is None or free is None:
        raise ValueError("give both alloc and free, or neither")

    def _a(nbytes, stream, _ctx):
        try:
            return int(alloc(int(nbytes), int(stream or 0))) or None
        except Exception:  # noqa: BLE001 -- a failed allocation is reported as NULL
            return None

    def _f(ptr, stream, _ctx):
        free(int(ptr), int(stream or 0))

    cb = (ALLOC_FN(_a), FREE_FN(_f))
    _check(L.hg_set_allocator(cb[0], cb[1], None), "hg_set_allocator")
    _hook = cb


def use_torch_allocator():
    """Back the library's workspace with PyTorch's caching allocator (stream
    ordered: a freed block is reused by later work on the same stream)."""
    set_allocator(lambda nbytes, stream: torch.cuda.caching_allocator_alloc(nbytes, stream=stream),
                  lambda ptr, stream: torch.cuda.caching_allocator_delete(ptr))


def to_device(a: np.ndarray, device="cuda") -> torch.Tensor:
    """numpy unsigned array -> device tensor of the same bits (signed dtype)."""
    a = np.ascontiguousarray(a)
    view = {4: np.int32, 8: np.int64}[a.dtype.itemsize]
    return torch.from_numpy(a.view(view)).to(device)


def to_numpy(t: torch.Tensor, dtype) -> np.ndarray:
    """device tensor -> numpy array reinterpreted as `dtype` (uint32/uint64)."""
    return t.detach().cpu().numpy().view(dtype)


def _key_bits(t: torch.Tensor) -> int:
    if t.dtype in (torch.int32, torch.uint32):
        return 32
    if t.dtype in (torch.int64, torch.uint64):
        return 64
    raise TypeError("keys must be 32- or 64-bit integer tensors, got %s" % t.dtype)


def _dev_keys(t: torch.Tensor) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("keys/queries must be device tensors")
    if not t.is_contiguous():
        raise ValueError("keys/queries must be contiguous")
    return t


def _u32(n, device) -> torch.Tensor:
    return torch.empty(int(n), dtype=torch.int32, device=device)


# ---------------------------------------------------------- single steps ---

def hg_hash(keys: torch.Tensor, hash_range: int, seed: int = 0, out=None, stream=None):
    keys = _dev_keys(keys)
    out = out if out is not None else _u32(keys.numel(), keys.device)
    _check(lib().hg_hash(_ptr(keys), keys.numel(), _key_bits(keys), int(hash_range),
                         int(seed) & (2**64 - 1), _ptr(out), _stream(stream)), "hg_hash")
    return out


def hg_histogram(keys: torch.Tensor, hash_range: int, seed: int = 0, out=None, stream=None):
    keys = _dev_keys(keys)
    out = out if out is not None else _u32(hash_range, keys.device)
    _check(lib().hg_histogram(_ptr(keys), keys.numel(), _key_bits(keys), int(hash_range),
                              int(seed) & (2**64 - 1), _ptr(out), _stream(stream)),
           "hg_histogram")
    return out


def hg_exclusive_scan(counts: torch.Tensor, out=None, stream=None):
    out = out if out is not None else _u32(counts.numel() + 1, counts.device)
    _check(lib().hg_exclusive_scan(_ptr(counts), counts.numel(), ctypes.c_void_p(out.data_ptr()),
                                   _stream(stream)), "hg_exclusive_scan")
    return out


# ----------------------------------------------------------------- tables ---

def build_plan(n: int, hash_range: int, key_bits: int = 32, bins: int = 0) -> dict:
    """The V2 plan (Alg. 2) the library follows for n keys over hash_range
    buckets (host only)."""
    p = PlanInfo()
    _check(lib().hg_build_plan(int(n), int(hash_range), int(key_bits), int(bins),
                               ctypes.byref(p)), "hg_build_plan")
    return {"bucket_bits": p.bucket_bits, "bins": p.bins, "passes": p.passes,
            "digit_bits": list(p.digit_bits), "tiles": list(p.tiles),
            "tile_keys": p.tile_keys, "workspace_bytes": p.workspace_bytes}


def _opts(variant=VARIANT_AUTO, stable=0, bins=0, block=0, index=True, any_order=False,
          v1_plain=False):
    o = BuildOpts()
    o.variant, o.stable, o.bins, o.block = int(variant), int(stable), int(bins), int(block)
    o.no_index = 0 if index else 1
    o.any_order = 1 if any_order else 0
    o.v1_plain = 1 if v1_plain else 0
    return o


class Table:
    """A device-resident HashGraph (owns its library handle)."""

    def __init__(self, handle: ctypes.c_void_p, device):
        self._h = handle
        self.device = device

    @classmethod
    def create(cls, n_capacity: int, range_capacity: int, key_bits: int = 32, device="cuda"):
        h = ctypes.c_void_p()
        _check(lib().hg_table_create(int(n_capacity), int(range_capacity), int(key_bits),
                                     ctypes.byref(h)), "hg_table_create")
        return cls(h, torch.device(device))

    def rebuild(self, keys: torch.Tensor, hash_range: int, seed: int = 0, variant=VARIANT_AUTO,
                stable=0, bins=0, block=0, index=True, any_order=False, v1_plain=False,
                stream=None):
        keys = _dev_keys(keys)
        o = _opts(variant, stable, bins, block, index, any_order, v1_plain)
        _check(lib().hg_table_build(self._h, _ptr(keys), keys.numel(), int(hash_range),
                                    int(seed) & (2**64 - 1), ctypes.byref(o), _stream(stream)),
               "hg_table_build")
        return self

    def info(self) -> TableInfo:
        i = TableInfo()
        _check(lib().hg_table_view(self._h, ctypes.byref(i)), "hg_table_view")
        return i

    @property
    def handle(self):
        return self._h

    def export(self, stream=None):
        """(offsets[V+1], ids[n], keys[n]) copied into new device tensors."""
        i = self.info()
        n = self.live()
        off = _u32(i.hash_range + 1, self.device)
        ids = _u32(n, self.device)
        keys = torch.empty(n, dtype=torch.int64 if i.key_bits == 64 else torch.int32,
                           device=self.device)
        _check(lib().hg_table_export(self._h, _ptr(off), _ptr(ids), _ptr(keys), _stream(stream)),
               "hg_table_export")
        return off, ids, keys

    def erase(self, keys: torch.Tensor, stream=None) -> int:
        """Remove every entry whose key is in `keys`; returns how many."""
        keys = _dev_keys(keys)
        removed = ctypes.c_uint64(0)
        _check(lib().hg_table_erase(self._h, _ptr(keys), keys.numel(), ctypes.byref(removed),
                                    _stream(stream)), "hg_table_erase")
        return int(removed.value)

    def lengths(self):
        """Device pointer (int) of the live bucket lengths after an erase, or None."""
        p = ctypes.c_void_p()
        _check(lib().hg_table_lengths(self._h, ctypes.byref(p), None), "hg_table_lengths")
        return p.value

    def live(self) -> int:
        """Number of live entries (the built count until an erase)."""
        n = ctypes.c_uint64(0)
        _check(lib().hg_table_lengths(self._h, None, ctypes.byref(n)), "hg_table_lengths")
        return int(n.value)

    def free(self):
        if self._h is not None and self._h.value:
            _release(lib().hg_table_free, self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def hg_build(keys: torch.Tensor, hash_range: int, seed: int = 0, variant=VARIANT_AUTO, stable=0,
             bins=0, block=0, index=True, any_order=False, v1_plain=False, stream=None) -> Table:
    keys = _dev_keys(keys)
    o = _opts(variant, stable, bins, block, index, any_order, v1_plain)
    h = ctypes.c_void_p()
    _check(lib().hg_build(_ptr(keys), keys.numel(), _key_bits(keys), int(hash_range),
                          int(seed) & (2**64 - 1), ctypes.byref(o), _stream(stream),
                          ctypes.byref(h)), "hg_build")
    return Table(h, keys.device)


class TuneInfo(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("candidates", ctypes.c_uint32), ("skew_class", ctypes.c_uint32),
                ("max_bucket", ctypes.c_uint32), ("cached", ctypes.c_uint32)]


def build_tune(keys: torch.Tensor, hash_range: int, seed: int = 0, variant=VARIANT_AUTO,
               stable=0, index=True, any_order=False, stream=None):
    """hg_build_tune: (keyword arguments of hg_build / Table.rebuild with the
    tuned launch parameters, info dict)."""
    keys = _dev_keys(keys)
    L = lib()
    if not hasattr(L, "_tune_sig"):
        L.hg_build_tune.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                    ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(BuildOpts),
                                    ctypes.c_void_p, ctypes.POINTER(BuildOpts),
                                    ctypes.POINTER(TuneInfo)]
        L.hg_build_tune.restype = ctypes.c_int
        L._tune_sig = True
    base = _opts(variant, stable, 0, 0, index, any_order)
    out, info = BuildOpts(), TuneInfo()
    _check(L.hg_build_tune(_ptr(keys), keys.numel(), _key_bits(keys), int(hash_range),
                           int(seed) & (2**64 - 1), ctypes.byref(base), _stream(stream),
                           ctypes.byref(out), ctypes.byref(info)), "hg_build_tune")
    kw = {"variant": out.variant, "stable": out.stable, "bins": out.bins, "block": out.block,
          "index": not out.no_index, "any_order": bool(out.any_order),
          "v1_plain": bool(out.v1_plain)}
    return kw, {f: getattr(info, f) for f, _ in TuneInfo._fields_}


def hg_probe(table: Table, queries: torch.Tensor, counts=True, total=False, out=None,
             stream=None):
    """Per-query match counts (device uint32 as int32) and/or the total."""
    queries = _dev_keys(queries)
    c = None
    if counts:
        c = out if out is not None else _u32(queries.numel(), queries.device)
    tot = ctypes.c_uint64(0)
    _check(lib().hg_probe(table.handle, _ptr(queries), queries.numel(), _ptr(c),
                          ctypes.byref(tot) if total else None, _stream(stream)), "hg_probe")
    return c, (int(tot.value) if total else None)


PROBE_AUTO, PROBE_INPUT_ORDER, PROBE_GROUPED, PROBE_GROUPED_UNLESS_SKEWED = 0, 1, 2, 3


def hg_probe_ordered(table: Table, queries: torch.Tensor, order: int, counts=True, total=False,
                     out=None, stream=None):
    """hg_probe with the probing order given: PROBE_INPUT_ORDER, PROBE_GROUPED
    (queries grouped by bucket range first), PROBE_GROUPED_UNLESS_SKEWED (the
    device keeps input order for skewed queries) or PROBE_AUTO."""
    queries = _dev_keys(queries)
    c = None
    if counts:
        c = out if out is not None else _u32(queries.numel(), queries.device)
    tot = ctypes.c_uint64(0)
    _check(lib().hg_probe_ordered(table.handle, _ptr(queries), queries.numel(), _ptr(c),
                                  ctypes.byref(tot) if total else None, int(order),
                                  _stream(stream)), "hg_probe_ordered")
    return c, (int(tot.value) if total else None)


def hg_probe_pairs(table: Table, queries: torch.Tensor, capacity=None, stream=None):
    """(build_ids, probe_ids, total).  With capacity None the total is taken
    from a counting call first."""
    queries = _dev_keys(queries)
    if capacity is None:
        _, capacity = hg_probe(table, queries, counts=False, total=True, stream=stream)
    b = _u32(max(int(capacity), 1), queries.device)
    p = _u32(max(int(capacity), 1), queries.device)
    tot = ctypes.c_uint64(0)
    rc = lib().hg_probe_pairs(table.handle, _ptr(queries), queries.numel(), _ptr(b), _ptr(p),
                              int(capacity), ctypes.byref(tot), _stream(stream))
    if rc == HG_ERR_CAPACITY:
        return None, None, int(tot.value)
    _check(rc, "hg_probe_pairs")
    t = int(tot.value)
    return b[:t], p[:t], t


def hg_probe_pairs_noalloc(table: Table, queries: torch.Tensor, build_ids: torch.Tensor,
                           probe_ids: torch.Tensor, stream=None):
    """hg_probe_pairs into caller-allocated pair arrays (capacity = their
    length) with the library's fixed workspace: (total, status).  status is
    HG_OK or HG_ERR_CAPACITY (total still reported); other errors raise."""
    queries = _dev_keys(queries)
    cap = min(build_ids.numel(), probe_ids.numel())
    tot = ctypes.c_uint64(0)
    rc = lib().hg_probe_pairs_noalloc(table.handle, _ptr(queries), queries.numel(),
                                      _ptr(build_ids), _ptr(probe_ids), cap, ctypes.byref(tot),
                                      _stream(stream))
    if rc not in (HG_OK, HG_ERR_CAPACITY):
        _check(rc, "hg_probe_pairs_noalloc")
    return int(tot.value), rc


def hg_intersect(a: Table, b: Table, counts=True, total=True, capacity=0, stream=None):
    """Alg. 3.  Returns (counts_b by b's input index or None, a_ids, b_ids,
    total)."""
    ib = b.info()
    c = _u32(ib.n, b.device) if counts else None
    cap = int(capacity)
    ai = _u32(max(cap, 1), b.device) if cap else None
    bi = _u32(max(cap, 1), b.device) if cap else None
    tot = ctypes.c_uint64(0)
    want_total = total or cap > 0
    rc = lib().hg_intersect(a.handle, b.handle, _ptr(c), _ptr(ai), _ptr(bi), cap,
                            ctypes.byref(tot) if want_total else None, _stream(stream))
    if rc == HG_ERR_CAPACITY:
        return c, None, None, int(tot.value)
    _check(rc, "hg_intersect")
    t = int(tot.value) if want_total else None
    if cap:
        return c, ai[:t], bi[:t], t
    return c, None, None, t


def hg_intersect_edges(a: Table, b: Table, counts=True, total=True, out=None, stream=None):
    """Alg. 3's counts in b's edge order (no scatter).  Returns (counts or
    None, total or None)."""
    ib = b.info()
    c = (out if out is not None else _u32(ib.n, b.device)) if counts else None
    tot = ctypes.c_uint64(0)
    _check(lib().hg_intersect_edges(a.handle, b.handle, _ptr(c),
                                    ctypes.byref(tot) if total else None, _stream(stream)),
           "hg_intersect_edges")
    return c, (int(tot.value) if total else None)


# ------------------------------------------------------------ collections ---

class CollectionInfo(ctypes.Structure):
    _fields_ = [("sets", ctypes.c_uint32), ("key_bits", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("range_shift", ctypes.c_int32),
                ("reserved", ctypes.c_uint32), ("n", ctypes.c_uint64),
                ("buckets", ctypes.c_uint64), ("heavy_keys", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64), ("d_set_offsets", ctypes.c_void_p),
                ("d_bucket_base", ctypes.c_void_p), ("d_offsets", ctypes.c_void_p),
                ("d_ids", ctypes.c_void_p), ("d_keys", ctypes.c_void_p)]


def _coll_sig():
    L = lib()
    if getattr(L, "_coll_sig", False):
        return L
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    L.hg_collection_build.argtypes = [vp, vp, u32, i32, u64, ctypes.c_int32,
                                      ctypes.POINTER(vp), vp]
    L.hg_collection_build.restype = i32
    L.hg_collection_view.argtypes = [vp, ctypes.POINTER(CollectionInfo)]
    L.hg_collection_view.restype = i32
    L.hg_collection_intersect.argtypes = [vp, vp, vp, u64, vp, ctypes.POINTER(ctypes.c_uint64),
                                          vp]
    L.hg_collection_intersect.restype = i32
    L.hg_collection_export.argtypes = [vp, vp, vp, vp, vp, vp]
    L.hg_collection_export.restype = i32
    L.hg_collection_free.argtypes = [vp]
    L.hg_collection_free.restype = None
    L._coll_sig = True
    return L


class Collection:
    """Many key sets, each with its own table, built once (hg_collection_build).

    keys: device tensor of all sets' keys, concatenated; set_offsets: device
    int32 tensor of S + 1 offsets (set s = keys[set_offsets[s]:set_offsets[s+1]])."""

    def __init__(self, keys: torch.Tensor, set_offsets: torch.Tensor, seed: int = 0,
                 range_shift: int = 0, stream=None):
        keys = _dev_keys(keys)
        if set_offsets.dtype not in (torch.int32, torch.uint32) or not set_offsets.is_cuda:
            raise ValueError("set_offsets must be a 32-bit device tensor")
        set_offsets = set_offsets.contiguous()
        self.device = keys.device
        self._h = ctypes.c_void_p()
        S = set_offsets.numel() - 1
        if S < 0:
            raise ValueError("set_offsets needs at least one entry")
        _check(_coll_sig().hg_collection_build(
            _ptr(keys), ctypes.c_void_p(set_offsets.data_ptr()), S, _key_bits(keys),
            int(seed) & 0xFFFFFFFFFFFFFFFF, int(range_shift), ctypes.byref(self._h),
            _stream(stream)), "hg_collection_build")

    @property
    def handle(self):
        return self._h

    def info(self) -> CollectionInfo:
        i = CollectionInfo()
        _check(_coll_sig().hg_collection_view(self._h, ctypes.byref(i)), "hg_collection_view")
        return i

    def arrays(self, stream=None):
        """Device copies (hg_collection_export): (bucket_base int64[S+2],
        offsets int32[buckets+1], ids int32[n], keys[n])."""
        i = self.info()
        kdt = torch.int64 if i.key_bits == 64 else torch.int32
        bb = torch.empty(i.sets + 2, dtype=torch.int64, device=self.device)
        off = torch.empty(i.buckets + 1, dtype=torch.int32, device=self.device)
        ids = torch.empty(i.n, dtype=torch.int32, device=self.device)
        ek = torch.empty(i.n, dtype=kdt, device=self.device)
        _check(_coll_sig().hg_collection_export(self._h, _ptr(bb), _ptr(off), _ptr(ids), _ptr(ek),
                                                _stream(stream)), "hg_collection_export")
        return bb, off, ids, ek

    def intersect(self, other: "Collection", pairs: torch.Tensor, counts=True, total=True,
                  stream=None):
        """Join sizes of (set i of self, set j of other) for each row (i, j) of
        pairs (device int32 [Q, 2]).  Returns (counts int64[Q] or None, total or None)."""
        if pairs.dtype not in (torch.int32, torch.uint32) or not pairs.is_cuda:
            raise ValueError("pairs must be a 32-bit device tensor")
        pairs = pairs.contiguous()
        Q = pairs.numel() // 2
        c = torch.empty(Q, dtype=torch.int64, device=self.device) if counts else None
        tot = ctypes.c_uint64(0)
        _check(_coll_sig().hg_collection_intersect(
            self._h, other._h, _ptr(pairs), Q, _ptr(c),
            ctypes.byref(tot) if total else None, _stream(stream)), "hg_collection_intersect")
        return c, (int(tot.value) if total else None)

    def free(self):
        if self._h is not None and self._h.value:
            _release(_coll_sig().hg_collection_free, self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ------------------------------------------------------------ measurement ---

def _prof_sig():
    L = lib()
    if getattr(L, "_prof_ready", False):
        return L
    L.hg_profile_enable.argtypes, L.hg_profile_enable.restype = [ctypes.c_int], ctypes.c_int
    L.hg_profile_reset.argtypes, L.hg_profile_reset.restype = [], ctypes.c_int
    L.hg_profile_count.argtypes = [ctypes.POINTER(ctypes.c_uint32)]
    L.hg_profile_count.restype = ctypes.c_int
    L.hg_profile_get.argtypes = [ctypes.c_uint32, ctypes.c_char_p, ctypes.c_uint32,
                                 ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double)]
    L.hg_profile_get.restype = ctypes.c_int
    L._prof_ready = True
    return L


MICRO_READ4, MICRO_READ16, MICRO_ATOMIC4 = 0, 1, 2


def random_access_rate(kind: int, footprint_bytes: int, accesses: int, stream=None) -> float:
    """Random accesses per second (hg_random_access_rate) of the given kind
    over a power-of-two footprint."""
    L = lib()
    L.hg_random_access_rate.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
    L.hg_random_access_rate.restype = ctypes.c_int
    ms = ctypes.c_double(0)
    _check(L.hg_random_access_rate(int(kind), int(footprint_bytes), int(accesses),
                                   ctypes.byref(ms), _stream(stream)), "hg_random_access_rate")
    return accesses / (ms.value * 1e-3)


def profile_enable(on: bool = True):
    _check(_prof_sig().hg_profile_enable(1 if on else 0), "hg_profile_enable")


def profile_reset():
    _check(_prof_sig().hg_profile_reset(), "hg_profile_reset")


def profile_report() -> dict:
    """{kernel name: (launches, total_ms)} for launches recorded while
    profiling was on (waits for their events)."""
    L = _prof_sig()
    cnt = ctypes.c_uint32(0)
    _check(L.hg_profile_count(ctypes.byref(cnt)), "hg_profile_count")
    out = {}
    buf = ctypes.create_string_buffer(128)
    for i in range(cnt.value):
        n = ctypes.c_uint64(0)
        ms = ctypes.c_double(0)
        _check(L.hg_profile_get(i, buf, 128, ctypes.byref(n), ctypes.byref(ms)), "hg_profile_get")
        out[buf.value.decode()] = (int(n.value), float(ms.value))
    return out


# ---------------------------------------------------------------- batched ---

class BatchItem(ctypes.Structure):
    _fields_ = [("d_keys", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("hash_range", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("d_queries", ctypes.c_void_p), ("m", ctypes.c_uint64),
                ("d_offsets", ctypes.c_void_p), ("d_ids", ctypes.c_void_p),
                ("d_ekeys", ctypes.c_void_p), ("d_counts", ctypes.c_void_p)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("autotune", ctypes.c_uint32), ("bin_target", ctypes.c_uint32),
                ("any_order", ctypes.c_uint32), ("part_items", ctypes.c_uint32),
                ("probe_threads", ctypes.c_uint32), ("probe_items", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 2)]


def _batch_sig():
    L = lib()
    if getattr(L, "_batch_ready", False):
        return L
    vp = ctypes.c_void_p
    L.hg_batch_create.argtypes = [ctypes.POINTER(BatchItem), ctypes.c_uint32, ctypes.c_int,
                                  ctypes.POINTER(BatchOpts), ctypes.POINTER(vp)]
    L.hg_batch_create.restype = ctypes.c_int
    L.hg_batch_run.argtypes, L.hg_batch_run.restype = [vp, vp], ctypes.c_int
    L.hg_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32),
                                ctypes.POINTER(ctypes.c_uint64)]
    L.hg_batch_info.restype = ctypes.c_int
    L.hg_batch_config.argtypes = [vp, ctypes.POINTER(BatchOpts)]
    L.hg_batch_config.restype = ctypes.c_int
    L.hg_batch_free.argtypes, L.hg_batch_free.restype = [vp], None
    L._batch_ready = True
    return L


class Batch:
    """A batched build+probe plan over device tensors.

    `tables` is a list of dicts with keys: keys, hash_range, seed, queries,
    and (outputs) offsets, ids, ekeys, counts -- all device tensors except the
    two integers.  Missing outputs are allocated here.  The plan keeps the
    tensors alive."""

    def __init__(self, tables, key_bits=32, autotune=True, bin_target=0, any_order=False,
                 part_items=0, probe_shape=(0, 0)):
        L = _batch_sig()
        self.tables = []
        items = (BatchItem * max(1, len(tables)))()
        kdt = torch.int64 if key_bits == 64 else torch.int32
        for i, t in enumerate(tables):
            keys, q = t["keys"], t.get("queries")
            dev = keys.device
            V = int(t["hash_range"])
            n = keys.numel()
            m = 0 if q is None else q.numel()
            d = dict(t)
            d.setdefault("offsets", torch.empty(V + 1, dtype=torch.int32, device=dev))
            d.setdefault("ids", torch.empty(max(n, 1), dtype=torch.int32, device=dev))
            d.setdefault("ekeys", torch.empty(max(n, 1), dtype=kdt, device=dev))
            d.setdefault("counts", torch.empty(max(m, 1), dtype=torch.int32, device=dev))
            it = items[i]
            it.d_keys = keys.data_ptr() if n else None
            it.n = n
            it.hash_range = V
            it.seed = int(t.get("seed", 0)) & (2**64 - 1)
            it.d_queries = q.data_ptr() if m else None
            it.m = m
            it.d_offsets = d["offsets"].data_ptr()
            it.d_ids = d["ids"].data_ptr()
            it.d_ekeys = d["ekeys"].data_ptr()
            it.d_counts = d["counts"].data_ptr() if m else None
            self.tables.append(d)
        o = BatchOpts()
        o.autotune = 1 if autotune else 0
        o.bin_target = int(bin_target)
        o.any_order = 1 if any_order else 0
        o.part_items = int(part_items)
        o.probe_threads, o.probe_items = int(probe_shape[0]), int(probe_shape[1])
        h = ctypes.c_void_p()
        _check(L.hg_batch_create(items, len(tables), int(key_bits), ctypes.byref(o),
                                 ctypes.byref(h)), "hg_batch_create")
        self._h = h

    def run(self, stream=None):
        _check(_batch_sig().hg_batch_run(self._h, _stream(stream)), "hg_batch_run")

    def info(self):
        t = ctypes.c_uint32(0)
        w = ctypes.c_uint64(0)
        _check(_batch_sig().hg_batch_info(self._h, ctypes.byref(t), ctypes.byref(w)),
               "hg_batch_info")
        o = BatchOpts()
        _check(_batch_sig().hg_batch_config(self._h, ctypes.byref(o)), "hg_batch_config")
        return {"bin_target": int(t.value), "workspace_bytes": int(w.value),
                "part_items": int(o.part_items),
                "probe_shape": (int(o.probe_threads), int(o.probe_items))}

    def free(self):
        if self._h is not None and self._h.value:
            _release(_batch_sig().hg_batch_free, self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------- serving ---

class ServerOpts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("streams", ctypes.c_uint32),
                ("max_inflight", ctypes.c_uint32), ("merge_max", ctypes.c_uint32),
                ("merge_keys", ctypes.c_uint32), ("workers", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 3)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("evictions", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("merged_requests", ctypes.c_uint64),
                ("keys", ctypes.c_uint64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("resident_bytes", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("resident_tables", ctypes.c_uint32), ("held_requests", ctypes.c_uint32)]


def _server_sig():
    L = lib()
    if getattr(L, "_server_ready", False):
        return L
    vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    pu64 = ctypes.POINTER(u64)
    L.hg_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    L.hg_server_submit_build.argtypes = [vp, vp, u64, i32, u64, u64, pu64, pu64]
    L.hg_server_submit_probe.argtypes = [vp, u64, vp, u64, vp, pu64]
    L.hg_server_wait.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_int)]
    L.hg_server_drain.argtypes = [vp]
    L.hg_server_export.argtypes = [vp, u64, vp, vp, vp, vp]
    L.hg_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.hg_server_reset_stats.argtypes = [vp]
    for f in ("hg_server_create", "hg_server_submit_build", "hg_server_submit_probe",
              "hg_server_wait", "hg_server_drain", "hg_server_export", "hg_server_stats_get",
              "hg_server_reset_stats"):
        getattr(L, f).restype = i32
    L.hg_server_destroy.argtypes, L.hg_server_destroy.restype = [vp], None
    L._server_ready = True
    return L


class Server:
    """The library's request loop.  Submitted tensors are kept alive here
    until their request completes."""

    def __init__(self, budget_bytes=0, streams=0, max_inflight=0, merge_max=0, merge_keys=0,
                 workers=0):
        L = _server_sig()
        o = ServerOpts()
        o.budget_bytes, o.streams, o.max_inflight = int(budget_bytes), int(streams), int(max_inflight)
        o.merge_max, o.merge_keys = int(merge_max), int(merge_keys)
        o.workers = int(workers)
        h = ctypes.c_void_p()
        _check(L.hg_server_create(ctypes.byref(o), ctypes.byref(h)), "hg_server_create")
        self._h = h
        self._keep = {}  # tensors the device still reads, until their request completes
        self._meta = {}
        self._seq = 0

    def submit_build(self, keys: torch.Tensor, hash_range: int, seed: int = 0, want_id=True):
        """(table_id, request_id).  With want_id False the request keeps no
        record after it completes (request_id None: it cannot be waited on;
        drain() waits for it)."""
        keys = _dev_keys(keys)
        tid, rid = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(_server_sig().hg_server_submit_build(
            self._h, _ptr(keys), keys.numel(), _key_bits(keys), int(hash_range),
            int(seed) & (2**64 - 1), ctypes.byref(tid), ctypes.byref(rid) if want_id else None),
            "hg_server_submit_build")
        self._hold(rid.value if want_id else None, (keys,))
        self._meta[tid.value] = (keys.numel(), int(hash_range), _key_bits(keys))
        return tid.value, (rid.value if want_id else None)

    def submit_probe(self, table_id: int, queries: torch.Tensor, counts: torch.Tensor = None,
                     want_id=True):
        """(request_id, counts); request_id is None with want_id False."""
        queries = _dev_keys(queries)
        if counts is None:
            counts = _u32(max(queries.numel(), 1), queries.device)
        rid = ctypes.c_uint64(0)
        _check(_server_sig().hg_server_submit_probe(
            self._h, int(table_id), _ptr(queries), queries.numel(), _ptr(counts),
            ctypes.byref(rid) if want_id else None), "hg_server_submit_probe")
        self._hold(rid.value if want_id else None, (queries, counts))
        return (rid.value if want_id else None), counts

    def wait(self, request_id: int) -> int:
        st = ctypes.c_int(0)
        _check(_server_sig().hg_server_wait(self._h, int(request_id), ctypes.byref(st)),
               "hg_server_wait")
        self._keep.pop(int(request_id), None)
        return int(st.value)

    def _hold(self, rid, tensors):
        # a request without an id is held under a negative key until drain()
        if rid is None:
            self._seq += 1
            rid = -self._seq
        self._keep[rid] = tensors

    def drain(self):
        _check(_server_sig().hg_server_drain(self._h), "hg_server_drain")
        self._keep.clear()

    def export(self, table_id: int, stream=None):
        """(offsets, ids, keys) copies of a resident table, or None if it is
        not resident."""
        n, V, kb = self._meta[int(table_id)]
        dev = torch.device("cuda")
        off = _u32(V + 1, dev)
        ids = _u32(max(n, 1), dev)
        keys = torch.empty(max(n, 1), dtype=torch.int64 if kb == 64 else torch.int32, device=dev)
        rc = _server_sig().hg_server_export(self._h, int(table_id), _ptr(off), _ptr(ids),
                                            _ptr(keys), _stream(stream))
        if rc == HG_ERR_NOT_FOUND:
            return None
        _check(rc, "hg_server_export")
        return off, ids[:n], keys[:n]

    def stats(self) -> dict:
        s = ServerStats()
        _check(_server_sig().hg_server_stats_get(self._h, ctypes.byref(s)), "hg_server_stats_get")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_ if f != "reserved"}

    def reset_stats(self):
        _check(_server_sig().hg_server_reset_stats(self._h), "hg_server_reset_stats")

    def close(self):
        if self._h is not None and self._h.value:
            # the tensors stay referenced until the server has finished
            keep = self._keep
            _release(lambda h: (_server_sig().hg_server_destroy(h), keep.clear()), self._h)
        self._h = None
        self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
