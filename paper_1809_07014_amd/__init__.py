"""Python binding of the kmerhip C ABI (``include/kmerhip.h``).

Argument marshalling only: every step of k-mer analysis runs in the HIP
library ``libkmerhip.so`` built next to this file.  PyTorch is used for device
memory (read buffers, export destinations) and for the current HIP stream.
If the library is missing, every entry point raises; there is no CPU path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkmerhip.so")

KH_OK, KH_EINVAL, KH_ENOMEM, KH_EOVERFLOW, KH_EAGAIN, KH_EDEVICE, KH_ENOTFOUND = range(7)
_NAMES = {1: "KH_EINVAL", 2: "KH_ENOMEM", 3: "KH_EOVERFLOW", 4: "KH_EAGAIN",
          5: "KH_EDEVICE", 6: "KH_ENOTFOUND"}

PHASES = ("pack", "bloom", "count", "classify", "sort", "gather")
STATS = ("capacity", "claimed", "bloom_l1_new", "bloom_l2_new", "windows",
         "rows", "rebuilds", "table_bytes", "passed", "heavy", "k", "full_key_sort")

_lib = None


class KHError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_NAMES.get(code, str(code)), msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("min_count", ctypes.c_uint32),
                ("qual_offset", ctypes.c_uint32), ("qual_cutoff", ctypes.c_uint32),
                ("t_min_ext", ctypes.c_uint32), ("t_base", ctypes.c_uint32),
                ("err_ppm", ctypes.c_uint32), ("use_bloom", ctypes.c_uint32),
                ("bloom_bits", ctypes.c_uint32), ("load_factor", ctypes.c_float),
                ("owner_shards", ctypes.c_uint32), ("owner", ctypes.c_uint32)]


class ReadsStruct(ctypes.Structure):
    _fields_ = [("seq", ctypes.c_void_p), ("qual", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p), ("n_reads", ctypes.c_int64),
                ("on_device", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("load_factor", ctypes.c_float), ("bloom_bits", ctypes.c_uint32),
                ("bloom_lanes", ctypes.c_uint32), ("count_lanes", ctypes.c_uint32),
                ("tiles_per_block", ctypes.c_uint32), ("aggregate", ctypes.c_uint32),
                ("tails_overlap", ctypes.c_uint32), ("partitioned", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {f: (round(getattr(self, f), 4) if f == "load_factor" else getattr(self, f))
                for f, _ in self._fields_}


class TuneReport(ctypes.Structure):
    _fields_ = [("trials", ctypes.c_uint32), ("skipped", ctypes.c_uint32),
                ("start_ms", ctypes.c_double), ("best_ms", ctypes.c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_uint32), ("queue_cap", ctypes.c_uint32),
                ("chunk_reads", ctypes.c_int64), ("batch_bases", ctypes.c_int64),
                ("plain", ctypes.c_uint32)]


class PruneParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double)]


class PruneReport(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("removed", ctypes.c_int64),
                ("tau", ctypes.c_double), ("max_depth", ctypes.c_double)]


SERVER_STATS = ("completed", "launches", "windows", "busy_s", "max_active",
                "samples_resident", "device_bytes", "rehashes", "replayed",
                "pack_s", "grow_s", "peak_bytes", "allocs", "alloc_s", "retried",
                "in_use_bytes", "reserved_bytes")


def load():
    """Load ``libkmerhip.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libkmerhip.so is not built (run "
                           "paper_1809_07014_amd.build.build_library())")
    # torch ships its own HIP runtime (libamdhip64.so.7).  Loading torch first
    # makes the library's libamdhip64.so.7 dependency resolve to that same
    # runtime, so library and torch share one device context, streams and
    # memory instead of two runtimes competing for the GPU.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                             ctypes.c_uint32, ctypes.c_uint64)
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "kh_default_params": ([ctypes.POINTER(Params), u32], None),
        "kh_owner_of": ([P, u32, u32], u32),
        "kh_create": ([PP, i32, u64, P, P, P], i32),
        "kh_destroy": ([P], i32),
        "kh_release_cached": ([i32], i32),
        "kh_trim": ([P], i32),
        "kh_last_error": ([], ctypes.c_char_p),
        "kh_count": ([P, ctypes.POINTER(ReadsStruct), ctypes.POINTER(Params), P, PP], i32),
        "kh_count_multi_k": ([P, ctypes.POINTER(ReadsStruct), ctypes.POINTER(Params),
                              P, i32, P, PP], i32),
        "kh_table_info": ([P, P, P, P, P], i32),
        "kh_table_export": ([P, P, P, P, P, i32, P], i32),
        "kh_table_device_rows": ([P, PP, PP, PP, PP], i32),
        "kh_table_free": ([P], i32),
        "kh_set_timing": ([P, i32], i32),
        "kh_last_timing": ([P, P], i32),
        "kh_last_stats": ([P, P], i32),
        "kh_last_k_report": ([P, i32, P, P], i32),
        "kh_last_graphed": ([P, ctypes.POINTER(ctypes.c_int)], i32),
        "kh_count_noalloc": ([ctypes.POINTER(ReadsStruct), ctypes.POINTER(Params), P,
                              P, P, P, P, i64, ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_uint64)], i32),
        "kh_default_tuning": ([ctypes.POINTER(Tuning)], None),
        "kh_traverse": ([P, P, P, PP], i32),
        "kh_contigs_info": ([P, P, P, P, P, P], i32),
        "kh_contigs_export": ([P, P, P, P, P, P, i32], i32),
        "kh_contigs_free": ([P], i32),
        "kh_contigs_device": ([P, PP, PP], i32),
        "kh_merge_contigs": ([P, P, P, P, ctypes.c_int64, i32, P, PP], i32),
        "kh_default_prune_params": ([ctypes.POINTER(PruneParams)], None),
        "kh_heavy_hitters": ([P, u32, P, P, P, i64, P], i32),
        "kh_localize_reads": ([P, P, P, ctypes.POINTER(ReadsStruct), P, P, i32], i32),
        "kh_gather_reads": ([P, ctypes.POINTER(ReadsStruct), P, P, P, P, P], i32),
        "kh_prune": ([P, P, P, ctypes.POINTER(PruneParams), P, PP, P,
                      ctypes.POINTER(PruneReport)], i32),
        "kh_get_tuning": ([P, ctypes.POINTER(Tuning)], i32),
        "kh_set_tuning": ([P, ctypes.POINTER(Tuning)], i32),
        "kh_autotune": ([P, ctypes.POINTER(ReadsStruct), ctypes.POINTER(Params), P, i32, P,
                         i32, ctypes.POINTER(Tuning), ctypes.POINTER(TuneReport)], i32),
        "kh_autotune_cached": ([P, ctypes.POINTER(ReadsStruct), ctypes.POINTER(Params), P, i32,
                                P, i32, ctypes.c_char_p, ctypes.POINTER(Tuning),
                                ctypes.POINTER(TuneReport), ctypes.POINTER(ctypes.c_int)], i32),
        "kh_server_default_config": ([ctypes.POINTER(ServerConfig)], None),
        "kh_server_create": ([PP, i32, u64, ctypes.POINTER(Params), P, i32,
                              ctypes.POINTER(ServerConfig)], i32),
        "kh_server_submit": ([P, u64, ctypes.POINTER(ReadsStruct),
                              ctypes.POINTER(ctypes.c_uint64)], i32),
        "kh_server_poll": ([P, u64, ctypes.POINTER(ctypes.c_int),
                            ctypes.POINTER(ctypes.c_double)], i32),
        "kh_server_wait": ([P, u64, ctypes.POINTER(ctypes.c_double)], i32),
        "kh_server_finalize": ([P, u64, P], i32),
        "kh_server_stats": ([P, P], i32),
        "kh_server_destroy": ([P], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != KH_OK:
        raise KHError(rc, (load().kh_last_error() or b"").decode())


def release_cached(device: int = 0):
    """Return the device memory kept from destroyed contexts and servers on
    ``device`` to the driver."""
    _check(load().kh_release_cached(device))


def default_tuning() -> dict:
    t = Tuning()
    load().kh_default_tuning(ctypes.byref(t))
    return t.as_dict()


def params(k: int, min_count: int = 2, qual_offset: int = 33,
           qual_cutoff: int = 20, t_min_ext: int = 2, t_base: int = 1,
           err_ppm: int = 5000, use_bloom: bool = False, bloom_bits: int = 0,
           load_factor: float = 0.0, owner_shards: int = 0, owner: int = 0) -> Params:
    p = Params()
    load().kh_default_params(ctypes.byref(p), k)
    p.min_count, p.qual_offset, p.qual_cutoff = min_count, qual_offset, qual_cutoff
    p.t_min_ext, p.t_base, p.err_ppm = t_min_ext, t_base, err_ppm
    p.use_bloom, p.bloom_bits, p.load_factor = int(bool(use_bloom)), bloom_bits, load_factor
    p.owner_shards, p.owner = owner_shards, owner
    return p


def owner_of(key, shards: int) -> int:
    """Part of the k-mer space owning a canonical key (export words)."""
    k = np.ascontiguousarray(key, dtype=np.uint64)
    return int(load().kh_owner_of(k.ctypes.data_as(ctypes.c_void_p), k.size, shards))


@dataclass
class DeviceReads:
    """Read set resident in device memory (torch uint8/int64 tensors)."""
    seq: "object"
    qual: "object"
    offsets: "object"

    @property
    def n_reads(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @staticmethod
    def from_host(reads, device: str = "cuda") -> "DeviceReads":
        import torch
        seq = torch.from_numpy(np.ascontiguousarray(reads.seq)).to(device)
        qual = torch.from_numpy(np.ascontiguousarray(reads.qual)).to(device)
        off = torch.from_numpy(np.ascontiguousarray(reads.offsets, dtype=np.int64)).to(device)
        return DeviceReads(seq, qual, off)


NOALLOC_SCRATCH_BYTES = 64 << 20  # KH_NOALLOC_SCRATCH_BYTES
NOALLOC_MAX_BASES = 16 << 20      # KH_NOALLOC_MAX_BASES


def count_noalloc(reads: "DeviceReads", k: int, keys, counts, ext, codes, stream=None,
                  **kw):
    """kh_count_noalloc: count ``reads`` (on the device) at k into the
    caller's device tensors keys (uint64, max_rows x W), counts (int32/uint32,
    max_rows), ext (max_rows x 8) and codes (uint8, max_rows x 2); nothing is
    allocated on the device.  Returns (n_rows, n_windows); raises KHError
    (code KH_EOVERFLOW with the needed row count in ``needed``) on failure."""
    rs, keep = _reads_struct(reads)
    if not rs.on_device and rs.n_reads > 0:
        raise ValueError("count_noalloc takes DeviceReads")
    p = params(k, **kw)
    max_rows = int(counts.shape[0])
    W = (int(k) + 31) // 32
    if (tuple(keys.shape) != (max_rows, W) or tuple(ext.shape) != (max_rows, 8)
            or tuple(codes.shape) != (max_rows, 2)):
        raise ValueError("output shapes must be (n, W), (n,), (n, 8), (n, 2)")
    for tns, size in ((keys, 8), (counts, 4), (ext, 4), (codes, 1)):
        if not tns.is_cuda or not tns.is_contiguous() or tns.element_size() != size:
            raise ValueError("outputs must be contiguous device tensors of the row widths")
    n_rows, n_win = ctypes.c_int64(0), ctypes.c_uint64(0)
    rc = load().kh_count_noalloc(ctypes.byref(rs), ctypes.byref(p), _stream_ptr(stream),
                                 keys.data_ptr(), counts.data_ptr(), ext.data_ptr(),
                                 codes.data_ptr(), max_rows, ctypes.byref(n_rows),
                                 ctypes.byref(n_win))
    del keep
    if rc != KH_OK:
        err = KHError(rc, (load().kh_last_error() or b"").decode())
        err.needed = int(n_rows.value)
        raise err
    return int(n_rows.value), int(n_win.value)


def _reads_struct(reads):
    """ReadsStruct for host reads (numpy) or DeviceReads (torch, on device)."""
    if isinstance(reads, DeviceReads):
        return ReadsStruct(reads.seq.data_ptr(), reads.qual.data_ptr(),
                           reads.offsets.data_ptr(), reads.n_reads, 1), reads
    seq = np.ascontiguousarray(reads.seq, dtype=np.uint8)
    qual = np.ascontiguousarray(reads.qual, dtype=np.uint8)
    off = np.ascontiguousarray(reads.offsets, dtype=np.int64)
    keep = (seq, qual, off)
    return ReadsStruct(seq.ctypes.data, qual.ctypes.data, off.ctypes.data,
                       int(off.shape[0] - 1), 0), keep


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


class Table:
    """A k-mer table owned by the library (freed by ``free`` or on GC)."""

    def __init__(self, handle: int, ctx: "Context"):
        self._h = ctypes.c_void_p(handle)
        self._ctx = ctx  # keeps the context (and its memory pool) alive

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        k, W = ctypes.c_uint32(), ctypes.c_uint32()
        n, nw = ctypes.c_int64(), ctypes.c_uint64()
        _check(load().kh_table_info(self._h, ctypes.byref(k), ctypes.byref(W),
                                    ctypes.byref(n), ctypes.byref(nw)))
        return dict(k=k.value, W=W.value, n_rows=n.value, n_windows=nw.value)

    def to_numpy(self) -> dict:
        """Rows copied to host arrays, in the oracle's dictionary format."""
        inf = self.info()
        n, W = inf["n_rows"], inf["W"]
        keys = np.zeros((n, W), np.uint64)
        counts = np.zeros(n, np.uint32)
        ext = np.zeros((n, 8), np.uint32)
        codes = np.zeros((n, 2), np.uint8)
        if n:
            _check(load().kh_table_export(self._h, keys.ctypes.data,
                                          counts.ctypes.data, ext.ctypes.data,
                                          codes.ctypes.data, 0, None))
        return dict(k=inf["k"], W=W, n_rows=n, keys=keys, counts=counts,
                    ext=ext, codes=codes, n_windows=inf["n_windows"])

    def heavy_hitters(self, min_count: int = 4096, stream=None):
        """(keys (n, W), counts) of the rows with count >= min_count, in key
        order (kh_heavy_hitters)."""
        W = self.info()["W"]
        n = ctypes.c_int64()
        _check(load().kh_heavy_hitters(self._h, min_count, _stream_ptr(stream), None, None, 0,
                                       ctypes.byref(n)))
        keys = np.zeros((n.value, W), np.uint64)
        counts = np.zeros(n.value, np.uint32)
        if n.value:
            m = ctypes.c_int64()
            _check(load().kh_heavy_hitters(self._h, min_count, _stream_ptr(stream),
                                           keys.ctypes.data, counts.ctypes.data, n.value,
                                           ctypes.byref(m)))
        return keys, counts

    def free(self):
        if self._h:
            load().kh_table_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Contigs:
    """Contigs of a table (de Bruijn graph traversal), owned by the library."""

    def __init__(self, handle: int, ctx: "Context"):
        self._h = ctypes.c_void_p(handle)
        self._ctx = ctx

    def info(self) -> dict:
        k, nc, tb, ck = ctypes.c_uint32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        rounds = ctypes.c_int()
        _check(load().kh_contigs_info(self._h, ctypes.byref(k), ctypes.byref(nc),
                                      ctypes.byref(tb), ctypes.byref(ck), ctypes.byref(rounds)))
        return dict(k=k.value, n_contigs=nc.value, total_bases=tb.value,
                    cycle_kmers=ck.value, rounds=rounds.value)

    def to_numpy(self) -> dict:
        """seq (uint8 ASCII, back to back), offsets, n_kmers, depth, cycle."""
        inf = self.info()
        m, tb = inf["n_contigs"], inf["total_bases"]
        seq = np.zeros(tb, np.uint8)
        off = np.zeros(m + 1, np.int64)
        nk = np.zeros(m, np.int64)
        depth = np.zeros(m, np.uint64)
        cyc = np.zeros(m, np.uint8)
        _check(load().kh_contigs_export(self._h, seq.ctypes.data, off.ctypes.data,
                                        nk.ctypes.data, depth.ctypes.data, cyc.ctypes.data, 0))
        return dict(k=inf["k"], n_contigs=m, seq=seq, offsets=off, n_kmers=nk,
                    depth=depth, cycle=cyc.astype(bool))

    def lengths(self) -> np.ndarray:
        """Contig lengths in bases (offsets only are copied)."""
        m = self.info()["n_contigs"]
        off = np.zeros(m + 1, np.int64)
        _check(load().kh_contigs_export(self._h, None, off.ctypes.data, None, None, None, 0))
        return np.diff(off)

    def to_python(self) -> dict:
        """As ``to_numpy`` with the sequences as a list of str."""
        d = self.to_numpy()
        raw = d.pop("seq").tobytes().decode()
        off = d["offsets"]
        d["seqs"] = [raw[off[i]:off[i + 1]] for i in range(d["n_contigs"])]
        return d

    def free(self):
        if self._h:
            load().kh_contigs_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                            ctypes.c_void_p)


def _allocator_hooks(allocator):
    """(alloc_fn, free_fn, user) for kh_create; the callbacks are kept alive
    by the context that holds the tuple."""
    if allocator is None:
        return (None, None, None)
    if allocator == "torch":
        import torch

        def alloc(nbytes, device):
            return torch.cuda.caching_allocator_alloc(nbytes, device)

        def free(ptr, nbytes, device):
            torch.cuda.caching_allocator_delete(ptr)
    else:
        alloc, free = allocator

    def c_alloc(nbytes, device, _user):
        try:
            return int(alloc(int(nbytes), int(device)) or 0)
        except Exception:  # e.g. out of memory: the library reports KH_ENOMEM
            return 0

    def c_free(ptr, nbytes, device, _user):
        free(int(ptr), int(nbytes), int(device))

    return (_ALLOC_FN(c_alloc), _FREE_FN(c_free), None)


class Context:
    """A library context on one GPU with its own device memory pool."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, allocator=None):
        """allocator: None (hipMalloc), "torch" (torch's caching allocator)
        or a pair (alloc(bytes, device) -> int address or 0,
        free(address, bytes, device))."""
        self._hooks = _allocator_hooks(allocator)
        h = ctypes.c_void_p()
        _check(load().kh_create(ctypes.byref(h), device, hbm_budget, *self._hooks))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def count(self, reads, k: int, stream=None, **kw) -> Table:
        rs, keep = _reads_struct(reads)
        p = params(k, **kw)
        out = ctypes.c_void_p()
        _check(load().kh_count(self._h, ctypes.byref(rs), ctypes.byref(p),
                               _stream_ptr(stream), ctypes.byref(out)))
        del keep
        return Table(out.value, self)

    def count_multi_k(self, reads, ks, stream=None, **kw):
        rs, keep = _reads_struct(reads)
        p = params(int(ks[0]), **kw)
        karr = (ctypes.c_uint32 * len(ks))(*[int(x) for x in ks])
        outs = (ctypes.c_void_p * len(ks))()
        _check(load().kh_count_multi_k(self._h, ctypes.byref(rs), ctypes.byref(p),
                                       karr, len(ks), _stream_ptr(stream), outs))
        del keep
        return [Table(outs[i], self) for i in range(len(ks))]

    def trim(self):
        """Return the pool's cached device blocks to the driver (kh_trim)."""
        _check(load().kh_trim(self._h))

    def traverse(self, table: Table, stream=None) -> Contigs:
        """Contigs of ``table`` (kh_traverse)."""
        h = ctypes.c_void_p()
        _check(load().kh_traverse(self._h, table.handle, _stream_ptr(stream), ctypes.byref(h)))
        return Contigs(h.value, self)

    def merge_contigs(self, table: Table, contigs, stream=None) -> Table:
        """Table ``table`` merged with the k-mers of ``contigs`` (a Contigs
        object, used in place on the device, or a list of str)."""
        h = ctypes.c_void_p()
        if isinstance(contigs, Contigs):
            sp, op = ctypes.c_void_p(), ctypes.c_void_p()
            _check(load().kh_contigs_device(contigs._h, ctypes.byref(sp), ctypes.byref(op)))
            n = contigs.info()["n_contigs"]
            _check(load().kh_merge_contigs(self._h, table.handle, sp, op, n, 1,
                                           _stream_ptr(stream), ctypes.byref(h)))
        else:
            raw = "".join(contigs).encode()
            seq = np.frombuffer(raw, dtype=np.uint8).copy() if raw else np.zeros(1, np.uint8)
            off = np.zeros(len(contigs) + 1, np.int64)
            np.cumsum([len(c) for c in contigs], out=off[1:])
            _check(load().kh_merge_contigs(self._h, table.handle, seq.ctypes.data,
                                           off.ctypes.data, len(contigs), 0,
                                           _stream_ptr(stream), ctypes.byref(h)))
        return Table(h.value, self)

    def prune(self, table: Table, contigs: Contigs, alpha=None, beta=None, stream=None,
              removed_at: bool = False):
        """Algorithm 2 over ``contigs``, which were walked from ``table``
        (kh_prune).  Returns (kept Contigs, report dict) and, with
        removed_at=True, also the sweep that removed each contig (-1: kept)."""
        p = PruneParams()
        load().kh_default_prune_params(ctypes.byref(p))
        if alpha is not None:
            p.alpha = float(alpha)
        if beta is not None:
            p.beta = float(beta)
        rep = PruneReport()
        h = ctypes.c_void_p()
        arr = None
        if removed_at:
            arr = np.zeros(max(1, contigs.info()["n_contigs"]), np.int32)
        _check(load().kh_prune(self._h, table.handle, contigs._h, ctypes.byref(p),
                               _stream_ptr(stream), ctypes.byref(h),
                               None if arr is None else arr.ctypes.data, ctypes.byref(rep)))
        out = Contigs(h.value, self)
        report = dict(sweeps=rep.sweeps, removed=rep.removed, tau=rep.tau,
                      max_depth=rep.max_depth)
        if removed_at:
            return out, report, arr[:contigs.info()["n_contigs"]].copy()
        return out, report

    def localize_order(self, table: Table, contigs: Contigs, reads, stream=None):
        """Read order grouped by contig (kh_localize_reads): a torch int64
        tensor on the device for DeviceReads, else a numpy array."""
        rs, keep = _reads_struct(reads)
        n = rs.n_reads
        if isinstance(reads, DeviceReads):
            import torch
            order = torch.empty(max(n, 1), dtype=torch.int64, device=reads.offsets.device)
            _check(load().kh_localize_reads(self._h, table.handle, contigs._h, ctypes.byref(rs),
                                            _stream_ptr(stream), order.data_ptr(), 1))
            return order[:n]
        order = np.zeros(max(n, 1), np.int64)
        _check(load().kh_localize_reads(self._h, table.handle, contigs._h, ctypes.byref(rs),
                                        _stream_ptr(stream), order.ctypes.data, 0))
        del keep
        return order[:n]

    def gather_reads(self, reads: "DeviceReads", order, stream=None) -> "DeviceReads":
        """DeviceReads copied in ``order`` (a device int64 tensor;
        kh_gather_reads)."""
        import torch
        rs, _ = _reads_struct(reads)
        seq = torch.empty_like(reads.seq)
        qual = torch.empty_like(reads.qual)
        off = torch.empty_like(reads.offsets)
        order = order.contiguous()
        _check(load().kh_gather_reads(self._h, ctypes.byref(rs), order.data_ptr(),
                                      _stream_ptr(stream), seq.data_ptr(), qual.data_ptr(),
                                      off.data_ptr()))
        return DeviceReads(seq, qual, off)

    def localize(self, table: Table, contigs: Contigs, reads: "DeviceReads",
                 stream=None) -> "DeviceReads":
        """Reads grouped by contig, as new device buffers."""
        return self.gather_reads(reads, self.localize_order(table, contigs, reads, stream),
                                 stream)

    def tuning(self) -> dict:
        t = Tuning()
        _check(load().kh_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        """Change fields of the context's tuning (see kh_tuning)."""
        t = Tuning()
        _check(load().kh_get_tuning(self._h, ctypes.byref(t)))
        for k, v in kw.items():
            if k not in dict(Tuning._fields_):
                raise KeyError(k)
            setattr(t, k, v)
        _check(load().kh_set_tuning(self._h, ctypes.byref(t)))

    def autotune(self, reads, ks, stream=None, reps: int = 1, **kw):
        """Run the library's autotuner on this read set; the context keeps
        the chosen tuning.  Returns (tuning dict, report dict)."""
        rs, keep = _reads_struct(reads)
        p = params(int(ks[0]), **kw)
        karr = (ctypes.c_uint32 * len(ks))(*[int(x) for x in ks])
        t, r = Tuning(), TuneReport()
        _check(load().kh_autotune(self._h, ctypes.byref(rs), ctypes.byref(p), karr, len(ks),
                                  _stream_ptr(stream), reps, ctypes.byref(t), ctypes.byref(r)))
        del keep
        return t.as_dict(), {f: getattr(r, f) for f, _ in TuneReport._fields_}

    def autotune_cached(self, reads, ks, cache_path: str, stream=None, reps: int = 1, **kw):
        """kh_autotune_cached: the stored choice for this case if
        ``cache_path`` holds one, else the autotuner (its choice appended to
        the file).  Returns (tuning dict, report dict, hit)."""
        rs, keep = _reads_struct(reads)
        p = params(int(ks[0]), **kw)
        karr = (ctypes.c_uint32 * len(ks))(*[int(x) for x in ks])
        t, r, hit = Tuning(), TuneReport(), ctypes.c_int(0)
        _check(load().kh_autotune_cached(self._h, ctypes.byref(rs), ctypes.byref(p), karr,
                                         len(ks), _stream_ptr(stream), reps,
                                         os.fsencode(cache_path), ctypes.byref(t),
                                         ctypes.byref(r), ctypes.byref(hit)))
        del keep
        return (t.as_dict(), {f: getattr(r, f) for f, _ in TuneReport._fields_},
                bool(hit.value))

    def set_timing(self, on: bool = True):
        _check(load().kh_set_timing(self._h, int(on)))

    def timing(self) -> dict:
        ms = (ctypes.c_float * 6)()
        _check(load().kh_last_timing(self._h, ms))
        return dict(zip(PHASES, list(ms)))

    def stats(self) -> dict:
        v = (ctypes.c_uint64 * 12)()
        _check(load().kh_last_stats(self._h, v))
        return dict(zip(STATS, list(v)))

    def last_graphed(self) -> bool:
        """True if the last batched multi-k call replayed its counting
        passes as one HIP graph."""
        g = ctypes.c_int(0)
        _check(load().kh_last_graphed(self._h, ctypes.byref(g)))
        return bool(g.value)

    def k_report(self, i: int):
        """(phase times, statistics) of the i-th k of the last call."""
        ms = (ctypes.c_float * 6)()
        v = (ctypes.c_uint64 * 12)()
        _check(load().kh_last_k_report(self._h, i, ms, v))
        return dict(zip(PHASES, list(ms))), dict(zip(STATS, list(v)))

    def close(self):
        if self._h:
            load().kh_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching k-mer counting server (see kh_server_* in the
    header).  Submitted host read sets are referenced, not copied: the
    binding keeps them alive until their ticket completes."""

    def __init__(self, ks, device: int = 0, hbm_budget: int = 0, plain: bool = False,
                 max_active: int = 16, queue_cap: int = 1024,
                 chunk_reads: int = 16384, batch_bases: int = 32 << 20, **kw):
        lib = load()
        self.ks = [int(x) for x in ks]
        p = params(self.ks[0], **kw)
        cfg = ServerConfig()
        lib.kh_server_default_config(ctypes.byref(cfg))
        cfg.max_active, cfg.queue_cap = max_active, queue_cap
        cfg.chunk_reads, cfg.batch_bases, cfg.plain = chunk_reads, batch_bases, int(plain)
        karr = (ctypes.c_uint32 * len(self.ks))(*self.ks)
        h = ctypes.c_void_p()
        _check(lib.kh_server_create(ctypes.byref(h), device, hbm_budget,
                                    ctypes.byref(p), karr, len(self.ks),
                                    ctypes.byref(cfg)))
        self._h = h
        self._keep = {}

    def submit(self, sample: int, reads) -> int:
        rs, keep = _reads_struct(reads)
        if rs.on_device:
            raise ValueError("serving takes host reads")
        t = ctypes.c_uint64()
        _check(load().kh_server_submit(self._h, sample, ctypes.byref(rs), ctypes.byref(t)))
        self._keep[t.value] = keep
        return t.value

    def poll(self, ticket: int):
        done, lat = ctypes.c_int(), ctypes.c_double()
        _check(load().kh_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(lat)))
        if done.value:
            self._keep.pop(ticket, None)
        return bool(done.value), lat.value

    def wait(self, ticket: int) -> float:
        lat = ctypes.c_double()
        _check(load().kh_server_wait(self._h, ticket, ctypes.byref(lat)))
        self._keep.pop(ticket, None)
        return lat.value

    def finalize(self, sample: int):
        outs = (ctypes.c_void_p * len(self.ks))()
        _check(load().kh_server_finalize(self._h, sample, outs))
        return [Table(outs[i], self) for i in range(len(self.ks))]

    def stats(self) -> dict:
        v = (ctypes.c_double * len(SERVER_STATS))()
        _check(load().kh_server_stats(self._h, v))
        return dict(zip(SERVER_STATS, list(v)))

    def close(self):
        if self._h:
            load().kh_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
