"""CPU oracle for k-mer analysis -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It wraps ``oracle.c`` (plain C, built into ``liboracle.so``) with
ctypes and returns NumPy arrays in the same row format as the GPU library's
export, so that tests can compare the two byte for byte.  It imports nothing
from the GPU package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC_TRAVERSE = os.path.join(_HERE, "traverse.c")
_SRC_MERGE = os.path.join(_HERE, "merge.c")
_SRC_PRUNE = os.path.join(_HERE, "prune.c")
_SRC_LOCALIZE = os.path.join(_HERE, "localize.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-ffp-contract=off", "-o", tmp, _SRC,
                               _SRC_TRAVERSE, _SRC_MERGE, _SRC_PRUNE, _SRC_LOCALIZE])
        os.replace(tmp, _SO)
    return _SO


class _Contigs(ctypes.Structure):
    _fields_ = [("n_contigs", ctypes.c_int64), ("total_len", ctypes.c_int64),
                ("seq", ctypes.POINTER(ctypes.c_char)),
                ("offsets", ctypes.POINTER(ctypes.c_int64)),
                ("n_kmers", ctypes.POINTER(ctypes.c_int64)),
                ("depth", ctypes.POINTER(ctypes.c_uint64)),
                ("cycle", ctypes.POINTER(ctypes.c_uint8))]


class _Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("min_count", ctypes.c_uint32),
                ("qual_offset", ctypes.c_int32), ("qual_cutoff", ctypes.c_int32),
                ("t_min_ext", ctypes.c_uint32), ("t_base", ctypes.c_uint32),
                ("err_ppm", ctypes.c_uint32)]


class _Table(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("W", ctypes.c_uint32),
                ("n_rows", ctypes.c_int64),
                ("keys", ctypes.POINTER(ctypes.c_uint64)),
                ("counts", ctypes.POINTER(ctypes.c_uint32)),
                ("ext", ctypes.POINTER(ctypes.c_uint32)),
                ("codes", ctypes.POINTER(ctypes.c_uint8)),
                ("n_windows", ctypes.c_uint64), ("n_distinct", ctypes.c_uint64),
                ("sum_left", ctypes.c_uint64), ("sum_right", ctypes.c_uint64)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        TP = ctypes.POINTER(ctypes.POINTER(_Table))
        lib.oracle_count.argtypes = [P, P, P, ctypes.c_int64,
                                     ctypes.POINTER(_Params), TP]
        lib.oracle_count_shard.argtypes = [P, P, P, ctypes.c_int64,
                                           ctypes.POINTER(_Params),
                                           ctypes.c_uint64, ctypes.c_uint64, TP]
        lib.oracle_count_keys.argtypes = [P, P, P, ctypes.c_int64,
                                          ctypes.POINTER(_Params), P,
                                          ctypes.c_int64, P, P]
        lib.oracle_shard_of.argtypes = [P, ctypes.c_uint32, ctypes.c_uint64]
        lib.oracle_shard_of.restype = ctypes.c_uint64
        lib.oracle_classify_side.argtypes = [P, ctypes.c_uint64,
                                             ctypes.POINTER(_Params)]
        lib.oracle_classify_side.restype = ctypes.c_uint8
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        lib.oracle_free.argtypes = [ctypes.POINTER(_Table)]
        lib.oracle_free.restype = None
        lib.oracle_traverse.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.POINTER(_Contigs))]
        lib.oracle_merge.argtypes = [P, P, P, P, ctypes.c_int64, ctypes.c_uint32, P, P,
                                     ctypes.c_int64, TP]
        lib.oracle_contigs_free.argtypes = [ctypes.POINTER(_Contigs)]
        lib.oracle_contigs_free.restype = None
        lib.oracle_prune.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_uint32,
                                     ctypes.c_double, ctypes.c_double, P, P]
        lib.oracle_localize.argtypes = [P, P, ctypes.c_int64, ctypes.c_uint32, P, P,
                                        ctypes.c_int64, P]
        _lib = lib
    return _lib


def params(k: int, min_count: int = 2, qual_offset: int = 33,
           qual_cutoff: int = 20, t_min_ext: int = 2, t_base: int = 1,
           err_ppm: int = 5000) -> _Params:
    return _Params(k, min_count, qual_offset, qual_cutoff, t_min_ext, t_base,
                   err_ppm)


def _reads_args(reads):
    seq = np.ascontiguousarray(reads.seq, dtype=np.uint8)
    qual = np.ascontiguousarray(reads.qual, dtype=np.uint8)
    off = np.ascontiguousarray(reads.offsets, dtype=np.int64)
    keep = (seq, qual, off)
    return keep, (seq.ctypes.data, qual.ctypes.data, off.ctypes.data,
                  int(off.shape[0] - 1))


def _to_numpy(tp) -> dict:
    t = tp.contents
    n, W = int(t.n_rows), int(t.W)
    def arr(ptr, count, dtype):
        if count == 0:
            return np.zeros(0, dtype=dtype)
        return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dtype, copy=True)
    out = dict(k=int(t.k), W=W, n_rows=n,
               keys=arr(t.keys, n * W, np.uint64).reshape(n, W),
               counts=arr(t.counts, n, np.uint32),
               ext=arr(t.ext, n * 8, np.uint32).reshape(n, 8),
               codes=arr(t.codes, n * 2, np.uint8).reshape(n, 2),
               n_windows=int(t.n_windows), n_distinct=int(t.n_distinct),
               sum_left=int(t.sum_left), sum_right=int(t.sum_right))
    _load().oracle_free(tp)
    return out


def count(reads, k: int, **kw) -> dict:
    """Full k-mer table of ``reads`` (rows ascending by key)."""
    lib = _load()
    keep, a = _reads_args(reads)
    p = params(k, **kw)
    tp = ctypes.POINTER(_Table)()
    rc = lib.oracle_count(*a, ctypes.byref(p), ctypes.byref(tp))
    if rc != 0:
        raise ValueError("oracle_count failed (%d)" % rc)
    del keep
    return _to_numpy(tp)


def count_shard(reads, k: int, S: int, s: int, **kw) -> dict:
    """Rows of the k-mers in shard s of S (see ``shard_of``)."""
    lib = _load()
    keep, a = _reads_args(reads)
    p = params(k, **kw)
    tp = ctypes.POINTER(_Table)()
    rc = lib.oracle_count_shard(*a, ctypes.byref(p), S, s, ctypes.byref(tp))
    if rc != 0:
        raise ValueError("oracle_count_shard failed (%d)" % rc)
    del keep
    return _to_numpy(tp)


def set_threads(n: int) -> None:
    """OpenMP threads of the calling thread's later oracle calls."""
    _load().oracle_set_threads(int(n))


def count_keys(reads, k: int, keys: np.ndarray, **kw):
    """(counts[nq], ext[nq, 8]) of the query keys, before the threshold."""
    lib = _load()
    keep, a = _reads_args(reads)
    p = params(k, **kw)
    q = np.ascontiguousarray(keys, dtype=np.uint64)
    nq = int(q.shape[0])
    counts = np.zeros(nq, np.uint64)
    ext = np.zeros((nq, 8), np.uint64)
    rc = lib.oracle_count_keys(*a, ctypes.byref(p), q.ctypes.data, nq,
                               counts.ctypes.data, ext.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_count_keys failed (%d)" % rc)
    del keep
    return counts, ext


def shard_of(key_words, S: int) -> int:
    w = np.ascontiguousarray(key_words, dtype=np.uint64)
    return int(_load().oracle_shard_of(w.ctypes.data, int(w.shape[0]), S))


def classify_side(c, depth: int, **kw) -> str:
    """Extension letter of one side from its A,C,G,T tallies and the depth."""
    a = np.ascontiguousarray(c, dtype=np.uint64)
    p = params(1, **kw)
    return chr(_load().oracle_classify_side(a.ctypes.data, depth, ctypes.byref(p)))


def traverse(table: dict) -> dict:
    """Contigs of a k-mer table (rows as returned by ``count`` or the GPU
    export): sequences (str), k-mers and depth per contig, cycle flags, in
    the order of each contig's smallest k-mer."""
    lib = _load()
    n, k = int(table["n_rows"]), int(table["k"])
    keys = np.ascontiguousarray(table["keys"], dtype=np.uint64)
    counts = np.ascontiguousarray(table["counts"], dtype=np.uint32)
    codes = np.ascontiguousarray(table["codes"], dtype=np.uint8)
    cp = ctypes.POINTER(_Contigs)()
    rc = lib.oracle_traverse(keys.ctypes.data, counts.ctypes.data, codes.ctypes.data,
                             n, k, ctypes.byref(cp))
    if rc != 0:
        raise ValueError("oracle_traverse failed (%d)" % rc)
    c = cp.contents
    m = int(c.n_contigs)
    total = int(c.total_len)
    seq = ctypes.string_at(c.seq, total).decode() if total else ""
    off = np.ctypeslib.as_array(c.offsets, shape=(m + 1,)).copy()
    out = dict(k=k, n_contigs=m,
               seqs=[seq[off[i]:off[i + 1]] for i in range(m)],
               n_kmers=(np.ctypeslib.as_array(c.n_kmers, shape=(m,)).copy()
                        if m else np.zeros(0, np.int64)),
               depth=(np.ctypeslib.as_array(c.depth, shape=(m,)).copy()
                      if m else np.zeros(0, np.uint64)),
               cycle=(np.ctypeslib.as_array(c.cycle, shape=(m,)).astype(bool)
                      if m else np.zeros(0, bool)))
    lib.oracle_contigs_free(cp)
    return out


def merge(table: dict, contigs) -> dict:
    """Rows of ``table`` merged with every k-mer of ``contigs`` (list of str),
    in the table dictionary format; n_windows is the table's."""
    lib = _load()
    n, k = int(table["n_rows"]), int(table["k"])
    keys = np.ascontiguousarray(table["keys"], dtype=np.uint64)
    counts = np.ascontiguousarray(table["counts"], dtype=np.uint32)
    ext = np.ascontiguousarray(table["ext"], dtype=np.uint32)
    codes = np.ascontiguousarray(table["codes"], dtype=np.uint8)
    raw = "".join(contigs).encode()
    seq = np.frombuffer(raw, dtype=np.uint8).copy() if raw else np.zeros(1, np.uint8)
    off = np.zeros(len(contigs) + 1, np.int64)
    np.cumsum([len(c) for c in contigs], out=off[1:])
    tp = ctypes.POINTER(_Table)()
    rc = lib.oracle_merge(keys.ctypes.data, counts.ctypes.data, ext.ctypes.data,
                          codes.ctypes.data, n, k, seq.ctypes.data, off.ctypes.data,
                          len(contigs), ctypes.byref(tp))
    if rc != 0:
        raise ValueError("oracle_merge failed (%d)" % rc)
    out = _to_numpy(tp)
    out["n_windows"] = int(table.get("n_windows", 0))
    return out


PRUNE_ALPHA = 0.1  # tau grows by 10 % per sweep (the paper gives no value)
PRUNE_BETA = 0.2   # relative depth cut (the paper gives no value)


def prune(contigs, k: int, depth, alpha: float = PRUNE_ALPHA, beta: float = PRUNE_BETA):
    """Algorithm 2 over contigs (list of str, A/C/G/T, no k-mer shared
    between contigs) with the given depth sums.  Returns (removed_at, sweeps):
    removed_at[c] = the sweep that removed contig c, or -1."""
    lib = _load()
    n = len(contigs)
    raw = "".join(contigs).encode()
    seq = np.frombuffer(raw, dtype=np.uint8).copy() if raw else np.zeros(1, np.uint8)
    off = np.zeros(n + 1, np.int64)
    np.cumsum([len(c) for c in contigs], out=off[1:])
    dep = np.ascontiguousarray(depth, dtype=np.uint64)
    if len(dep) != n:
        raise ValueError("one depth per contig")
    if n == 0:
        dep = np.zeros(1, np.uint64)
    removed = np.zeros(max(n, 1), np.int32)
    sweeps = ctypes.c_int64(0)
    rc = lib.oracle_prune(seq.ctypes.data, off.ctypes.data, dep.ctypes.data, n, k,
                          float(alpha), float(beta), removed.ctypes.data,
                          ctypes.addressof(sweeps))
    if rc != 0:
        raise ValueError("oracle_prune failed (%d)" % rc)
    return removed[:n].copy(), int(sweeps.value)


def localize(reads, contigs, k: int) -> np.ndarray:
    """Read order grouped by the contig (index into ``contigs``, list of
    str) holding each read's first k-mer found in a contig; reads without
    one last.  Returns read indices (int64)."""
    lib = _load()
    seq = np.ascontiguousarray(reads.seq, dtype=np.uint8)
    off = np.ascontiguousarray(reads.offsets, dtype=np.int64)
    n = int(off.shape[0] - 1)
    raw = "".join(contigs).encode()
    cseq = np.frombuffer(raw, dtype=np.uint8).copy() if raw else np.zeros(1, np.uint8)
    coff = np.zeros(len(contigs) + 1, np.int64)
    np.cumsum([len(c) for c in contigs], out=coff[1:])
    order = np.zeros(max(n, 1), np.int64)
    rc = lib.oracle_localize(seq.ctypes.data if len(seq) else None, off.ctypes.data, n, k,
                             cseq.ctypes.data, coff.ctypes.data, len(contigs),
                             order.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_localize failed (%d)" % rc)
    return order[:n].copy()
