#!/usr/bin/env python3
"""Benchmark: canonical k-mers counted per second on one MI355X.

Workload (default): the synthetic metagenome read set -- 100 random genomes of
2-5 Mbp (GC ~ U(0.3, 0.7), log-normal(0, 1.5) abundances), 10M paired 150 bp
reads with 0.5 % substitutions and Phred qualities -- counted at
k = 21, 33, 55, 77, 99 in one batched call (Bloom singleton screen, count
threshold 2, extension quality cutoff 20).  One step is one full pass of the
hot path over the resident reads: pack, Bloom pass, counting pass, classify,
sort and gather, for every k.  ``value`` = valid windows (k-mer occurrences)
over all k per second of step time.

Also reported:
  roofline      the counting pass (the dominant kernel): algorithmic bytes per
                window x windows / its HIP-event duration, against 8 TB/s
  cpu_baseline  the CPU oracle on the host's cores: each of nproc threads owns
                one hash shard of the k-mer space and scans every read of a
                bounded sample (k = 21); single-thread figures beside it
  plain         the same work as five separate single-k calls
  small_k21     the small single-genome read set (6,667 reads) at k = 21
                without the Bloom screen: microseconds per call
  single_k21    the metagenome at k = 21 alone (one kh_count call)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
# DRAM bytes moved per random access to a table slot or Bloom word: one
# 128-byte line.  Measured with the roofline microbenchmark under rocprofv3's
# request-size counters: 2^28 random 8-byte reads over a 32 GiB buffer issue
# 2^28 L2-to-memory read requests, none of them a 32- or 64-byte request (so
# each is a 128-byte one, the size a streaming copy's reads use too).
GRANULE_BYTES = 128
# Memory-side 64-bit atomic adds over an 8 GiB buffer at hashed addresses:
# the rate the roofline microbenchmark measures on MI355X (no published
# figure exists); the counting pass's table is of that size class.
ATOMIC_CEILING = 1.748e10
# Memory-side 64-bit atomic adds at hashed addresses over buffers up to
# 256 MB (the small read set's table is of that size class): measured.
ATOMIC_CEILING_SMALL = 2.37e10
KS = (21, 33, 55, 77, 99)
TUNING_CACHE = os.path.join(ROOT, "paper_1809_07014_amd", "tuning_cache.txt")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "count_pass_traffic.txt")
REQUESTS_FILE = os.path.join(ROOT, "profiles", "count_pass_requests.txt")
OWNER_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "owner_pass_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1809_07014_amd", "csrc", f)
                  for f in ("kh_kernels.hip", "kh_device.hpp")]
OWNER_SOURCES = [os.path.join(ROOT, "paper_1809_07014_amd", "csrc", f)
                 for f in ("kh_owner.hip", "kh_device.hpp")]


def record_words(k: int) -> int:
    """Words of a routed record of the owner-partitioned count: the key
    without its level-1 digit (the top min(10, 2k) bits, which the record's
    bucket implies), shifted left by 6 bits over the extension byte."""
    return (2 * k - min(10, 2 * k) + 6 + 63) // 64


def row_bytes(k: int) -> int:
    """Bytes of one exported row: key words, count, eight tallies, codes."""
    return 8 * ((k + 31) // 32) + 4 + 32 + 2


def stream_bytes_per_window(read_len: int, k: int) -> float:
    """Read bytes the method streams per window in one pass: a 2-bit base and
    a high-quality bit per base (3 bits), spread over the read's windows."""
    return (3.0 / 8.0) * read_len / (read_len - k + 1)


def kernel_source_hash(sources=None) -> str:
    import hashlib
    h = hashlib.sha1()
    for f in sources or KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(ks, path=TRAFFIC_FILE, sources=None):
    """(HBM bytes per step of the dominant kernel's launches, tuning they were
    taken under) from the committed rocprofv3 counter runs, or (None, None)
    if the kernels changed since."""
    if not os.path.exists(path):
        return None, None
    vals = {}
    with open(path) as f:
        for line in f:
            t = line.split()
            if len(t) >= 2 and not t[0].startswith("#"):
                vals[t[0]] = t[1:]
    if vals.get("source_sha1", [""])[0] != kernel_source_hash(sources):
        return None, None
    ff, wf = float(vals["fetch_factor"][0]), float(vals["write_factor"][0])
    total = 0.0
    for k in ks:
        key = "k%d" % k
        if key not in vals:
            return None, None
        fetch_kib, write_kib = float(vals[key][0]), float(vals[key][1])
        total += (fetch_kib * ff + write_kib * wf) * 1024.0
    return total, vals.get("tuning", [None])[0]


def _counter_file(path):
    """Fields of a committed counter file, or None if it is missing or the
    kernels changed since it was taken."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            t = line.split()
            if len(t) >= 2 and not t[0].startswith("#"):
                vals[t[0]] = t[1:]
    if vals.get("source_sha1", [""])[0] != kernel_source_hash():
        return None
    return vals


def measured_requests(ks):
    """Memory requests of the counting-pass launches per step, by size, from
    the committed rocprofv3 request counters: (read bytes, write bytes,
    fraction of reads that are 128-byte requests, atomic requests, tuning),
    or None if the kernels changed since."""
    vals = _counter_file(REQUESTS_FILE)
    if vals is None:
        return None
    rd = wr = rd128 = rdn = atom = 0.0
    for k in ks:
        key = "k%d" % k
        if key not in vals:
            return None
        r, r32, r64, w, w64, a = (float(x) for x in vals[key][:6])
        rd += 32 * r32 + 64 * r64 + 128 * (r - r32 - r64)
        rd128 += r - r32 - r64
        rdn += r
        wr += 64 * w64 + 32 * (w - w64)  # atomics and other sub-64-byte writes: 32 B
        atom += a
    return rd, wr, rd128 / max(rdn, 1.0), atom, vals.get("tuning", [None])[0]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=float, default=1.0,
                    help="fraction of the read set (1.0 = 10M reads)")
    ap.add_argument("--ks", type=str, default=",".join(map(str, KS)))
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-reads", type=int, default=1_000_000,
                    help="reads of the metagenome in the sharded CPU-oracle sample")
    ap.add_argument("--cpu-single-reads", type=int, default=100_000,
                    help="reads of the metagenome in the single-thread oracle sample")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the small read set and single-k legs")
    ap.add_argument("--small-calls", type=int, default=50)
    ap.add_argument("--tuning-cache", type=str, default=TUNING_CACHE,
                    help="stored autotuner choices (kh_autotune_cached)")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner even if the cache holds this case")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-traverse", action="store_true",
                    help="skip the contig leg (merge, traversal, pruning per k)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (library default tuning)")
    ap.add_argument("--tuning", type=str, default="",
                    help="fixed tuning instead of the autotuner, e.g. "
                         "load_factor=0.4,bloom_bits=2,count_lanes=2,tiles_per_block=4")
    ap.add_argument("--tune-reps", type=int, default=2,
                    help="timed calls per setting in the autotuner (best of)")
    ap.add_argument("--serving-samples", type=int, default=64)
    ap.add_argument("--serving-genome-scale", type=float, default=1.0,
                    help="genome lengths relative to the metagenome's (2-5 Mbp)")
    ap.add_argument("--serving-reads-per-genome", type=int, default=100_000)
    ap.add_argument("--serving-loads", type=str, default="0.5,0.7,0.9",
                    help="offered loads, as fractions of the plain path's capacity")
    return ap.parse_args()


SERVING_KS = (21, 33, 55)


def serving_leg(args, kh, synth, np):
    """Serving workload: samples of U{5..40} genomes (lengths scaled by
    --serving-genome-scale), reads_per_genome x #genomes paired reads each;
    each sample's reads arrive as batches of log-uniform[1e4, 5e6] reads
    (capped by what is left of the sample), the samples one after another,
    on one Poisson stream; k = 21, 33, 55 with per-sample resident tables.
    A client thread waits for the batches in arrival order and finalizes
    each sample as soon as its last batch has completed, so finished
    samples leave the device.  Capacity is measured closed-loop (every batch
    submitted at once); the open-loop runs replay one arrival pattern, scaled
    to each offered load of --serving-loads (a fraction of the plain path's
    capacity), against continuous batching and plain FIFO."""
    import threading
    import time as _t
    rng = np.random.default_rng(1809)
    specs = synth.serving_samples(args.serving_samples,
                                  reads_per_genome=args.serving_reads_per_genome,
                                  scale=1.0)
    batches = []
    total_reads = 0
    for spec in specs:
        spec = dict(spec)
        spec["lengths"] = np.maximum(
            5000, (spec["lengths"] * args.serving_genome_scale).astype(np.int64))
        r = synth.sample_reads(spec)
        total_reads += r.n_reads
        i = 0
        while i < r.n_reads:
            n = int(np.exp(rng.uniform(np.log(1e4), np.log(5e6))))
            batches.append((spec["sample"], r.slice(i, min(r.n_reads, i + n))))
            i += n
    last = {smp: j for j, (smp, _) in enumerate(batches)}
    mean_batch = total_reads / len(batches)

    def run(plain, arrivals):
        srv = kh.Server(SERVING_KS, plain=plain, max_active=16)
        n = len(batches)
        tickets, sub_at, lat = [None] * n, [0.0] * n, [0.0] * n
        ready = threading.Semaphore(0)
        fin = []
        errors = []

        def finalize_some(pending):
            """Finalize what the server can; a sample it refuses for room
            (KH_ENOMEM: other samples hold the memory) is tried again later."""
            left = []
            for smp in pending:
                tf = _t.perf_counter()
                try:
                    tabs = srv.finalize(smp)
                except kh.KHError as ex:
                    if ex.code != kh.KH_ENOMEM:
                        raise
                    left.append(smp)
                    continue
                for t in tabs:
                    t.free()
                fin.append(_t.perf_counter() - tf)
            return left

        def client():
            try:
                pending = []
                for j, (smp, _) in enumerate(batches):
                    ready.acquire()
                    lat[j] = srv.wait(tickets[j]) / 1e3
                    if last[smp] == j:
                        pending.append(smp)
                    if pending:
                        pending = finalize_some(pending)
                while pending:
                    left = finalize_some(pending)
                    if len(left) == len(pending):
                        raise RuntimeError("samples %s cannot be finalized" % left)
                    pending = left
            except Exception as ex:  # reported after the run
                errors.append(ex)

        th = threading.Thread(target=client)
        th.start()
        t0 = _t.perf_counter()
        for j, ((smp, b), at) in enumerate(zip(batches, arrivals)):
            now = _t.perf_counter() - t0
            if at > now:
                _t.sleep(at - now)
            sub_at[j] = _t.perf_counter() - t0
            tickets[j] = srv.submit(smp, b)
            ready.release()
        th.join()
        if errors:
            raise errors[0]
        span = max(sa + l for sa, l in zip(sub_at, lat))
        st = srv.stats()
        srv.close()
        lat_ms = np.array(lat) * 1e3
        return dict(windows_per_s=round(st["windows"] / span, 1),
                    reads_per_s=round(total_reads / span, 1),
                    p50_ms=round(float(np.percentile(lat_ms, 50)), 3),
                    p99_ms=round(float(np.percentile(lat_ms, 99)), 3),
                    makespan_s=round(span, 4), launches=int(st["launches"]),
                    max_active=int(st["max_active"]),
                    finalize_ms_mean=round(1e3 * float(np.mean(fin)), 2),
                    replayed=int(st["replayed"]), rehashes=int(st["rehashes"]),
                    retried=int(st["retried"]), grow_s=round(st["grow_s"], 4),
                    alloc_s=round(st["alloc_s"], 4),
                    peak_gb=round(st["peak_bytes"] / 1e9, 1))

    def note(what, r):
        print("# serving %s: %.3e windows/s, p50/p99 %.1f/%.1f ms, %.1f s" %
              (what, r["windows_per_s"], r["p50_ms"], r["p99_ms"], r["makespan_s"]),
              file=sys.stderr, flush=True)

    closed = [0.0] * len(batches)
    plain_cap = run(True, closed)
    note("plain capacity", plain_cap)
    batched_cap = run(False, closed)
    note("batched capacity", batched_cap)
    gaps = rng.exponential(1.0, size=len(batches))  # one arrival pattern, scaled per load
    loads = {}
    for rho in [float(x) for x in args.serving_loads.split(",")]:
        lam = rho * plain_cap["reads_per_s"] / mean_batch  # batches / s
        arrivals = np.cumsum(gaps / lam)
        arrivals -= arrivals[0]
        b = run(False, list(arrivals))
        note("batched at %.0f%%" % (100 * rho), b)
        p = run(True, list(arrivals))
        note("plain at %.0f%%" % (100 * rho), p)
        loads["%.2f" % rho] = dict(batched=b, plain=p)
    return dict(workload="serving: %d samples of 5-40 genomes (%.2g x 2-5 Mbp), %d batches, "
                         "%d reads, k=21,33,55, Poisson arrivals"
                         % (len(specs), args.serving_genome_scale, len(batches), total_reads),
                plain_capacity=plain_cap, batched_capacity=batched_cap,
                capacity_ratio=round(batched_cap["windows_per_s"] /
                                     plain_cap["windows_per_s"], 3),
                loads=loads)


def small_leg(args, kh, ctx, synth, torch, stream):
    """kh_count at k = 21 without the Bloom screen on the small read set
    (resident on the device): microseconds per call (pack, count, classify,
    sort, gather and the table's release) and the counting pass's atomics
    against the memory-side rate measured for tables of its size class."""
    r1 = synth.config(1)
    d1 = kh.DeviceReads.from_host(r1, "cuda:0")
    for _ in range(5):
        ctx.count(d1, 21, stream=stream).free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.small_calls):
        ctx.count(d1, 21, stream=stream).free()
    torch.cuda.synchronize()
    call_s = (time.perf_counter() - t0) / args.small_calls
    ms, st = ctx.k_report(0)
    out = dict(workload="one 50 kbp genome, 6,667 single-end 150 bp reads, k=21, no Bloom",
               windows=st["windows"], rows=st["rows"], calls=args.small_calls,
               us_per_call=round(call_s * 1e6, 1),
               value=round(st["windows"] / call_s, 1), unit="windows/s",
               count_us=round(ms["count"] * 1e3, 1),
               phases_us={p: round(v * 1e3, 1) for p, v in ms.items()})
    if not ctx.tuning().get("partitioned", 0):  # device-scope atomics of the table
        atomics = st["passed"] + st["claimed"]
        out.update(count_atomics_per_s=round(atomics / (ms["count"] * 1e-3), 1),
                   atomic_ceiling=ATOMIC_CEILING_SMALL,
                   atomic_frac=round(atomics / (ms["count"] * 1e-3) / ATOMIC_CEILING_SMALL, 4))
    return out


def single_k_leg(kh, ctx, dev, torch, stream, read_len, opts, calls=3):
    """kh_count at k = 21 with the Bloom screen on the metagenome (one k,
    the plain path): windows/s and its counting pass against the HBM model."""
    ctx.count(dev, 21, stream=stream, **opts).free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    count_ms = 0.0
    for _ in range(calls):
        ctx.count(dev, 21, stream=stream, **opts).free()
        ms, st = ctx.k_report(0)
        count_ms += ms["count"]
    torch.cuda.synchronize()
    call_s = (time.perf_counter() - t0) / calls
    count_ms /= calls
    if ctx.tuning().get("partitioned", 0):  # owner pass: records in, rows out
        alg = st["windows"] * 8 * record_words(21) + st["rows"] * row_bytes(21)
    else:
        alg = (st["windows"] * (stream_bytes_per_window(read_len, 21) + 1 / 8)
               + st["bloom_l1_new"] * GRANULE_BYTES + st["passed"] * 2 * GRANULE_BYTES)
    gbs = alg / (count_ms * 1e-3) / 1e9
    return dict(workload="metagenome 10M reads, k=21, Bloom", windows=st["windows"],
                rows=st["rows"], ms=round(call_s * 1e3, 2),
                value=round(st["windows"] / call_s, 1), unit="windows/s",
                phases_ms={p: round(v, 3) for p, v in ms.items()},
                count_ms=round(count_ms, 3), count_GBps=round(gbs, 1),
                count_frac=round(gbs / HBM_PEAK_GBS, 4))


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(args, reads, synth):
    """The CPU oracle on the host's cores, k = 21.  Sharded: each of nproc
    threads owns one shard of the k-mer space (the oracle's own partition
    function) and scans every read of the sample, keeping its shard's k-mers
    (oracle_count_shard, one OpenMP thread per call; the C code runs without
    the interpreter lock).  Single thread: oracle_count on the whole small
    read set and on the first reads of the metagenome."""
    import concurrent.futures as cf
    import oracle
    nproc = os.cpu_count() or 1
    sample = reads.slice(0, min(args.cpu_reads, reads.n_reads))

    def shard(s):
        oracle.set_threads(1)  # one thread per shard
        return oracle.count_shard(sample, 21, nproc, s)

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(nproc) as ex:
        tabs = list(ex.map(shard, range(nproc)))
    par_s = time.perf_counter() - t0
    windows = sum(t["n_windows"] for t in tabs)
    rows = sum(t["n_rows"] for t in tabs)
    single = {}
    for name, rs in (("small read set (6,667 reads)", synth.config(1)),
                     ("first %d reads of the metagenome" % args.cpu_single_reads,
                      reads.slice(0, min(args.cpu_single_reads, reads.n_reads)))):
        t1 = time.perf_counter()
        w = oracle.count(rs, 21)["n_windows"]
        dt = time.perf_counter() - t1
        single[name] = dict(windows=w, s=round(dt, 2), value=round(w / dt, 1))
    return dict(value=round(windows / par_s, 1), unit="windows/s", cores=nproc,
                kind="oracle",
                sample="first %d reads of the metagenome, k=21, %d shards on %d threads, "
                       "%d rows, %.1f s" % (sample.n_reads, nproc, nproc, rows, par_s),
                cpu_model=_cpu_model(), single_thread=single)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(it would shard k-mers by hash owner across GPUs); run with "
              "--gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_1809_07014_amd as kh

    ks = [int(x) for x in args.ks.split(",")]
    t0 = time.time()
    reads = synth.config(2, scale=args.scale)
    read_len = 150
    print("# generated %d reads (%d bases) in %.1fs" %
          (reads.n_reads, reads.n_bases, time.time() - t0), file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    ctx = kh.Context(0)
    dev = kh.DeviceReads.from_host(reads, "cuda:0")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    opts = dict(use_bloom=True, min_count=2, qual_cutoff=20)

    # ---- autotuner (outside the timed region): the context keeps its choice
    if args.tuning:
        ctx.set_tuning(**{k: (float(v) if k == "load_factor" else int(v))
                          for k, v in (x.split("=") for x in args.tuning.split(","))})
    tuning = dict(ctx.tuning(), autotuned=False)
    if not args.no_tune and not args.tuning:
        tt = time.perf_counter()
        if args.retune:  # tune afresh; the choice is appended to the cache (last wins)
            fresh = args.tuning_cache + ".retune"
            if os.path.exists(fresh):
                os.remove(fresh)
            tuned, rep, hit = ctx.autotune_cached(dev, ks, fresh, stream=stream,
                                                  reps=args.tune_reps, **opts)
            with open(fresh) as f, open(args.tuning_cache, "a") as g:
                g.write(f.read())
            os.remove(fresh)
        else:
            tuned, rep, hit = ctx.autotune_cached(dev, ks, args.tuning_cache, stream=stream,
                                                  reps=args.tune_reps, **opts)
        tuning = dict(tuned, autotuned=True, cached=hit,
                      autotune_s=round(time.perf_counter() - tt, 2),
                      trials=rep["trials"], start_ms=round(rep["start_ms"], 2),
                      best_ms=round(rep["best_ms"], 2))
        print("# tuning %s in %.1fs: %s" % ("from the cache" if hit else "autotuned",
                                            tuning["autotune_s"], tuned),
              file=sys.stderr, flush=True)

    def step():
        tabs = ctx.count_multi_k(dev, ks, stream=stream, **opts)
        info = [t.info() for t in tabs]
        for t in tabs:
            t.free()
        return info

    ctx.set_timing(True)
    for _ in range(args.warmup):
        step()
        print("# warmup step done", file=sys.stderr, flush=True)

    owned = bool(ctx.tuning().get("partitioned", 0))
    phases = {p: 0.0 for p in kh.PHASES}
    count_ms = {k: 0.0 for k in ks}
    alg = {k: 0.0 for k in ks}
    pipe = {k: 0.0 for k in ks}
    passed = {k: 0 for k in ks}
    atomics = {k: 0 for k in ks}
    sightings = {k: (0, 0) for k in ks}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    infos = None
    for i in range(args.steps):
        infos = step()
        for p, v in ctx.timing().items():
            phases[p] += v
        for j, k in enumerate(ks):
            ms, st = ctx.k_report(j)
            count_ms[k] += ms["count"]
            passed[k] = st["passed"]
            sightings[k] = (st["bloom_l1_new"], st["bloom_l2_new"])
            # returning atomics of the counting pass: one add per counted
            # window, one compare-and-swap per stored key word of a claimed
            # slot (62-bit words: ceil(k / 31) per key)
            atomics[k] += st["passed"] + st["claimed"] * ((k + 30) // 31)
            if owned:
                # owner pass: every routed record read once, every kept row
                # written once to its staging slot
                alg[k] += (st["windows"] * 8 * record_words(k)
                           + infos[j]["n_rows"] * row_bytes(k))
                # the whole owner-partitioned count: a record is written by
                # the level-1 emit, read by the level-2 histogram, read and
                # written by the level-2 scatter and read by the owner pass;
                # a row is written to staging, then read and written by the
                # copy into the table
                pipe[k] += (st["windows"] * 40 * record_words(k)
                            + infos[j]["n_rows"] * 3 * row_bytes(k))
            else:
                # counting-pass algorithmic bytes: the read stream and its
                # sighting bits, one Bloom word per window that was its key's
                # first sighting in pass A (the others skip the filter), one
                # slot read-modify-write per counted window
                alg[k] += (st["windows"] * (stream_bytes_per_window(read_len, k) + 1 / 8)
                           + st["bloom_l1_new"] * GRANULE_BYTES
                           + st["passed"] * 2 * GRANULE_BYTES)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    windows = sum(x["n_windows"] for x in infos)
    value = windows * args.steps / elapsed
    for p in phases:
        phases[p] /= args.steps
    print("# timed %d steps: %.1f ms/step, %.3e windows/s" %
          (args.steps, ms_per_step, value), file=sys.stderr, flush=True)

    # ---- roofline of the dominant kernel: the counting pass (single-table
    # path) or the owner pass (owner-partitioned path), one launch per k
    alg_step = sum(alg.values()) / args.steps
    count_step_s = sum(count_ms.values()) / args.steps * 1e-3
    achieved = alg_step / count_step_s / 1e9
    if owned:
        traffic, traffic_tuning = measured_traffic(ks, OWNER_TRAFFIC_FILE, OWNER_SOURCES)
    else:
        traffic, traffic_tuning = measured_traffic(ks)
    req = None if owned else measured_requests(ks)
    requests = None
    if req is not None:
        rd, wr, f128, atom, req_tuning = req
        requests = dict(read_GB=round(rd / 1e9, 2), write_GB=round(wr / 1e9, 2),
                        read_128B_fraction=round(f128, 4), atomic_requests=atom,
                        achieved=round((rd + wr) / count_step_s / 1e9, 1),
                        frac=round((rd + wr) / count_step_s / 1e9 / HBM_PEAK_GBS, 4),
                        tuning=req_tuning,
                        note="L2-to-memory requests of the counting passes at their "
                             "counted sizes (profiles/count_pass_requests.txt); "
                             "memory-side atomics' line write-backs are not seen")
    roofline = dict(bound="hbm", kernel="k_windows<W,2> counting pass, one launch per k",
                    achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=None if traffic is None else round(traffic / 1e9, 2),
                    traffic_unit="GB per step (five launches)",
                    traffic_tuning=traffic_tuning,
                    alg_bytes=round(alg_step / 1e9, 2),
                    requests=requests,
                    launch_ms_avg=round(count_step_s * 1e3 / len(ks), 3),
                    atomic=dict(achieved=round(sum(atomics.values()) / args.steps
                                               / count_step_s, 1),
                                ceiling=ATOMIC_CEILING, unit="atomics/s",
                                frac=round(sum(atomics.values()) / args.steps / count_step_s
                                           / ATOMIC_CEILING, 4),
                                source="measured: 64-bit atomic add at hashed addresses "
                                       "over 8 GiB (profiles/roofline_microbench.txt)"),
                    model="per window: 3/8 B/base x L/(L-k+1) read stream + 1/8 B "
                          "sighting bit + f_1 x G (Bloom word, first sightings only) + "
                          "f_s x 2G (slot read-modify-write), G = %d B (the request size "
                          "of a random 8-byte read, measured)" % GRANULE_BYTES)
    if owned:
        pipe_s = sum(phases[p] for p in ("bloom", "count", "classify", "sort", "gather")) * 1e-3
        pipe_step = sum(pipe.values()) / args.steps
        roofline = dict(
            bound="hbm",
            kernel="k_own_count owner pass (Bloom pass A, count pass B, classify in "
                   "LDS), one launch per k",
            achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
            frac=round(achieved / HBM_PEAK_GBS, 4),
            traffic=None if traffic is None else round(traffic / 1e9, 2),
            traffic_unit="GB per step (five launches)",
            traffic_tuning=traffic_tuning,
            alg_bytes=round(alg_step / 1e9, 2),
            launch_ms_avg=round(count_step_s * 1e3 / len(ks), 3),
            model="per k: every routed record (8 x ceil((2k - 10 + 6) / 64) bytes) read once, "
                  "every kept row (key words, count, 8 tallies, codes) written once",
            pipeline=dict(
                what="the whole owner-partitioned count: level-1 histogram and emit, "
                     "level-2 histogram and scatter, owner pass, row copy",
                alg_bytes=round(pipe_step / 1e9, 2), ms=round(pipe_s * 1e3, 2),
                achieved=round(pipe_step / pipe_s / 1e9, 1),
                frac=round(pipe_step / pipe_s / 1e9 / HBM_PEAK_GBS, 4),
                model="per record 40 x ceil((2k - 10 + 6) / 64) bytes (written, read, read and "
                      "written, read), per kept row 3 x its bytes"))
    per_k = {}
    for k, inf in zip(ks, infos):
        per_k[str(k)] = dict(windows=inf["n_windows"], rows=inf["n_rows"],
                             pass_fraction=round(passed[k] / max(1, inf["n_windows"]), 4),
                             bloom_first_sightings=sightings[k][0],
                             bloom_second_sightings=sightings[k][1],
                             count_ms=round(count_ms[k] / args.steps, 3),
                             count_atomics_per_s=None if owned else
                             round(atomics[k] / (count_ms[k] * 1e-3), 1),
                             count_GBps=round(alg[k] / (count_ms[k] * 1e-3) / 1e9, 1))

    # ---- the same work as separate single-k calls
    plain = None
    if not args.no_plain:
        torch.cuda.synchronize()
        tp = time.perf_counter()
        plain_phases = {p: 0.0 for p in kh.PHASES}
        for k in ks:
            ctx.count(dev, k, stream=stream, **opts).free()
            for p, v in ctx.timing().items():
                plain_phases[p] += v
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - tp
        # phases of the single-k calls run one after another (no overlap)
        plain = dict(value=round(windows / plain_s, 1), ms=round(plain_s * 1e3, 2),
                     phases_ms={p: round(v, 3) for p, v in plain_phases.items()})

    # ---- the single-table path's batched call (one device hash table per k,
    # fused Bloom launches, graph-replayed counting passes, tails beside
    # them), which the owner-partitioned count replaces by default
    single_table = None
    if owned and not args.no_plain:
        keep = ctx.tuning()
        ctx.set_tuning(partitioned=0, load_factor=0.4)
        for t in ctx.count_multi_k(dev, ks, stream=stream, **opts):  # warm-up
            t.free()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(2):
            for t in ctx.count_multi_k(dev, ks, stream=stream, **opts):
                t.free()
        torch.cuda.synchronize()
        st_s = (time.perf_counter() - ts) / 2
        single_table = dict(value=round(windows / st_s, 1), ms=round(st_s * 1e3, 2),
                            graphed=ctx.last_graphed(),
                            tuning="partitioned=0, load_factor=0.4, other fields as the "
                                   "default tuning")
        ctx.set_tuning(**keep)
        print("# single-table batched call: %.1f ms" % (st_s * 1e3), file=sys.stderr,
              flush=True)

    # ---- the same batched call from host-resident (pageable) reads: the
    # PCIe copy of bases, qualities and offsets is inside the time; the copy
    # alone is timed beside it (never the headline value)
    end_to_end = None
    if not args.no_plain:
        torch.cuda.synchronize()
        th = time.perf_counter()
        for t in ctx.count_multi_k(reads, ks, stream=stream, **opts):
            t.free()
        torch.cuda.synchronize()
        e2e_s = time.perf_counter() - th
        th = time.perf_counter()
        copies = [torch.from_numpy(a).to("cuda:0") for a in (reads.seq, reads.qual, reads.offsets)]
        torch.cuda.synchronize()
        h2d_s = time.perf_counter() - th
        del copies
        end_to_end = dict(value=round(windows / e2e_s, 1), ms=round(e2e_s * 1e3, 2),
                          h2d_ms=round(h2d_s * 1e3, 2),
                          h2d_GBps=round((reads.seq.nbytes + reads.qual.nbytes
                                          + reads.offsets.nbytes) / h2d_s / 1e9, 2),
                          source="pageable host arrays")

    # ---- Algorithm 1's in-scope steps over the k of the step: the k-mer
    # table of each k, merged with the pruned contigs of the previous k,
    # traversed into contigs, pruned (Algorithm 2)
    traversal = None
    if not args.no_traverse:
        from paper_1809_07014_amd import pipeline
        ctx.trim()  # the timed steps' cached tables give the device back
        # run twice and report the second: the first pays for the device
        # memory the pool takes back from the driver after the trim
        for _ in range(2):
            last, reps = pipeline.iterate(ctx, dev, ks, stream=stream, **opts)
            last.free()
        traversal = {}
        for r in reps:
            n_all = r["rows"] + r["merged_rows"]
            traversal[str(r["k"])] = dict(
                rows=r["rows"], merged_rows=r["merged_rows"], merge_ms=round(r["merge_ms"], 2),
                contigs=r["n_contigs"], bases=r["total_bases"], ms=round(r["traverse_ms"], 2),
                rows_per_s=round(n_all / (r["traverse_ms"] / 1e3), 1), rounds=r["rounds"],
                cycle_kmers=r["cycle_kmers"], prune_ms=round(r["prune_ms"], 2),
                pruned=r["pruned"], sweeps=r["sweeps"], kept=r["kept_contigs"], n50=r["n50"],
                longest=r["longest"])
        print("# contigs: %s" % ", ".join(
            "k=%s traverse %.0f ms prune %.0f ms merge %.0f ms n50 %d" % (
                k, v["ms"], v["prune_ms"], v["merge_ms"], v["n50"])
            for k, v in traversal.items()), file=sys.stderr, flush=True)

    # ---- read localisation (Section II): the reads grouped by the first k's
    # contigs, then the other k counted from both read orders
    localized = None
    if not args.no_traverse and len(ks) > 1:
        t0k = ctx.count(dev, ks[0], stream=stream, **opts)
        c0 = ctx.traverse(t0k, stream=stream)
        torch.cuda.synchronize()
        tl = time.perf_counter()
        moved = ctx.localize(t0k, c0, dev, stream=stream)
        torch.cuda.synchronize()
        loc_ms = (time.perf_counter() - tl) * 1e3
        c0.free()
        t0k.free()

        def multi(rs):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for x in ctx.count_multi_k(rs, ks[1:], stream=stream, **opts):
                x.free()
            torch.cuda.synchronize()
            return (time.perf_counter() - t1) * 1e3

        ms = [multi(dev), multi(moved), multi(dev), multi(moved)]
        localized = dict(ks=ks[1:], localize_ms=round(loc_ms, 2),
                         input_order_ms=round(min(ms[0], ms[2]), 2),
                         localized_ms=round(min(ms[1], ms[3]), 2))
        del moved
        print("# localised reads: %.0f ms to order and gather; k=%s counted in %.0f ms "
              "(input order %.0f ms)" % (loc_ms, ",".join(map(str, ks[1:])),
                                         localized["localized_ms"],
                                         localized["input_order_ms"]),
              file=sys.stderr, flush=True)

    # ---- the small read set (one 50 kbp genome, 6,667 reads) at k = 21
    # without the Bloom screen, and the metagenome at k = 21 alone
    small = single = None
    if not args.no_small:
        small = small_leg(args, kh, ctx, synth, torch, stream)
        single = single_k_leg(kh, ctx, dev, torch, stream, read_len, opts)
        print("# small read set: %.1f us per call; metagenome k=21 alone: %.1f ms, "
              "%.3e windows/s" % (small["us_per_call"], single["ms"], single["value"]),
              file=sys.stderr, flush=True)

    # ---- CPU oracle on bounded samples of the read set
    cpu = None
    if not args.no_cpu:
        cpu = cpu_leg(args, reads, synth)
        print("# cpu oracle: %.3e windows/s on %d threads (%s)" %
              (cpu["value"], cpu["cores"], cpu["sample"]), file=sys.stderr, flush=True)

    # the serving leg starts from a clean device: this context's cached
    # blocks (tables of the runs above) go back to the driver first
    dev = None
    torch.cuda.empty_cache()
    ctx.close()
    kh.release_cached(0)
    serving = None
    if not args.no_serving:
        serving = serving_leg(args, kh, synth, np)

    out = dict(
        metric="canonical k-mers counted/sec (k=21..99)",
        value=round(value, 1), unit="windows/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(ms_per_step, 3),
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype="u64",
        data="synthetic",
        config=dict(workload="metagenome-10M-reads-batched-k",
                    reads=reads.n_reads, read_len=read_len, ks=ks,
                    genomes=100, bloom=True, min_count=2, qual_cutoff=20,
                    scale=args.scale),
        roofline=roofline, cpu_baseline=cpu, plain_sequential=plain,
        batched_over_plain=None if plain is None else round(value / plain["value"], 3),
        single_table_batched=single_table,
        over_single_table=None if single_table is None
        else round(value / single_table["value"], 3),
        small_k21=small, single_k21=single,
        end_to_end_host_reads=end_to_end, tuning=tuning,
        traversal=traversal, localized=localized,
        serving=serving,
        phases_ms={p: round(v, 3) for p, v in phases.items()}, per_k=per_k)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
