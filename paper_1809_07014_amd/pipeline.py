"""Iterative contig generation, the steps of the paper's Algorithm 1 that
this library covers: for each k in increasing order, k-mer analysis of the
reads (Section II-B), merge of the previous k's contigs into that table
(Algorithm 1's Merge), and de Bruijn graph traversal into contigs (Section
II-C).  Bubble merging, pruning, alignment and local assembly, which the
paper runs between traversal and the next k, are not part of it: the
contigs of one k go straight into the next k's table.

Command line (synthetic reads; one line per k with the time of each step):

    python paper_1809_07014_amd/pipeline.py --workload metagenome --ks 21,33,55
"""
from __future__ import annotations

import argparse
import sys
import time


def iterate(ctx, reads, ks, stream=None, use_bloom=True, on_step=None, **params):
    """Run the steps for every k of ``ks`` (increasing).  Returns the last k's
    Contigs (the caller frees it) and a list of per-k reports.  ``on_step``,
    if given, is called with each report as soon as its k is done."""
    import torch

    reports, prev = [], None
    tabs = ctx.count_multi_k(reads, ks, stream=stream, use_bloom=use_bloom, **params)
    try:
        for i, (k, t) in enumerate(zip(ks, tabs)):
            rep = dict(k=k, rows=t.info()["n_rows"], merged_rows=0, merge_ms=0.0)
            if prev is not None:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                merged = ctx.merge_contigs(t, prev, stream=stream)
                torch.cuda.synchronize()
                rep["merge_ms"] = (time.perf_counter() - t0) * 1e3
                rep["merged_rows"] = merged.info()["n_rows"] - rep["rows"]
                t.free()
                tabs[i] = t = merged
                prev.free()
                prev = None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            prev = ctx.traverse(t, stream=stream)
            torch.cuda.synchronize()
            rep["traverse_ms"] = (time.perf_counter() - t0) * 1e3
            rep.update({x: v for x, v in prev.info().items() if x != "k"})
            t.free()
            reports.append(rep)
            if on_step:
                on_step(rep)
    finally:
        for t in tabs:
            t.free()
    return prev, reports


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", choices=("small", "metagenome"), default="metagenome")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--ks", default="21,33,55,77,99")
    ap.add_argument("--no-bloom", action="store_true")
    ap.add_argument("--repeat", type=int, default=1, help="run the steps this many times")
    args = ap.parse_args(argv)

    import torch  # the library's HIP runtime comes with torch
    import synth
    import paper_1809_07014_amd as kh

    reads = synth.config(1 if args.workload == "small" else 2, scale=args.scale)
    ks = [int(x) for x in args.ks.split(",")]
    ctx = kh.Context(0)
    dev = kh.DeviceReads.from_host(reads, "cuda:0")
    torch.cuda.synchronize()
    for r in range(args.repeat):
        def show(rep, r=r):
            print("run %d k=%d rows=%d merged=%d merge %.1f ms traverse %.1f ms contigs=%d "
                  "bases=%d rounds=%d" % (r, rep["k"], rep["rows"], rep["merged_rows"],
                                          rep["merge_ms"], rep["traverse_ms"], rep["n_contigs"],
                                          rep["total_bases"], rep["rounds"]), flush=True)
        last, _ = iterate(ctx, dev, ks, use_bloom=not args.no_bloom, on_step=show)
        last.free()
    ctx.close()
    return 0


if __name__ == "__main__":  # run as a file: the repository root holds the packages
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    sys.exit(main())
