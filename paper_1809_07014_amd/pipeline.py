"""Iterative contig generation, the steps of the paper's Algorithm 1 that
this library covers: for each k in increasing order, k-mer analysis of the
reads (Section II-B), merge of the previous k's contigs into that table
(Algorithm 1's Merge), de Bruijn graph traversal into contigs (Section
II-C) and iterative graph pruning (Algorithm 2).  Bubble merging, hair
removal, alignment and local assembly, which the paper also runs between
traversal and the next k, are not part of it: the pruned contigs of one k go
straight into the next k's table.

Command line (synthetic reads; one line per k with the time of each step):

    python paper_1809_07014_amd/pipeline.py --workload metagenome --ks 21,33,55
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np


def n50(lengths) -> int:
    """Length L such that contigs of length >= L hold half of all bases."""
    lens = np.sort(np.asarray(lengths))[::-1]
    if not len(lens):
        return 0
    return int(lens[np.searchsorted(np.cumsum(lens), lens.sum() / 2)])


def iterate(ctx, reads, ks, stream=None, use_bloom=True, prune=True, alpha=None, beta=None,
            on_step=None, **params):
    """Run the steps for every k of ``ks`` (increasing).  Returns the last k's
    contigs (pruned if ``prune``; the caller frees them) and a list of per-k
    reports.  ``on_step``, if given, is called with each report as soon as
    its k is done."""
    import torch

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) * 1e3

    reports, prev = [], None
    tabs = ctx.count_multi_k(reads, ks, stream=stream, use_bloom=use_bloom, **params)
    try:
        for i, (k, t) in enumerate(zip(ks, tabs)):
            rep = dict(k=k, rows=t.info()["n_rows"], merged_rows=0, merge_ms=0.0)
            if prev is not None:
                merged, rep["merge_ms"] = timed(lambda: ctx.merge_contigs(t, prev, stream=stream))
                rep["merged_rows"] = merged.info()["n_rows"] - rep["rows"]
                t.free()
                tabs[i] = t = merged
                prev.free()
                prev = None
            prev, rep["traverse_ms"] = timed(lambda: ctx.traverse(t, stream=stream))
            rep.update({x: v for x, v in prev.info().items() if x != "k"})
            rep.update(prune_ms=0.0, pruned=0, sweeps=0)
            if prune:
                (kept, pr), rep["prune_ms"] = timed(
                    lambda: ctx.prune(t, prev, alpha=alpha, beta=beta, stream=stream))
                rep.update(pruned=pr["removed"], sweeps=pr["sweeps"])
                prev.free()
                prev = kept
            t.free()
            lens = prev.lengths()
            rep.update(kept_contigs=len(lens), n50=n50(lens),
                       longest=int(lens.max()) if len(lens) else 0)
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
    ap.add_argument("--no-prune", action="store_true", help="skip iterative graph pruning")
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
                  "bases=%d rounds=%d prune %.1f ms pruned=%d sweeps=%d n50=%d" % (
                      r, rep["k"], rep["rows"], rep["merged_rows"], rep["merge_ms"],
                      rep["traverse_ms"], rep["n_contigs"], rep["total_bases"], rep["rounds"],
                      rep["prune_ms"], rep["pruned"], rep["sweeps"], rep["n50"]), flush=True)
        last, _ = iterate(ctx, dev, ks, use_bloom=not args.no_bloom,
                          prune=not args.no_prune, on_step=show)
        last.free()
    ctx.close()
    return 0


if __name__ == "__main__":  # run as a file: the repository root holds the packages
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    sys.exit(main())
