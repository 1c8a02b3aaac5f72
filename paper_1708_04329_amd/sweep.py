"""Parameter sweeps of the paper's sensitivity study, on synthetic inputs, through the C ABI.

    python -m paper_1708_04329_amd.sweep [--genome-len G] [--reads N] [--json PATH]

Two studies (paper Section 6.1), both on the 3.1 Gbp synthetic reference with
45% interspersed repeats and 100 bp reads whose error rates are spread over
0..5 %:

* read existence: the share of all bins that pass the filter, i.e. would go on
  to alignment, for token lengths q = 4, 5, 6, bin counts N x 64k (N = 100,
  200, 300, 450, so bins of 473 down to 106 bases) and error tolerances
  e = 0..5 % (the read-existence figure: lower is better, zero would mean every
  location is filtered);
* the false-negative rate in the paper's sense: of the candidate locations that
  pass the filter, the share that yields no mapping within E edits (the bins
  parameter sweep figure), with candidates from 12-mer seed hits and mappings
  from verification, beside the same share without the filter.

The sweep drives the library only (index build, all-bins scan, per-read pass
counts, seeding, candidate filter, verification); PyTorch holds the device
buffers and sums the library's per-read counts.
"""

from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import grim


def log(*a):
    print("[sweep]", *a, file=sys.stderr, flush=True)


def existence_study(ref_dev, d_bases, d_offs, n_reads: int, qs, bins, O: int, e_list):
    """Read existence (paper Section 6.1): for each token length q, bin size and
    error tolerance e (per cent), the number of (read, bin) cells that pass the
    all-bins filter, and its share of all cells. ``bins`` is a list of
    (label, bin size) pairs. Pass counts come from grim_mask_summary."""
    import torch
    out = []
    for q in qs:
        for label, B in bins:
            idx = grim.grim_build_index(ref_dev, B, O, q, grim.LAYOUT_TM)
            info = idx.info()
            nb, W = info["n_bins"], info["mask_words"]
            mask = torch.empty((n_reads, W), dtype=torch.uint32, device="cuda")
            passed = torch.empty(n_reads, dtype=torch.uint32, device="cuda")
            for e in e_list:
                grim.grim_filter_scan(idx, grim.ReadSet(d_bases, d_offs, err_permille_all=10 * e), mask)
                grim.grim_mask_summary(mask, pass_count=passed)
                total = int(passed.to(torch.int64).sum().item())
                out.append({"q": q, "bins": label, "n_bins": nb, "bin_size": B, "e_pct": e, "passing_cells": total,
                            "read_existence": total / (n_reads * nb)})
                log(f"q={q} bins={label} (B={B}) e={e}%: read existence {out[-1]['read_existence']:.4g}")
            del mask, passed
            idx.free()
            torch.cuda.empty_cache()
    return out


def fn_study(ref_dev, d_bases, d_offs, n_reads: int, bins, O: int, e_list, cap: int, k: int = 12, q: int = 5):
    """False-negative rate in the paper's sense (Section 6.1, bins sweep): of the
    seed-hit candidate locations (non-overlapping k-mer seeds, at most ``cap``
    bins per read) that pass the filter, the share that does not map within E
    edits; beside it the same share without the filter, and the mapping
    locations the filter dropped (zero by construction)."""
    import torch
    out = []
    seeds = grim.grim_seeds_build(ref_dev, k)
    for label, B in bins:
        idx = grim.grim_build_index(ref_dev, B, O, q, grim.LAYOUT_BM | grim.LAYOUT_REF)
        co = torch.empty(n_reads + 1, dtype=torch.int64, device="cuda")
        cb = torch.empty(max(1, n_reads * cap), dtype=torch.int32, device="cuda")
        P = grim.grim_seed_candidates(seeds, grim.ReadSet(d_bases, d_offs), B, cap, co, cb)
        cbv = cb[:max(P, 1)]
        cnt = torch.empty(max(P, 1), dtype=torch.uint16, device="cuda")
        pas = torch.empty(max(P, 1), dtype=torch.uint8, device="cuda")
        dist = torch.empty(max(P, 1), dtype=torch.uint16, device="cuda")
        match = torch.empty(max(P, 1), dtype=torch.uint8, device="cuda")
        for e in e_list:
            rs = grim.ReadSet(d_bases, d_offs, err_permille_all=10 * e)
            if P:
                grim.grim_filter_candidates(idx, rs, co, cbv[:P], cnt, pas)
                grim.grim_verify_candidates_bounded(idx, rs, co, cbv[:P], None, dist, match)   # every candidate
            torch.cuda.synchronize()
            pv, mv = pas[:P].to(torch.int64), match[:P].to(torch.int64)
            n_pass = int(pv.sum().item())
            n_map = int(mv.sum().item())
            n_pass_map = int((pv & mv).sum().item())
            out.append({"bins": label, "bin_size": B, "e_pct": e, "candidates": P, "passing": n_pass,
                        "mapping": n_map, "passing_and_mapping": n_pass_map,
                        "fn_rate_filter": 1 - n_pass_map / max(1, n_pass),
                        "fn_rate_no_filter": 1 - n_map / max(1, P),
                        "mapping_locations_filtered_out": n_map - n_pass_map})
            log(f"bins={label} e={e}%: {P:,} candidates, {n_pass:,} pass, {n_map:,} map; "
                f"false-negative rate {out[-1]['fn_rate_filter']:.4f} (no filter {out[-1]['fn_rate_no_filter']:.4f})")
        del co, cb, cbv, cnt, pas, dist, match
        idx.free()
        torch.cuda.empty_cache()
    seeds.free()
    return out


def main(argv=None):
    import torch
    import synth
    import synth.configs as C

    p = argparse.ArgumentParser()
    p.add_argument("--genome-len", type=int, default=3_100_000_000)
    p.add_argument("--reads", type=int, default=2000)
    p.add_argument("--bins-64k", default="100,200,300,450")
    p.add_argument("--q", default="4,5,6")
    p.add_argument("--cap", type=int, default=2048, help="seed-hit candidates kept per read")
    p.add_argument("--json", default="")
    args = p.parse_args(argv)

    torch.cuda.set_device(0)
    gspec = C.workload("c3").genome
    if args.genome_len != gspec.length:
        from dataclasses import replace
        gspec = replace(gspec, length=args.genome_len)
    t0 = time.time()
    ref = synth.genome(gspec)
    L, e_max = 100, 5
    rd = synth.reads(sweep_reads_spec(gspec.seed, args.reads, L, e_max), ref)
    log(f"genome {len(ref):,} bp, {rd.n} reads of {L} bp in {time.time() - t0:.1f}s")
    G = len(ref)
    O = L + e_max
    dref = torch.from_numpy(ref).cuda()
    d_bases = torch.from_numpy(rd.bases).cuda()
    d_offs = torch.from_numpy(rd.offsets).cuda()
    # the paper's bin counts: N x 64k bins over the genome
    bins = [(f"{n}x64k", math.ceil(G / (n * 65536))) for n in (int(x) for x in args.bins_64k.split(","))]
    qs = [int(x) for x in args.q.split(",")]
    e_list = list(range(e_max + 1))
    existence = existence_study(dref, d_bases, d_offs, rd.n, qs, bins, O, e_list)
    fn = fn_study(dref, d_bases, d_offs, rd.n, bins, O, e_list, args.cap)
    out = {"genome_bp": G, "reads": rd.n, "read_len": L, "overlap": O, "read_existence": existence,
           "false_negative_rate": fn}
    if args.json:
        with open(args.json, "w") as f:
            json.dump(out, f, indent=1)
    print(json.dumps(out))


def sweep_reads_spec(seed: int, n: int, L: int = 100, e_max: int = 5):
    """Reads of the sweep: L bases, error rates spread evenly over 0..e_max per cent,
    floor(e * L) edits applied."""
    import synth
    return synth.ReadSpec(n_reads=n, seed=seed + 77, lens=(L,), len_w=(1,),
                          err_pm=tuple(10 * e for e in range(e_max + 1)), err_w=(1,) * (e_max + 1), edit_mode=1)


if __name__ == "__main__":
    main()
