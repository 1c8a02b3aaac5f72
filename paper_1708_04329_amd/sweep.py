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

The sweep drives the library only (index build, all-bins scan, seeding,
candidate filter, verification); PyTorch holds the device buffers and counts
the pass bits.
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


def popcount_rows(mask) -> "np.ndarray":
    """Set bits per row of a uint32 [n][W] device mask (SWAR popcount, in row chunks)."""
    import torch
    n = mask.shape[0]
    out = np.empty(n, np.int64)
    step = max(1, (1 << 27) // max(1, mask.shape[1]))
    for r0 in range(0, n, step):
        x = mask[r0:r0 + step].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        x = x - ((x >> 1) & 0x55555555)
        x = (x & 0x33333333) + ((x >> 2) & 0x33333333)
        x = (x + (x >> 4)) & 0x0F0F0F0F
        x = (x * 0x01010101) & 0xFFFFFFFF
        out[r0:r0 + step] = (x >> 24).sum(dim=1).cpu().numpy()
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
    rspec = synth.ReadSpec(n_reads=args.reads, seed=gspec.seed + 77, lens=(L,), len_w=(1,),
                           err_pm=tuple(10 * e for e in range(e_max + 1)), err_w=(1,) * (e_max + 1), edit_mode=1)
    rd = synth.reads(rspec, ref)
    log(f"genome {len(ref):,} bp, {rd.n} reads of {L} bp in {time.time() - t0:.1f}s")
    G = len(ref)
    O = L + e_max
    dref = torch.from_numpy(ref).cuda()
    d_bases = torch.from_numpy(rd.bases).cuda()
    d_offs = torch.from_numpy(rd.offsets).cuda()
    bins_list = [int(x) for x in args.bins_64k.split(",")]
    qs = [int(x) for x in args.q.split(",")]

    existence = []
    for q in qs:
        for nb64 in bins_list:
            B = math.ceil(G / (nb64 * 65536))
            idx = grim.grim_build_index(dref, B, O, q, grim.LAYOUT_TM)
            info = idx.info()
            nb, W = info["n_bins"], info["mask_words"]
            mask = torch.empty((rd.n, W), dtype=torch.uint32, device="cuda")
            for e in range(e_max + 1):
                rs = grim.ReadSet(d_bases, d_offs, err_permille_all=10 * e)
                grim.grim_filter_scan(idx, rs, mask)
                torch.cuda.synchronize()
                frac = float(popcount_rows(mask).mean() / nb)
                existence.append({"q": q, "bins": f"{nb64}x64k", "n_bins": nb, "bin_size": B, "e_pct": e,
                                  "read_existence": frac})
                log(f"q={q} bins={nb64}x64k (B={B}) e={e}%: read existence {frac:.4g}")
            del mask
            idx.free()
            torch.cuda.empty_cache()

    fn = []
    seeds = grim.grim_seeds_build(dref, 12)
    q = 5
    for nb64 in bins_list:
        B = math.ceil(G / (nb64 * 65536))
        idx = grim.grim_build_index(dref, B, O, q, grim.LAYOUT_BM | grim.LAYOUT_REF)
        co = torch.empty(rd.n + 1, dtype=torch.int64, device="cuda")
        cb = torch.empty(rd.n * args.cap, dtype=torch.int32, device="cuda")
        P = grim.grim_seed_candidates(seeds, grim.ReadSet(d_bases, d_offs), B, args.cap, co, cb)
        cbv = cb[:max(P, 1)]
        cnt = torch.empty(max(P, 1), dtype=torch.uint16, device="cuda")
        pas = torch.empty(max(P, 1), dtype=torch.uint8, device="cuda")
        dist = torch.empty(max(P, 1), dtype=torch.uint16, device="cuda")
        match = torch.empty(max(P, 1), dtype=torch.uint8, device="cuda")
        for e in range(e_max + 1):
            rs = grim.ReadSet(d_bases, d_offs, err_permille_all=10 * e)
            grim.grim_filter_candidates(idx, rs, co, cbv[:P], cnt, pas)
            grim.grim_verify_candidates_bounded(idx, rs, co, cbv[:P], None, dist, match)   # every candidate
            torch.cuda.synchronize()
            pv, mv = pas[:P].to(torch.int64), match[:P].to(torch.int64)
            n_pass = int(pv.sum().item())
            n_map = int(mv.sum().item())
            n_pass_map = int((pv & mv).sum().item())
            missed = n_map - n_pass_map          # mapping candidates the filter dropped
            fn.append({"bins": f"{nb64}x64k", "bin_size": B, "e_pct": e, "candidates": P, "passing": n_pass,
                       "mapping": n_map, "fn_rate_filter": 1 - n_pass_map / max(1, n_pass),
                       "fn_rate_no_filter": 1 - n_map / max(1, P), "mapping_locations_filtered_out": missed})
            log(f"bins={nb64}x64k e={e}%: {P:,} candidates, {n_pass:,} pass, {n_map:,} map; "
                f"false-negative rate {fn[-1]['fn_rate_filter']:.4f} (no filter {fn[-1]['fn_rate_no_filter']:.4f})")
        del co, cb, cbv, cnt, pas, dist, match
        idx.free()
        torch.cuda.empty_cache()
    seeds.free()
    out = {"genome_bp": G, "reads": rd.n, "read_len": L, "overlap": O, "read_existence": existence,
           "false_negative_rate": fn}
    if args.json:
        with open(args.json, "w") as f:
            json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
