"""The five synthetic workloads, each with the sizes its description states.

A workload bundles a genome recipe, a read recipe and the filter parameters
(bin size B, overlap O, token length q, error budget). Choices the workload
descriptions leave open are made here:
B = 2048 everywhere; O = L_max + E_max (105 for 100 bp reads at E=5; 263 for
the 3.1 Gbp index, enough for 250 bp reads at 5%); the human-scale repeat
families are 64 consensus sequences of 300 bp and 64 of 6 kbp; reads use
substitution:insertion:deletion = 8:1:1 unless stated.
"""

from __future__ import annotations

from dataclasses import dataclass, replace
from typing import Optional

from . import MASTER_SEED, GenomeSpec, ReadSpec

HUMAN_G = 3_100_000_000


@dataclass
class Workload:
    name: str
    genome: GenomeSpec
    reads: ReadSpec
    bin_size: int
    overlap: int
    q: int
    max_edits: Optional[int] = None      # one explicit E for every read
    per_read_error: bool = False         # E_r from each read's own error rate
    mode: str = "allbins"                # "allbins" or "candidates"
    cand_cap: int = 0
    cand_k: int = 12
    layout: str = "tm"                   # index layout the mode needs: "tm" or "bm"


def _c1(seed: int) -> Workload:
    return Workload(
        name="c1_allbins_1Mbp_q5",
        genome=GenomeSpec(length=1_000_000, seed=seed),
        reads=ReadSpec(n_reads=2000, seed=seed + 1, lens=(100,), len_w=(1,), err_pm=(50,), err_w=(1,),
                       edit_mode=0, edits=5, w_sub=8, w_ins=1, w_del=1),
        bin_size=2048, overlap=105, q=5, max_edits=5)


def _c2(seed: int) -> Workload:
    return Workload(
        name="c2_candidates_100Mbp_q5",
        genome=GenomeSpec(length=100_000_000, seed=seed, repeat_frac=0.015, n_families=20,
                          fam_len_lo=300, fam_len_hi=6000, fam_len_mode=0, div_lo=0.10, div_hi=0.20,
                          indel_share=0.10),
        reads=ReadSpec(n_reads=4_000_000, seed=seed + 1, lens=(100,), len_w=(1,), err_pm=(40,), err_w=(1,),
                       edit_mode=2, n_sub=3, n_indel=1),
        bin_size=2048, overlap=105, q=5, max_edits=5, mode="candidates", cand_cap=256, layout="bm")


def _human_genome(seed: int) -> GenomeSpec:
    return GenomeSpec(length=HUMAN_G, seed=seed, repeat_frac=0.45, n_families=128,
                      fam_len_lo=300, fam_len_hi=6000, fam_len_mode=1, div_lo=0.05, div_hi=0.25,
                      indel_share=0.10)


def _c3(seed: int) -> Workload:
    return Workload(
        name="c3_allbins_3.1Gbp_q5",
        genome=_human_genome(seed),
        reads=ReadSpec(n_reads=1_000_000, seed=seed + 1, lens=(150,), len_w=(1,), err_pm=(50,), err_w=(1,),
                       edit_mode=0, edits=7, w_sub=8, w_ins=1, w_del=1),
        bin_size=2048, overlap=263, q=5, max_edits=7)


def _c4(seed: int) -> Workload:
    return Workload(
        name="c4_candidates_uneven_3.1Gbp_q6",
        genome=_human_genome(seed),
        reads=ReadSpec(n_reads=2_000_000, seed=seed + 1, lens=(100, 150, 250), len_w=(30, 40, 30),
                       err_pm=(20, 30, 40, 50), err_w=(1, 1, 1, 1), edit_mode=1, w_sub=8, w_ins=1, w_del=1),
        bin_size=2048, overlap=263, q=6, per_read_error=True, mode="candidates", cand_cap=1024,
        layout="bm")


def _c5(seed: int) -> Workload:
    # The serving workload scans every bin of the q=5 human-scale index; its
    # request stream (Poisson arrivals, log-uniform sizes) is drawn separately.
    return Workload(
        name="c5_serving_3.1Gbp_q5",
        genome=_human_genome(seed),
        reads=ReadSpec(n_reads=0, seed=seed + 1, lens=(100, 150, 250), len_w=(30, 40, 30),
                       err_pm=(20, 30, 40, 50), err_w=(1, 1, 1, 1), edit_mode=1, w_sub=8, w_ins=1, w_del=1),
        bin_size=2048, overlap=263, q=5, per_read_error=True)


_MAKERS = {"c1": _c1, "c2": _c2, "c3": _c3, "c4": _c4, "c5": _c5}


def workload(key: str, scale: float = 1.0) -> Workload:
    """Workload ``key`` (c1..c5) seeded with MASTER_SEED + its index.

    ``scale`` < 1 shrinks read counts (and, for c1/c2, nothing else) for quick
    runs; sizes at scale 1.0 are the stated ones.
    """
    idx = int(key[1]) - 1
    w = _MAKERS[key](MASTER_SEED + idx)
    if scale != 1.0:
        w.reads = replace(w.reads, n_reads=max(1, int(w.reads.n_reads * scale)))
    return w


def shrink(w: Workload, genome_len: Optional[int] = None, n_reads: Optional[int] = None) -> Workload:
    """Copy of ``w`` with a shorter genome and/or fewer reads (same recipe otherwise)."""
    g = w.genome if genome_len is None else replace(w.genome, length=genome_len)
    r = w.reads if n_reads is None else replace(w.reads, n_reads=n_reads)
    return replace(w, genome=g, reads=r)
