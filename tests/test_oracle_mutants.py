"""The pins must catch plausible mistakes in the oracle.

Each case copies the oracle source, plants one mistake by text substitution,
builds it on the CPU, and runs the pin functions against it: at least one pin
must fail. The oracle source itself is never modified.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

import pytest

import test_oracle_pins as pins
import test_oracle_seed_pins as spins
import test_oracle_verify_pins as vpins
from oracle import Oracle
from oracle.oracle import BUILD_CMD, _SRC

MUTANTS = {
    "threshold_q_minus_1_per_error": ("(int64_t)q * (int64_t)E", "((int64_t)q - 1) * (int64_t)E"),
    "threshold_token_count_off_by_one": ("((int64_t)L - (int64_t)q + 1)", "((int64_t)L - (int64_t)q)"),
    "no_bin_overlap": ("a + (uint64_t)B + (uint64_t)O", "a + (uint64_t)B"),
    "strict_comparison_pass": ("(int64_t)cnt >= T ? 1 : 0;\n  }\n  return 0;", "(int64_t)cnt > T ? 1 : 0;\n  }\n  return 0;"),
    "floor_error_budget": ("e_permille + 999) / 1000", "e_permille) / 1000"),
    "last_read_token_dropped": ("i + q <= L", "i + q < L"),
    "colliding_token_code": ("code = code * 4 + c;", "code = code * 3 + c;"),
    "n_read_as_a": ("if (c < 0) return -1;\n    code", "if (c < 0) c = 0;\n    code"),
    "last_reference_window_dropped": ("? G - q + 1 : 0", "? G - q : 0"),
    "partial_last_bin_dropped": ("return (G + B - 1) / B;", "return G / B;"),
    "bins_not_extended_at_start": ("uint64_t a = x * (uint64_t)B;", "uint64_t a = x * (uint64_t)B + 1;"),
    "verify_global_not_semiglobal": ("col[0] = 0;", "col[0] = diag + 1;"),
    "verify_alignment_must_reach_text_end": ("if (col[L] < best) best = col[L];", ""),
    "verify_n_matches_n": ("(rc >= 0 && rc == tc)", "(rc == tc)"),
    "verify_window_misses_last_token_bases": ("*hi = b > a ? b + q - 1 : a;", "*hi = b > a ? b : a;"),
    "verify_match_strict": ("match[k] = d <= E ? 1 : 0;", "match[k] = d < E ? 1 : 0;"),
    "verify_substitution_free": ("((rc >= 0 && rc == tc) ? 0u : 1u)", "0u"),
    "verify_bounded_cap_at_budget": ("(uint16_t)(E + 1 < 0xFFFE ? E + 1 : 0xFFFE)", "(uint16_t)(E < 0xFFFE ? E : 0xFFFE)"),
    "verify_bounded_overwrites_skipped": ("if (dist[k] == 0xFFFF) continue; /* not aligned */", ""),
    "verify_bounded_global_rate_only": ("  if (err_pm_per_read) return oracle_max_edits(L, err_pm_per_read[r]);\n", ""),
    "seed_overlapping_seeds": ("o + (int64_t)k <= L; o += k)", "o + (int64_t)k <= L; o += 1)"),
    "seed_no_clamp_at_start": ("if (loc < 0) loc = 0;\n        if (nh", "if (nh"),
    "seed_rank_ties_to_larger_bin": ("return x->bin < y->bin ? -1 : (x->bin > y->bin ? 1 : 0);\n}\n\nstatic int cmp_bin",
                                     "return x->bin > y->bin ? -1 : (x->bin < y->bin ? 1 : 0);\n}\n\nstatic int cmp_bin"),
    "seed_rank_fewer_votes_first": ("if (x->votes != y->votes) return x->votes > y->votes ? -1 : 1;",
                                    "if (x->votes != y->votes) return x->votes < y->votes ? -1 : 1;"),
    "seed_n_seed_used": ("if (code < 0) continue;\n      /* first entry", "if (code < 0) code = 0;\n      /* first entry"),
}

BOUNDED_PIN_CALLS = [
    lambda o: vpins.test_verify_bounded_explicit_budget(o),
    lambda o: vpins.test_verify_bounded_ceiling_budget(o),
    lambda o: vpins.test_verify_bounded_keeps_skipped_pairs(o),
    lambda o: vpins.test_verify_bounded_largest_values(o),
    *[(lambda o, s=s: vpins.test_verify_bounded_bruteforce(o, s)) for s in range(2)],
]

PIN_CALLS = [
    lambda o: pins.test_vector_length_q5(o),
    lambda o: pins.test_index_footprint_paper(o),
    lambda o: pins.test_counter_width_100bp(o),
    lambda o: pins.test_exact_match_threshold(o),
    lambda o: pins.test_ceil_error_budget(o),
    lambda o: pins.test_error_propagation_q4(o),
    *[(lambda o, a=a: pins.test_threshold_is_tight(o, *a)) for a in [(3, 30, 2), (4, 40, 3), (5, 60, 4)]],
    *[(lambda o, s=s: pins.test_counts_match_set_recount(o, s)) for s in range(6)],
    lambda o: pins.test_bits_match_set_definition(o),
    *[(lambda o, s=s: pins.test_no_false_negatives_bruteforce(o, s)) for s in range(2)],
    lambda o: pins.test_exact_substring_counts_all_tokens(o),
    lambda o: pins.test_homopolymer(o),
    lambda o: pins.test_first_base_rule(o),
    lambda o: pins.test_last_partial_bin_and_tail_token(o),
    lambda o: pins.test_n_windows(o),
    lambda o: pins.test_nonpositive_threshold_passes_everything(o),
    *[(lambda o, s=s: vpins.test_verify_distance_bruteforce(o, s)) for s in range(4)],
    lambda o: vpins.test_verify_nonacgt_matches_nothing(o),
    lambda o: vpins.test_verify_closed_forms(o),
    lambda o: vpins.test_verify_window_edges(o),
    lambda o: vpins.test_verify_truth_locations(o),
    lambda o: vpins.test_verify_mask_skips_pairs(o),
    *BOUNDED_PIN_CALLS,
    *[(lambda o, s=s: spins.test_seed_candidates_bruteforce(o, s)) for s in range(3)],
    lambda o: spins.test_seed_ties_cap_and_clamp(o),
]


def _build_mutant(tmp: str, old: str, new: str) -> str:
    src = open(_SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {old!r}"
    path = os.path.join(tmp, "mutant.c")
    open(path, "w").write(src.replace(old, new))
    out = os.path.join(tmp, "libmutant.so")
    subprocess.check_call(BUILD_CMD + [path, "-o", out])
    return out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name):
    old, new = MUTANTS[name]
    tmp = tempfile.mkdtemp(prefix="oracle_mutant_")
    try:
        mutant = Oracle(_build_mutant(tmp, old, new))
        caught = 0
        for call in PIN_CALLS:
            try:
                call(mutant)
            except (AssertionError, ValueError, IndexError):
                caught += 1
        assert caught > 0, f"no pin catches mutant {name}"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


# The mistakes a bounded verification could make: cap at E instead of E + 1,
# take E with a floor, overwrite the skipped marker, ignore per-read rates.
# The bounded pins alone must catch each of them.
BOUNDED_MUTANTS = ["verify_bounded_cap_at_budget", "verify_bounded_overwrites_skipped",
                   "verify_bounded_global_rate_only", "floor_error_budget"]


@pytest.mark.parametrize("name", BOUNDED_MUTANTS)
def test_bounded_pins_catch_mutant(name):
    old, new = MUTANTS[name]
    tmp = tempfile.mkdtemp(prefix="oracle_mutant_")
    try:
        mutant = Oracle(_build_mutant(tmp, old, new))
        caught = 0
        for call in BOUNDED_PIN_CALLS:
            try:
                call(mutant)
            except (AssertionError, ValueError, IndexError):
                caught += 1
        assert caught > 0, f"no bounded-verification pin catches mutant {name}"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
