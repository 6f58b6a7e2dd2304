"""The oracle's pins must fail for plausible mistakes planted in it.

Each case edits one spot of a copy of the C oracle (on the CPU), builds it
with the same flags, and runs the pin checks of ``test_oracle`` against it:
at least one pin has to fail.  The real oracle is restored afterwards.
"""
import os

import pytest

import oracle
import test_oracle as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "ivf_oracle.c")

MUTANTS = {
    # tie-break: ">=" lets a later equal cluster win
    "tie_rule": ("if (rho[j] > best) { best = rho[j]; a = j; }",
                 "if (rho[j] >= best && rho[j] > 0.0) { best = rho[j]; a = j; }"),
    # a dropped term: the last nonzero of every object is skipped
    "dropped_term": ("for (int64_t h = xp[i]; h < xp[i + 1]; ++h) {\n                    const int32_t s = xi[h];",
                     "for (int64_t h = xp[i]; h + 1 < xp[i + 1]; ++h) {\n                    const int32_t s = xi[h];"),
    # the mean value alone is accumulated (object value dropped)
    "missing_factor": ("rho[f.cid[q]] = rho[f.cid[q]] + p;", "rho[f.cid[q]] = rho[f.cid[q]] + f.val[q];"),
    # wrong divisor in the update
    "wrong_size": ("w[p] = w[p] / (double)nj;", "w[p] = w[p] / (double)(nj + 1);"),
    # the norm sums values, not squares
    "norm_not_squared": ("double sq = w[p] * w[p];", "double sq = w[p];"),
    # transposed operand: the term id indexes the score vector
    "transposed_index": ("rho[f.cid[q]] = rho[f.cid[q]] + p;", "rho[s % k] = rho[s % k] + p;"),
    # sign error in the accumulation
    "sign_error": ("rho[f.cid[q]] = rho[f.cid[q]] + p;", "rho[f.cid[q]] = rho[f.cid[q]] - p;"),
    # zero-overlap objects reset to cluster 0 instead of keeping theirs
    "zero_overlap_reset": ("int32_t a = prev[i];", "int32_t a = 0;"),
    # IVFD: the score vector cleared once instead of before every mean
    "ivfd_rho_not_cleared": ("for (int64_t i = 0; i < n; ++i) rho[i] = 0.0;",
                             "if (j == 0) for (int64_t i = 0; i < n; ++i) rho[i] = 0.0;"),
    # IVFD: ">=" lets a later equal mean take the object
    "ivfd_tie_rule": ("if (rho[i] > rho_a[i]) {", "if (rho[i] >= rho_a[i] && rho[i] > 0.0) {"),
    # IVFD: objects without overlap reset to cluster 0
    "ivfd_zero_overlap_reset": ("out[i] = prev[i];", "out[i] = 0;"),
    # IVFD: one multiplication counted per posting list instead of per entry
    "ivfd_mult_count": ("m_total += optr[s + 1] - optr[s];", "m_total += optr[s + 1] > optr[s];"),
    # IVFD: the object's value replaced by 1 (the mean value alone is added)
    "ivfd_missing_factor": ("double p = v * oval[q];", "double p = v;"),
    # an empty cluster is zeroed rather than kept
    "empty_cluster_dropped": ("tlen[j] = len;\n                    continue;", "tlen[j] = 0;\n                    continue;"),
}

PIN_CHECKS = [
    lambda: pins.test_sparse_walk_bitwise_equals_dense_bruteforce(11, 90, 160, 7),
    lambda: pins.test_sparse_walk_bitwise_equals_dense_bruteforce(13, 60, 40, 5),
    lambda: pins.test_assignment_and_means_match_exact_rationals(21),
    pins.test_worked_example_golden,
    pins.test_duplicate_initial_means_lowest_j_wins_and_empty_keeps_mean,
    pins.test_zero_overlap_object_keeps_previous,
    pins.test_k_equals_n_each_object_its_own_mean,
    lambda: pins.test_ivfd_assignment_bitwise_equals_dense_bruteforce(71, 90, 160, 7),
    pins.test_ivfd_worked_example_golden,
    pins.test_ivfd_ties_go_to_the_lowest_j_and_zero_overlap_keeps_previous,
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert old in text, "mutation anchor missing: " + name
    so = oracle.compile_variant(text.replace(old, new, 1), str(tmp_path / ("m_%s.so" % name)))
    oracle.use_library(so)
    try:
        failed = 0
        for check in PIN_CHECKS:
            try:
                check()
            except AssertionError:
                failed += 1
        assert failed > 0, "no pin caught the planted mistake " + name
    finally:
        oracle.use_library(None)
