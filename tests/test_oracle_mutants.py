"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
never in the product path), builds it, routes the oracle through it and
requires at least one pin of test_oracle_pins to fail.
"""
import os

import pytest

import oracle
from tests import test_oracle_pins as pins
from tests import test_oracle_select as select_pins

MUTANTS = {
    # a dropped exchange term in the single-excitation element
    "single_exchange_dropped": ("v += phys_so(H, A, Q, P, Q) - phys_so(H, A, Q, Q, P);",
                                "v += phys_so(H, A, Q, P, Q);", 1),
    # wrong sign between direct and exchange integrals of a double
    "double_exchange_sign": ("return s * (phys_so(H, A, B, P, Q) - phys_so(H, A, B, Q, P));",
                             "return s * (phys_so(H, A, B, P, Q) + phys_so(H, A, B, Q, P));", 1),
    # the phase string counts the orbital itself
    "phase_inclusive": ("for (int j = 0; j < k; ++j) c += bit_get(d, j);",
                        "for (int j = 0; j <= k; ++j) c += bit_get(d, j);", 1),
    # creation operators lose their phase
    "create_no_phase": ("int s = (count_below(d, W, k) & 1) ? -1 : 1;\n    bit_flip(d, k);\n    return s;\n}\n\nstatic int key_cmp",
                        "int s = 1;\n    bit_flip(d, k);\n    return s;\n}\n\nstatic int key_cmp", 1),
    # physicists' <PQ|RS> mapped to (pq|rs) instead of (pr|qs)
    "eri_index_transposed": ("return chem(H, spatial_of(H, P), spatial_of(H, R), spatial_of(H, Q), spatial_of(H, S));",
                             "return chem(H, spatial_of(H, P), spatial_of(H, Q), spatial_of(H, R), spatial_of(H, S));", 1),
    # double counting in the diagonal
    "diag_half_dropped": ("return e1 + 0.5 * e2;", "return e1 + e2;", 1),
    # wrong one-body index in the single element
    "single_h_index": ("double v = h_so(H, A, P);", "double v = h_so(H, A, A);", 1),
    # mixed-spin doubles in (p, q, b, a) order
    "mixed_order_swapped": ("            for (int a = 0; a < nv[0]; ++a)\n                for (int b = 0; b < nv[1]; ++b) {",
                            "            for (int b = 0; b < nv[1]; ++b)\n                for (int a = 0; a < nv[0]; ++a) {", 1),
    # unique step keeps duplicates
    "unique_keeps_duplicates": ("if (nu == 0 || key_cmp(c + (nu - 1) * W, c + i * W, W) != 0) {", "if (1) {", 1),
    # merge emits a key present in both inputs twice
    "merge_duplicates_common": ("else { take = set_in + b * W; a++; b++; }", "else { take = set_in + b * W; a++; }", 1),
    # gradient without the factor 2
    "grad_factor": ("grad[i] = (double)(2.0L * (hp[i] - e * psi[i]) / den);", "grad[i] = (double)((hp[i] - e * psi[i]) / den);", 1),
    # diagonal left out of H psi
    "hpsi_no_diag": ("long double acc = (long double)diag_elem(&H, d) * psi[i];", "long double acc = 0.0L;", 2),
    # reverse index reports the insertion point instead of -1 for absent keys
    "inverse_absent_as_position": ("        else hi = mid;\n    }\n    return -1;\n}", "        else hi = mid;\n    }\n    return lo;\n}", 1),
    # selection ranks by signed amplitude
    "topk_signed": ("const double x = fabs(tk_psi[i]), y = fabs(tk_psi[j]);", "const double x = tk_psi[i], y = tk_psi[j];", 1),
    # equal magnitudes broken by the larger key
    "topk_tie_reversed": ("    return key_cmp(tk_keys + i * tk_W, tk_keys + j * tk_W, tk_W);\n}",
                          "    return key_cmp(tk_keys + j * tk_W, tk_keys + i * tk_W, tk_W);\n}", 1),
}

PIN_CALLS = [
    lambda: pins.test_golden_counts_fixture(),
    lambda: pins.test_canonical_order_classes(),
    lambda: pins.test_literal_equals_slater_condon(5, 2, 3),
    lambda: pins.test_literal_equals_slater_condon(7, 5, 5),
    lambda: pins.test_two_electron_opposite_spin_closed_form(),
    lambda: pins.test_two_electron_same_spin_closed_form(),
    lambda: pins.test_noninteracting_ground_state(),
    lambda: pins.test_orbital_rotation_invariance(5, 2, 2),
    lambda: pins.test_fci_hermitian_and_sc_matches_literal(),
    lambda: pins.test_dedup_set_algebra(1),
    lambda: pins.test_dedup_set_algebra(2),
    lambda: pins.test_energy_matches_dense_rayleigh_quotient(),
    lambda: pins.test_gradient_complex_step_and_finite_difference(),
    lambda: pins.test_eigenvector_has_zero_gradient(),
    lambda: select_pins.test_inverse_map_matches_dictionary(1),
    lambda: select_pins.test_inverse_map_special_cases(),
    lambda: select_pins.test_topk_matches_sort(2),
    lambda: select_pins.test_topk_special_cases(),
]


def _first_failing_pin():
    for i, call in enumerate(PIN_CALLS):
        try:
            call()
        except (AssertionError, ValueError, RuntimeError):
            return i
    return None


def test_unmodified_oracle_passes_all_pins():
    assert _first_failing_pin() is None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new, count = MUTANTS[name]
    src = oracle.source_text()
    assert src.count(old) >= count, f"mutation site for {name} not found"
    mutated = src.replace(old, new, count)
    lib = oracle.compile_variant(mutated, os.path.join(str(tmp_path), f"mut_{name}.so"))
    with oracle.use_library(lib):
        failing = _first_failing_pin()
    assert failing is not None, f"no pin catches the planted mistake {name}"
