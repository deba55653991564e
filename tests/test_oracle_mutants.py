"""The pins are sharp: plausible mistakes planted in a copy of the oracle
(compiled on the CPU into a temporary directory) each fail at least one pin.
"""
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as pins
from conftest import load_golden

SRC = os.path.join(os.path.dirname(oracle.__file__), "rans_oracle.c")

# (name, original text, mutated text, count of occurrences to replace)
MUTANTS = [
    ("C drops cum", "return M * (x / fs) + (x % fs) + m->cum[s];",
     "return M * (x / fs) + (x % fs);", 1),
    ("D wrong sign", "+ j - m->cum[s];", "+ j + m->cum[s];", 1),
    ("C transposed divisor", "return M * (x / fs) + (x % fs) + m->cum[s];",
     "return fs * (x / M) + (x % M) + m->cum[s];", 1),
    ("decoder digit weight", "y = g->b * y + dig[(*rd)++];",
     "y = y + g->b * dig[(*rd)++];", 1),
    ("interval upper bound off by one", "return x >= g->L && x < g->b * g->L;",
     "return x >= g->L && x <= g->b * g->L;", 1),
    ("coder order reversed", "j = (uint32_t)(i % g->N);",
     "j = (uint32_t)(g->N - 1 - i % g->N);", 4),
    ("initial state off by one", "states[j] = g->L; /* reading Q3 */",
     "states[j] = g->L + 1;", 2),
    ("emit wrong digit", "buf[--*pos] = (uint32_t)(*x % g->b);",
     "buf[--*pos] = (uint32_t)(*x / g->b % g->b);", 1),
    ("raw digit weight", "v = v * g->b + dig[rd++];", "v = v + g->b * dig[rd++];", 1),
    ("escape ignores zero frequency", "if (v >= E || m->f[v] == 0) {", "if (v >= E) {", 1),
    ("quantiser deficit ties to the higher index", "return i < j ? -1 : (i > j ? 1 : 0);",
     "return i > j ? -1 : (i < j ? 1 : 0);", 1),
    ("quantiser excess ties to the higher index", "if (f[s] > 1 && (best == n || f[s] > f[best]))",
     "if (f[s] > 1 && (best == n || f[s] >= f[best]))", 1),
    ("quantiser deficit to forced symbols too", "if (counts[s] > 0 && !forced[s])",
     "if (counts[s] > 0)", 1),
    # breadth-first rounds after the first taken in descending lane order,
    # consistently in the encoder and the decoder (round trips still pass)
    ("breadth-first later rounds lanes descending", [
        ("            for (j = active; j-- > 0;) {\n                if (q < lane_nd[j]) {",
         "            for (uint32_t jj = 0; jj < active; jj++) {\n                j = q ? jj : active - 1 - jj;\n"
         "                if (q < lane_nd[j]) {", 1),
        ("        do {\n            any = 0;\n            for (j = 0; j < active; j++) {\n"
         "                if (x[j] < g->L) {",
         "        int round_no = -1;\n        do {\n            any = 0;\n            round_no++;\n"
         "            for (uint32_t jj = 0; jj < active; jj++) {\n"
         "                j = round_no ? active - 1 - jj : jj;\n                if (x[j] < g->L) {", 1),
    ], None, None),
]


def _checks(golden):
    return [
        lambda: pins.test_example_C_and_D_equal_paper_formulas(golden),
        lambda: pins.test_example_precursor_sets_match_paper(golden),
        lambda: pins.test_example_decoder_passes_printed_state(golden),
        lambda: pins.test_example_encoder_decoder_lockstep(golden),
        lambda: pins.test_C_D_are_inverse_bruteforce(),
        lambda: pins.test_precursor_sets_are_b_unique_bruteforce(),
        lambda: pins.test_exhaustive_roundtrip_and_injectivity(2),
        lambda: pins.test_interleaved_stream_equals_instrumented_mux(3),
        lambda: pins.test_escape_with_one_symbol_table_is_raw_storage(16, 16),
        lambda: pins.test_escape_roundtrip_and_states_equal_token_stream(8, 23, 4, 1000),
        lambda: pins.test_digit_orders_equal_hand_derived_streams("digit_order_two_coders.txt"),
        lambda: pins.test_digit_orders_equal_hand_derived_streams("digit_order_packed_load.txt"),
        lambda: pins.test_breadth_first_rounds_read_lanes_ascending(),
        lambda: pins.test_quantizer_hand_computed_ties_and_excess(),
    ]


@pytest.mark.parametrize("name,old,new,count", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_fails_a_pin(tmp_path, name, old, new, count):
    src = open(SRC).read()
    edits = old if isinstance(old, list) else [(old, new, count)]
    mutated = src
    for o, n_, c in edits:
        assert mutated.count(o) == c, (name, o)
        mutated = mutated.replace(o, n_)
    cfile = tmp_path / "mutant.c"
    cfile.write_text(mutated)
    so = tmp_path / "mutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", "-pthread",
                           str(cfile), "-o", str(so)])
    golden = load_golden("worked_example.txt")
    failed = []
    oracle.use_library(str(so))
    try:
        for i, chk in enumerate(_checks(golden)):
            try:
                chk()
            except (AssertionError, oracle.OracleError, IndexError):
                failed.append(i)
    finally:
        oracle.use_library(None)
    assert failed, f"mutant '{name}' passed every pin"
