"""Plants plausible mistakes in copies of the oracle (on the CPU) and checks
that the pins in test_oracle_pins.py catch every one of them."""
from __future__ import annotations

import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, exact text in oracle.c, replacement)
MUTATIONS = [
    ("continuation payload mask", "v = (v << 6) | (c & 0x3F);", "v = (v << 6) | (c & 0x1F);"),
    ("continuation shift", "v = (v << 6) | (c & 0x3F);", "v = (v << 5) | (c & 0x3F);"),
    ("2-byte lead payload", "v = b & 0x1F;", "v = b & 0x0F;"),
    ("4-byte lead payload", "v = b & 0x07;", "v = b & 0x03;"),
    ("overlong bound off by one", "(L == 3 && v <= 0x7FF)", "(L == 3 && v < 0x7FF)"),
    ("too-large bound", "if (v >= 0x110000)", "if (v > 0x110000)"),
    ("surrogate range", "if (v >= 0xD800 && v <= 0xDFFF)\n        return ORACLE_ERR_SURROGATE;",
     "if (v >= 0xD800 && v < 0xDFFF)\n        return ORACLE_ERR_SURROGATE;"),
    ("rule 1 bound", "if (b >= 0xF8)", "if (b >= 0xF0)"),
    ("rule order 1 vs 3", "if (b < 0xC0)                   /* 10xxxxxx",
     "if (b < 0xC0 && b != 0xBF)                   /* 10xxxxxx"),
    ("truncation at end", "if (p + L > n)", "if (p + L > n + 1)"),
    ("high/low surrogate swapped", "uint32_t hi = 0xD800 | (v >> 10);", "uint32_t hi = 0xDC00 | (v >> 10);"),
    ("pair payload order", "*cp = 0x10000 + (((w & 0x3FF) << 10) | (w2 & 0x3FF));",
     "*cp = 0x10000 + (((w2 & 0x3FF) << 10) | (w & 0x3FF));"),
    ("pair offset sign", "uint32_t v = cp - 0x10000;", "uint32_t v = cp + 0x10000;"),
    ("lone low accepted", "if (w < 0xD800 || w > 0xDFFF) {", "if (w < 0xD800 || w > 0xDBFF) {"),
    ("3-byte encode lead", "out[0] = (uint8_t)(0xE0 | (cp >> 12));", "out[0] = (uint8_t)(0xE0 | (cp >> 11));"),
    ("utf8 length boundary", "if (cp < 0x800)\n        return 2;", "if (cp <= 0x800)\n        return 2;"),
    ("utf16 error position in words", "return make_result(e, 2 * (uint64_t)i);\n        i += len;\n    }\n    return make_result(ORACLE_OK, n);",
     "return make_result(e, (uint64_t)i);\n        i += len;\n    }\n    return make_result(ORACLE_OK, n);"),
]

PIN_TESTS = [
    pins.test_worked_example_section3,
    pins.test_truncation_respects_input_length,
    pins.test_table_utfsummary_lengths,
    lambda: pins.test_utf8_error_kinds_golden("error_kinds.txt"),
    pins.test_utf16_errors_golden,
    pins.test_roundtrip_every_scalar_value,
    pins.test_first_error_matches_cpython_utf8,
    pins.test_first_error_matches_cpython_utf16,
    lambda: pins.test_exhaustive_utf8_strings(2),
    lambda: pins.test_exhaustive_utf8_strings(3),
    pins.test_structured_4byte_strings,
    pins.test_utf16_single_words_and_pairs,
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_mutation(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found once: {name}"
    mutated = tmp_path / "oracle_mut.c"
    mutated.write_text(src.replace(old, new))
    import shutil
    shutil.copy(os.path.join(os.path.dirname(SRC), "oracle.h"), tmp_path / "oracle.h")
    lib = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-w", str(mutated), "-o", str(lib)], check=True)
    oracle.use_library(str(lib))
    try:
        caught = False
        for t in PIN_TESTS:
            try:
                t()
            except AssertionError:
                caught = True
                break
        assert caught, f"no pin caught mutation: {name}"
    finally:
        oracle.use_library(None)
