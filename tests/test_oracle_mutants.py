"""Each plausible mistake planted in a copy of the oracle is caught by a pin.

The mistake is planted in the C source of a temporary copy of the oracle,
which is compiled and run on the CPU; the real oracle is untouched.
"""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# (name, text in oracle.c, replacement): each is a mistake a reader could make.
MUTANTS = [
    ("reverses_k_plus_1_bits", "for (j = 0; j < k; ++j)", "for (j = 0; j <= k; ++j)"),
    ("reverses_k_minus_1_bits", "for (j = 0; j < k; ++j)", "for (j = 1; j < k; ++j)"),
    ("no_reversal", "((i >> j) & 1u)", "((i >> (k - 1 - j)) & 1u)"),
    ("swaps_every_pair_twice", "if (i < r)", "if (i != r)"),
    ("swaps_wrong_side", "if (i < r)", "if (i > r + 1)"),
    ("skips_index_one", "for (i = 0; i < n; ++i) {", "for (i = 2; i < n; ++i) {"),
    ("drops_last_byte", "for (t = 0; t < s; ++t)", "for (t = 1; t < s; ++t)"),
    ("oop_wrong_width", "oracle_rev(i, k) * elem_size", "oracle_rev(i, k - 1) * elem_size"),
    ("rows_forget_elem_size", "row_bytes = ((size_t)1 << k) * elem_size;",
     "row_bytes = ((size_t)1 << k);"),
    ("batched_offsets_in_bytes", "(size_t)offsets[a] * elem_size", "(size_t)offsets[a]"),
    ("batched_skips_last_array", "for (a = 0; a < num_arrays; ++a)",
     "for (a = 0; a + 1 < num_arrays; ++a)"),
    ("digits_reversed_bitwise", "r = (r << d) | ((i >> j) & mask);",
     "r = (r << d) | oracle_rev((i >> j) & mask, d);"),
    ("digit_dropped", "for (j = 0; j < k; j += d)", "for (j = d; j < k; j += d)"),
    ("evenodd_swapped_halves", "memcpy(out + j * elem_size, in + (2 * j) * elem_size",
     "memcpy(out + j * elem_size, in + (2 * j + 1) * elem_size"),
]


# A mutant may write out of bounds, so the pins run in a child process: a
# crash there counts as caught, as does any failing pin.
_CHILD = r"""
import sys
sys.path[:0] = [%r, %r]
import oracle, oracle_pins
o = oracle.Oracle(sys.argv[1])
failed = []
for pin in oracle_pins.ALL_PINS:
    try:
        pin(o)
    except (AssertionError, ValueError):
        failed.append(pin.__name__)
print("FAILED:" + ",".join(failed))
""" % (ROOT, HERE)


def _run_pins(so_path):
    p = subprocess.run([sys.executable, "-c", _CHILD, so_path], capture_output=True,
                       text=True, timeout=600)
    if p.returncode != 0:
        return ["crashed(%d)" % p.returncode]
    line = [ln for ln in p.stdout.splitlines() if ln.startswith("FAILED:")][-1]
    return [f for f in line[len("FAILED:"):].split(",") if f]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    src = open(oracle.SOURCE).read()
    assert src.count(old) >= 1, "mutation site vanished from oracle.c: %r" % old
    mutated = src.replace(old, new, 1)
    c_path = os.path.join(str(tmp_path), "oracle_%s.c" % name)
    with open(c_path, "w") as f:
        f.write(mutated)
    so = oracle.compile_source(c_path, os.path.join(str(tmp_path), "lib_%s.so" % name))
    failed = _run_pins(so)
    assert failed, "mutant %s passed every pin" % name
