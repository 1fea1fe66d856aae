"""Planted mistakes in the oracle are caught by the pins.

Each mutant is a copy of oracle.c with one plausible mistake (a dropped term,
a transposed operand, a wrong comparison or index), compiled with gcc into a
temporary library.  The pins in oracle_pins.py must reject every one of them.
"""
import os
import subprocess
import sys

import pytest

import oracle

MUTANTS = {
    "affine_transposed": ("*rb = (uint32_t)(a * d + b);", "*rb = (uint32_t)(c * b + d);"),
    "affine_dropped_term": ("*rb = (uint32_t)(a * d + b);", "*rb = (uint32_t)(a * d);"),
    "fold_short_window": ("uint32_t acc = x[i];\n            for (uint64_t j = 1; j < w; ++j)",
                          "uint32_t acc = x[i];\n            for (uint64_t j = 1; j + 1 < w; ++j)"),
    "min_as_max": ("acc = v < acc ? v : acc;", "acc = v > acc ? v : acc;"),
    "add_carry_lost": ("acc = (uint32_t)(acc + v);", "acc = (uint32_t)(acc | v);"),
    "revcomp_no_complement": ("r = r + (uint64_t)(3 - c) * place;", "r = r + (uint64_t)c * place;"),
    "canonical_max": ("if (!(flags & ORC_FORWARD) && rc < fwd) v = rc;",
                      "if (!(flags & ORC_FORWARD) && rc > fwd) v = rc;"),
    "hash_shift": ("    x ^= x >> 29;\n    x *= ORC_C2;", "    x ^= x >> 28;\n    x *= ORC_C2;"),
    "hash_constant": ("ORC_C1 = 0x9E3779B97F4A7C15ull", "ORC_C1 = 0x9E3779B97F4A7C17ull"),
    "naive_window_short": ("for (uint64_t j = p; j < p + w; ++j)", "for (uint64_t j = p; j + 1 < p + w; ++j)"),
    "tie_rightmost": ("return a->pos < b->pos;", "return a->pos > b->pos;"),
    "deque_pops_ties": ("while (tail > head && key_less(&keys[i], &keys[dq[tail - 1]])) --tail;",
                        "while (tail > head && keys[i].h <= keys[dq[tail - 1]].h) --tail;"),
    "no_dedup": ("    if (same) return;\n", "\n"),
    "deque_window_off_by_one": ("uint64_t p = i + 1 - w;", "uint64_t p = i + 2 - w;"),
    "invalid_base_ignored": ("if (c < 0) return 0;", "if (c < 0) c = 0;"),
    "seed_ptr_inclusive": ("        ptr[j] = run;\n        run += next[j];",
                           "        run += next[j];\n        ptr[j] = run;"),
    "seed_key_unshifted": ("next[(hash[i] >> shift) & mask] += 1;", "next[hash[i] & mask] += 1;"),
    "seed_order_reversed": ("        pos_out[next[j]] = pos[i];",
                            "        pos_out[ptr[j + 1] - 1 - (next[j] - ptr[j])] = pos[i];"),
    "split_clean_off_by_one": ("            next_clean = i + 1;", "            next_clean = i;"),
    "extremum_deque_stale_front": ("            while (dq[head] < first) {",
                                   "            while (dq[head] + 1 < first) {"),
    "extremum_deque_min_as_max": ("int beaten = op == ORC_MIN ? x[i] <= back : x[i] >= back;",
                                  "int beaten = op == ORC_MIN ? x[i] >= back : x[i] >= back;"),
    "affine_inverse_sign": ("uint32_t ib = (uint32_t)(0u - ia * x[2 * i + 1]);",
                            "uint32_t ib = (uint32_t)(ia * x[2 * i + 1]);"),
    "split_naive_ignored": ("if ((flags & ORC_SPLIT) && holds_invalid) best = NULL;",
                            "if ((flags & ORC_SPLIT) && holds_invalid && w > 2) best = NULL;"),
}


# Runs the pins against one mutated library in a child process: a mutant may
# write out of bounds, and its damage must not reach the test process.
CHILD = r"""
import sys
sys.path[:0] = [sys.argv[1], sys.argv[2]]
import oracle, oracle_pins
lib = oracle.load(path=sys.argv[3])
for pin in oracle_pins.ALL_PINS:
    try:
        pin(lib)
    except (AssertionError, ValueError, IndexError):
        print("CAUGHT " + pin.__name__)
        sys.exit(0)
print("MISSED")
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle._SRC).read()
    assert src.count(old) >= 1, "mutation site vanished: " + name
    mutated = tmp_path / "oracle_mutant.c"
    mutated.write_text(src.replace(old, new, 1))
    so = str(tmp_path / ("liboracle_%s.so" % name))
    oracle.build(out=so, src=str(mutated), extra_flags=("-w",))
    tests = os.path.dirname(os.path.abspath(__file__))
    r = subprocess.run([sys.executable, "-c", CHILD, os.path.dirname(tests), tests, so],
                       capture_output=True, text=True, timeout=600)
    # death by a signal (an out-of-bounds write caught by the allocator, a
    # fault) also rejects the mutant; a Python error in the child does not
    caught = "CAUGHT" in r.stdout or r.returncode < 0
    assert caught, "mutant %s passed every pin (rc %d): %s" % (name, r.returncode, r.stderr[-500:])
