"""The op-count and compression formulas of §2.D/§2.E reproduce the values
the paper prints for n = 80 (printed to one significant digit, truncated)."""
import json
import math
import os

import pytest

from oracle import opcount as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")))


def one_digit(x):
    e = math.floor(math.log10(x))
    return math.floor(x / 10 ** e) * 10 ** e


@pytest.mark.parametrize("key,val", [
    ("compression_ss_n80", lambda: O.compression_ss(80)),
    ("compression_ps_ngs_n80", lambda: O.compression_ps_ngs(80)),
    ("reduction_ss_n80_ngs6_a5", lambda: O.reduction_ss(80, 6)),
    ("reduction_ps_ngs_n80_ngs6_a5", lambda: O.reduction_ps_ngs(80, 6)),
    ("reduction_ps_lgs_n80_ngs6_nl9_a5", lambda: O.reduction_ps_lgs(80, 6, 9, 96)),
])
def test_printed_values(key, val):
    assert abs(one_digit(val()) - GOLD[key]["value"]) < 1e-12


def test_dense_count_ratio():
    # The fused product needs 2N_gs forward and inverse transforms instead of
    # one per block: its count is below the 4 N_gs^2 per-block 2RBT products.
    assert O.ops_ss(74, 6) < 4 * 36 * O.ops_2rbt(74, 74)
