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


def test_lgs_compression_printed_value():
    """§2.D prints 6e-3 for N_gs = 6, N_layer = 9, n = 80 without the layer
    altitudes (the 9-layer profile is only a figure).  Reading: n'_k from the
    paper's own rule n'_k ~ n h_lgs / (h_lgs - h_k), rounded up, on 9
    geometric altitudes 30 m - 26.5 km with h_lgs = 90 km."""
    import workloads as W
    h, _ = W.c2_profile(n_layer=9)
    nps = [math.ceil(80 * 90e3 / (90e3 - hk) - 1e-9) for hk in h]
    val = O.compression_ps_lgs(80, 6, nps)
    assert abs(one_digit(val) - GOLD["compression_ps_lgs_n80_ngs6_nl9"]["value"]) < 1e-12
    # the same count with every grid at n (no cone) or the worst-case common grid
    # brackets the printed value from both sides
    assert O.compression_ps_lgs(80, 6, [80] * 9) < 6e-3 < O.compression_ps_lgs(80, 6, [max(nps)] * 9)


def test_lgs_compression_counts_the_built_tables():
    """The formula's terms counted on built objects: the unique elements of
    every Xi'_{q,k} table (one per layer and slope channel, per-layer grid
    sizes), plus the paper's 4 n^2 non-zeros of each I'_k, over the size of the
    dense Sigma_phi_s of a full pupil."""
    import numpy as np

    import workloads as W
    from oracle import geometry as G
    from oracle.covariance import phase_slope_cov
    from oracle.projection import xi_prime_table
    wl = W.tiny(n=4, n_gs=2, lgs=True, n_layer=3, seed=3, mask="full")
    wl.h = np.array([0.0, 20e3, 45e3])
    s = G.cone_scale(wl.h, wl.h_lgs)
    nps = [math.ceil(wl.n / sk - 1e-9) for sk in s]
    unique = sum(xi_prime_table(wl, k, q // 2, q % 2, nps[k]).size
                 for k in range(wl.n_layer) for q in range(2 * wl.n_gs))
    dense = phase_slope_cov(wl, G.phase_points(wl.n, wl.d)).size
    assert dense == (wl.n + 1) ** 2 * 2 * wl.n_gs * wl.n ** 2
    expect = (unique + 4 * wl.n_layer * wl.n ** 2) / dense
    assert abs(O.compression_ps_lgs(wl.n, wl.n_gs, nps) - expect) <= 1e-15 * expect


@pytest.mark.parametrize("n", [2, 10, 74, 80])
def test_single_block_count_is_the_one_channel_fused_count(n):
    """§2.E gives the count of one 2RBT product (two transforms of length
    (2n-1)^2, the element-wise products, both shuffles) and the fused count of
    Sigma_ss zeta for 2 N_gs channels; with a single channel (N_gs = 1/2) the
    fused product is one 2RBT product, so the two printed formulas must agree
    (the fused one is pinned by the printed reduction factor above)."""
    assert abs(O.ops_2rbt(n, n) - O.ops_ss(n, 0.5)) <= 1e-9 * O.ops_2rbt(n, n)
    assert abs(O.ops_2rbt(n, n, a=3.0) - O.ops_ss(n, 0.5, a=3.0)) <= 1e-9 * O.ops_2rbt(n, n)
