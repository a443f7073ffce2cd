"""Pins of the 2RBT product by circulant embedding (§2.E) against the dense
product, brute force on tiny grids, including the paper's own one-dimensional
shuffle form and the independence of the padding L."""
import numpy as np
import pytest

import workloads as W
from oracle import covariance as C
from oracle import geometry as G
from oracle import toeplitz as T

CASES = [(n, g, lgs, seed) for n, g, lgs, seed in
         [(2, 1, False, 0), (3, 2, True, 1), (4, 3, True, 2), (5, 1, True, 3),
          (6, 4, False, 4), (7, 2, True, 5), (8, 2, True, 6)]]


@pytest.mark.parametrize("n,g,lgs,seed", CASES)
def test_fft_matvec_equals_dense(n, g, lgs, seed):
    wl = W.tiny(n=n, n_gs=g, lgs=lgs, n_layer=2, seed=seed)
    A = C.system_matrix(wl)
    tabs = C.kernel_tables(wl)
    x = np.random.default_rng(seed).standard_normal(wl.n_slopes)
    ref = A @ x
    for L in sorted({2 * n - 1, 2 * n, 2 * n + 3, 1 << int(np.ceil(np.log2(2 * n)))}):
        y = T.ToeplitzOperator(wl, tables=tabs, L=L)(x)
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max(), L


def test_padding_too_small_rejected():
    wl = W.tiny(n=4, n_gs=1)
    with pytest.raises(ValueError):
        T.ToeplitzOperator(wl, L=6)


def test_paper_one_dimensional_form():
    # §2.E step 1-5 literally, m = n: x reversed into a row-stride (2n-1) array
    # (b_mu = x_k, mu = 2n(n-1) - i(2n-1) - j), a 1-D cyclic convolution of
    # length (2n-1)^2 with the table laid out on the same stride, and y read at
    # mu = 2n(2n-1) - (i+1)(2n-1) - (j+1).
    wl = W.tiny(n=5, n_gs=1, lgs=False, n_layer=1, seed=3, mask="full")
    n = wl.n
    N = 2 * n - 1
    t = C.kernel_table(wl, 0, 0, 0, 0)            # t[v+n-1, u+n-1]
    S = C.slope_covariance(wl)[: n * n, : n * n]
    x = np.random.default_rng(0).standard_normal(n * n)
    b = np.zeros(N * N)
    for i in range(n):
        for j in range(n):
            b[2 * n * (n - 1) - i * N - j] = x[i * n + j]
    # the unique-element vector on the same stride: entry (R, C) holds t at
    # lag (u, v) = (n-1 - C', ...) chosen so that the read-out below equals Theta x
    tv = np.zeros(N * N)
    for R in range(N):
        for Cc in range(N):
            tv[R * N + Cc] = t[N - 1 - R, N - 1 - Cc]
    c = np.real(np.fft.ifft(np.fft.fft(tv) * np.fft.fft(b)))
    y = np.zeros(n * n)
    for i in range(n):
        for j in range(n):
            y[i * n + j] = c[2 * n * N - (i + 1) * N - (j + 1)]
    assert np.abs(y - S @ x).max() <= 1e-12 * np.abs(S @ x).max()


def test_linearity_and_noise_term():
    wl = W.tiny(n=4, n_gs=2, seed=8)
    op = T.ToeplitzOperator(wl)
    rng = np.random.default_rng(1)
    x, z = rng.standard_normal((2, wl.n_slopes))
    assert np.allclose(op(2 * x - 3 * z), 2 * op(x) - 3 * op(z), atol=1e-10)
    op0 = T.ToeplitzOperator(wl, tables=op.tables, noise_var=0.0)
    assert np.allclose(op(x) - op0(x), wl.noise_var * x, atol=1e-12)
