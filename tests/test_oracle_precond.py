"""Pins of the oracle's block-circulant preconditioner and PCG (oracle.precond,
oracle.solve.pcg).

* The frequency-by-frequency form (per-frequency eigen-decomposition, negative
  eigenvalues clamped, sigma^2 added, inverted, applied through the transform
  steps) equals an independent dense construction: the block-circulant matrix
  assembled entry by entry in the spatial domain from the embedded kernels,
  its positive part by a dense eigen-decomposition, plus sigma^2 I, inverted,
  restricted to the valid subapertures.
* P is symmetric positive definite.
* The clamp is not vacuous: the 10x10 workload's embedding has negative
  eigenvalues.
* PCG with P = I takes exactly CG's iterates; with P = A^-1 it finishes in one
  iteration; with the circulant P it reaches the Cholesky solution in fewer
  iterations than CG."""
import numpy as np
import pytest

import workloads as W
from oracle.covariance import kernel_tables, system_matrix
from oracle.precond import CirculantPreconditioner, inverse_spectra
from oracle.solve import cg, cholesky_solve, pcg
from oracle.toeplitz import embed_kernel, kernel_spectra

CASES = [dict(n=3, n_gs=2, lgs=True, n_layer=2, seed=2, pad_L=5),
         dict(n=4, n_gs=3, lgs=True, n_layer=3, seed=3, pad_L=8),
         dict(n=4, n_gs=1, lgs=False, n_layer=2, seed=5, pad_L=7, mask="full")]


def _dense_preconditioner(wl, L):
    """Spatial-domain block-circulant matrix, its positive part, + sigma^2, inverse, restricted."""
    tabs = kernel_tables(wl)
    C, n = 2 * wl.n_gs, wl.n
    N = L * L
    big = np.zeros((C * N, C * N))
    yy, xx = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    py, px = yy.ravel(), xx.ravel()
    for (gi, gj, p, q), t in tabs.items():
        a, b = 2 * gi + p, 2 * gj + q
        K = embed_kernel(t, L)
        # circular convolution: out[y] = sum_z K[(y - z) mod L] in[z]
        blk = K[(py[:, None] - py[None, :]) % L, (px[:, None] - px[None, :]) % L]
        big[a * N:(a + 1) * N, b * N:(b + 1) * N] = blk
    lam, V = np.linalg.eigh(0.5 * (big + big.T))
    inv = (V / (np.maximum(lam, 0.0) + wl.noise_var)) @ V.T
    # valid subapertures of each channel, in the slope-vector order
    idx = []
    for c in range(C):
        for i in range(n):
            for j in range(n):
                if wl.valid[i, j]:
                    idx.append(c * N + i * L + j)
    idx = np.array(idx)
    return inv[np.ix_(idx, idx)]


def _dense_of(op, m):
    return np.column_stack([op(e) for e in np.eye(m)])


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c['n']}g{c['n_gs']}L{c['pad_L']}")
def test_frequency_form_equals_dense_construction(case):
    wl = W.tiny(**case)
    P = CirculantPreconditioner(wl)
    got = _dense_of(P, wl.n_slopes)
    ref = _dense_preconditioner(wl, wl.pad_L)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_symmetric_positive_definite_10x10():
    wl = W.lgs3_10x10()
    P = _dense_of(CirculantPreconditioner(wl), wl.n_slopes)
    assert np.abs(P - P.T).max() <= 1e-12 * np.abs(P).max()
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0


def test_embedding_has_negative_eigenvalues_10x10():
    # the reading that clamps them is exercised, and the inverse is still finite Hermitian PD
    wl = W.lgs3_10x10()
    S = kernel_spectra(kernel_tables(wl), wl.n_gs, wl.pad_L)
    Mf = np.moveaxis(S, (0, 1), (-2, -1))
    assert np.linalg.eigvalsh(Mf).min() < -1.0
    inv = np.moveaxis(inverse_spectra(S, wl.noise_var), (0, 1), (-2, -1))
    assert np.all(np.isfinite(inv))
    assert np.abs(inv - np.conj(np.swapaxes(inv, -1, -2))).max() < 1e-12 * np.abs(inv).max()
    ev = np.linalg.eigvalsh(inv)
    assert ev.min() > 0 and ev.max() <= 1.0 / wl.noise_var * (1 + 1e-12)


def test_pcg_identity_is_cg():
    wl = W.lgs3_10x10()
    A = system_matrix(wl)
    s = W.turbulent_slopes(wl)[0]
    x1, k1, h1 = cg(lambda v: A @ v, s, tol=1e-8, history=True)
    x2, k2, h2 = pcg(lambda v: A @ v, lambda v: v.copy(), s, tol=1e-8, history=True)
    assert k1 == k2
    assert np.allclose(h1, h2, rtol=1e-9, atol=0)
    assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x1)


def test_pcg_exact_inverse_one_iteration():
    wl = W.tiny(n=4, n_gs=2, seed=1)
    A = system_matrix(wl)
    Ai = np.linalg.inv(A)
    s = W.gaussian_slopes(wl, seed=2)[0]
    x, k = pcg(lambda v: A @ v, lambda v: Ai @ v, s, tol=1e-10)
    assert k == 1
    assert np.linalg.norm(x - cholesky_solve(A, s)) <= 1e-10 * np.linalg.norm(x)


def test_pcg_circulant_reaches_cholesky_in_fewer_iterations_10x10():
    wl = W.lgs3_10x10()
    A = system_matrix(wl)
    s = W.turbulent_slopes(wl)[0]
    P = CirculantPreconditioner(wl)
    x, k = pcg(lambda v: A @ v, P, s, tol=1e-10)
    _, kcg = cg(lambda v: A @ v, s, tol=1e-10)
    zref = cholesky_solve(A, s)
    assert np.linalg.norm(s - A @ x) <= 1.0001e-10 * np.linalg.norm(s)
    assert np.linalg.norm(x - zref) <= 1e-5 * np.linalg.norm(zref)
    assert k < 0.75 * kcg
