"""Pins of the solvers (§2.C first step, §2.G): the Cholesky solution against
an independently assembled matrix, and CG against properties that any correct
CG has (finite termination on k distinct eigenvalues, agreement with the
direct solve, zero iterations from the exact solution)."""
import numpy as np
import pytest

import workloads as W
from oracle import covariance as C
from oracle import solve as S
from oracle import toeplitz as T
from test_oracle_covariance import stencil_product_cov


def test_cholesky_residual_against_stencil_matrix():
    wl = W.tiny(n=5, n_gs=3, lgs=True, n_layer=3, seed=21)
    A_ind = stencil_product_cov(wl) + wl.noise_var * np.eye(wl.n_slopes)
    s = W.turbulent_slopes(wl, seed=3)[0]
    z = S.cholesky_solve(C.system_matrix(wl), s)
    assert np.linalg.norm(A_ind @ z - s) <= 1e-10 * np.linalg.norm(s)


@pytest.mark.parametrize("k", [1, 3, 7])
def test_cg_finite_termination(k):
    rng = np.random.default_rng(k)
    ev = np.repeat(np.linspace(1.0, 50.0, k), 6)
    Q, _ = np.linalg.qr(rng.standard_normal((ev.size, ev.size)))
    A = (Q * ev) @ Q.T
    b = rng.standard_normal(ev.size)
    x, it = S.cg(lambda v: A @ v, b, tol=1e-10, maxiter=100)
    assert it == k
    assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)


def test_cg_matches_cholesky_config1():
    wl = W.c1()
    A = C.system_matrix(wl)
    s = W.turbulent_slopes(wl)[0]
    z = S.cholesky_solve(A, s)
    op = T.ToeplitzOperator(wl)
    x, it = S.cg(op, s, tol=1e-10, maxiter=5000)
    assert 0 < it < 2000
    assert S.relative_residual(lambda v: A @ v, x, s) <= 1e-10
    assert np.linalg.norm(x - z) <= 1e-7 * np.linalg.norm(z)


def test_cg_warm_start_at_solution_does_nothing():
    wl = W.tiny(n=4, n_gs=2, seed=2)
    A = C.system_matrix(wl)
    s = W.gaussian_slopes(wl)[0]
    z = S.cholesky_solve(A, s)
    x, it = S.cg(lambda v: A @ v, s, tol=1e-8, x0=z)
    assert it == 0
