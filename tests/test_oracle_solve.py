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
    wl = W.lgs3_10x10()
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


# --- MINRES (§2.G, the paper's Toeplitz solver) ---------------------------------

def test_minres_matches_cholesky_10x10():
    from oracle.solve import minres
    wl = W.lgs3_10x10()
    A = C.system_matrix(wl)
    s = W.turbulent_slopes(wl)[0]
    x, k, hist = minres(lambda v: A @ v, s, tol=1e-10, history=True)
    zref = S.cholesky_solve(A, s)
    assert np.linalg.norm(s - A @ x) <= 1.0001e-10 * np.linalg.norm(s)
    assert np.linalg.norm(x - zref) <= 1e-6 * np.linalg.norm(zref)
    # the QR estimate is the true residual norm, and it never increases
    assert abs(hist[-1] - np.linalg.norm(s - A @ x) / np.linalg.norm(s)) <= 1e-3 * hist[-1]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))


def test_minres_finite_termination_distinct_eigenvalues():
    from oracle.solve import minres
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    lam = np.repeat([0.5, 1.0, 3.0, 7.0, 20.0], 8)
    A = (Q * lam) @ Q.T
    b = rng.standard_normal(40)
    x, k = minres(lambda v: A @ v, b, tol=1e-10)
    assert k <= 5     # five distinct eigenvalues: the Krylov space is exhausted after five steps
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_minres_symmetric_indefinite():
    # where CG's energy norm does not exist MINRES still solves (the reason the paper uses it)
    from oracle.solve import minres
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    lam = np.concatenate([-np.linspace(1, 5, 20), np.linspace(0.5, 9, 40)])
    A = (Q * lam) @ Q.T
    b = rng.standard_normal(60)
    x, k = minres(lambda v: A @ v, b, tol=1e-10, maxiter=500)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-8 * np.linalg.norm(x)


def test_minres_equals_cg_iterate_count_order_on_spd():
    # on an SPD system MINRES and CG need iteration counts of the same order
    from oracle.solve import minres
    wl = W.lgs3_10x10()
    A = C.system_matrix(wl)
    s = W.turbulent_slopes(wl)[0]
    _, kcg = S.cg(lambda v: A @ v, s, tol=1e-8)
    _, kmr = minres(lambda v: A @ v, s, tol=1e-8)
    assert 0.5 * kcg <= kmr <= 1.5 * kcg
