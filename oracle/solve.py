"""Solvers for (Sigma_ss + Sigma_eta) zeta = s (§2.C, first step; §2.G).

* cholesky_solve: the plain definition, zeta = A^-1 s through a Cholesky
  factorisation of the dense SPD matrix (A is symmetric positive definite for
  sigma^2 > 0: a covariance of linear functionals plus a positive diagonal).
* cg: unpreconditioned conjugate gradients (§2.G names CG among the solvers the
  paper tests), in the textbook form
      alpha = r.r / p.Ap;  x += alpha p;  r -= alpha Ap;
      beta = r'.r' / r.r;  p = r' + beta p,
  x0 = 0 unless given, stopping when the recursive residual satisfies
  ||r||_2 <= tol ||s||_2.
* pcg: the same with a symmetric positive definite preconditioner P (the
  paper leaves preconditioning open, §2.G; `oracle.precond` gives the
  block-circulant one), textbook form
      z = P r;  alpha = r.z / p.Ap;  x += alpha p;  r -= alpha Ap;
      z' = P r';  beta = r'.z' / r.z;  p = z' + beta p,
  with the same stopping rule on the unpreconditioned residual.
"""
import numpy as np
import scipy.linalg


def cholesky_solve(A, s):
    c = scipy.linalg.cho_factor(A, lower=True)
    return scipy.linalg.cho_solve(c, s)


def cg(apply_A, s, tol=1e-6, maxiter=10000, x0=None, history=False):
    s = np.asarray(s, dtype=np.float64)
    x = np.zeros_like(s) if x0 is None else np.array(x0, dtype=np.float64)
    r = s - apply_A(x) if x0 is not None else s.copy()
    p = r.copy()
    rr = float(r @ r)
    bnorm = float(np.sqrt(s @ s))
    hist = [np.sqrt(rr) / bnorm if bnorm > 0 else 0.0]
    it = 0
    if bnorm == 0.0:
        return (x, 0, hist) if history else (x, 0)
    while it < maxiter and np.sqrt(rr) > tol * bnorm:
        Ap = apply_A(p)
        alpha = rr / float(p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
        hist.append(np.sqrt(rr) / bnorm)
    return (x, it, hist) if history else (x, it)


def relative_residual(apply_A, x, s):
    r = np.asarray(s) - apply_A(x)
    return float(np.linalg.norm(r) / np.linalg.norm(s))


def pcg(apply_A, apply_P, s, tol=1e-6, maxiter=10000, x0=None, history=False):
    s = np.asarray(s, dtype=np.float64)
    x = np.zeros_like(s) if x0 is None else np.array(x0, dtype=np.float64)
    r = s - apply_A(x) if x0 is not None else s.copy()
    bnorm = float(np.sqrt(s @ s))
    hist = [float(np.linalg.norm(r)) / bnorm if bnorm > 0 else 0.0]
    it = 0
    if bnorm == 0.0:
        return (x, 0, hist) if history else (x, 0)
    z = apply_P(r)
    p = z.copy()
    rz = float(r @ z)
    while it < maxiter and np.linalg.norm(r) > tol * bnorm:
        Ap = apply_A(p)
        alpha = rz / float(p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        z = apply_P(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
        hist.append(float(np.linalg.norm(r)) / bnorm)
    return (x, it, hist) if history else (x, it)
