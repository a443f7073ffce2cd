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
* fpcg: flexible preconditioned CG for a preconditioner that need not be a
  fixed symmetric operator (the learned one of `oracle.learned`, applied in
  reduced precision), with the Polak-Ribiere form of beta (Golub & Ye, SIAM J.
  Sci. Comput. 21 (1999); Notay, SIAM J. Sci. Comput. 22 (2000)):
      u = P r;  alpha = r.u / p.Ap;  x += alpha p;  r' = r - alpha Ap;
      u' = P r';  beta = r'.(u' - u) / r.u;  p = u' + beta p.
  Plain CG is the fallback: when r'.u' is not positive (P not positive on r')
  the iteration restarts from the current x with u = r from then on.  The
  stopping rule is that of cg on the unpreconditioned residual.
* minres: the minimum-residual method for symmetric matrices, the solver the
  paper uses for its Toeplitz system (§2.G; its experiments run it because CG
  stalls on the mode-removed, noiseless system).  Lanczos three-term
  recurrence with the Givens QR of the tridiagonal matrix, as in Paige and
  Saunders (SIAM J. Numer. Anal. 12, 1975):
      q = A v_k - alpha_k v_k - beta_k v_{k-1},  alpha_k = v_k.A v_k,
      beta_{k+1} = ||q||,  v_{k+1} = q / beta_{k+1};
      delta2_k = c_{k-1} delta1_k + s_{k-1} alpha_k,
      gamma1_k = s_{k-1} delta1_k - c_{k-1} alpha_k,
      eps_{k+1} = s_{k-1} beta_{k+1},  delta1_{k+1} = -c_{k-1} beta_{k+1},
      gamma2_k = hypot(gamma1_k, beta_{k+1}),  c_k = gamma1_k / gamma2_k,
      s_k = beta_{k+1} / gamma2_k,  tau_k = c_k phi_{k-1},  phi_k = s_k phi_{k-1},
      d_k = (v_k - delta2_k d_{k-1} - eps_k d_{k-2}) / gamma2_k,  x_k = x_{k-1} + tau_k d_k,
  starting from c_0 = -1, s_0 = 0, delta1_1 = eps_1 = 0, phi_0 = beta_1 =
  ||s - A x0||; phi_k is the residual norm of x_k, stopping at
  phi_k <= tol ||s||_2.
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


def fpcg(apply_A, apply_P, s, tol=1e-6, maxiter=10000, x0=None, history=False):
    s = np.asarray(s, dtype=np.float64)
    x = np.zeros_like(s) if x0 is None else np.array(x0, dtype=np.float64)
    r = s - apply_A(x) if x0 is not None else s.copy()
    bnorm = float(np.sqrt(s @ s))
    hist = [float(np.linalg.norm(r)) / bnorm if bnorm > 0 else 0.0]
    it = 0
    fallback = False
    if bnorm == 0.0:
        return (x, 0, hist, fallback) if history else (x, 0)
    u = apply_P(r)
    ru = float(r @ u)
    if not (ru > 0.0 and np.isfinite(ru)):
        fallback = True
        u = r.copy()
        ru = float(r @ r)
    p = u.copy()
    while it < maxiter and np.linalg.norm(r) > tol * bnorm:
        Ap = apply_A(p)
        alpha = ru / float(p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        it += 1
        hist.append(float(np.linalg.norm(r)) / bnorm)
        u_new = r.copy() if fallback else apply_P(r)
        ru_new = float(r @ u_new)
        if not fallback and not (ru_new > 0.0 and np.isfinite(ru_new)):
            fallback = True                      # restart as plain CG
            u_new = r.copy()
            ru_new = float(r @ r)
            p = u_new.copy()
        else:
            beta = (ru_new - float(r @ u)) / ru
            p = u_new + beta * p
        u, ru = u_new, ru_new
    return (x, it, hist, fallback) if history else (x, it)


def minres(apply_A, s, tol=1e-6, maxiter=10000, x0=None, history=False):
    s = np.asarray(s, dtype=np.float64)
    x = np.zeros_like(s) if x0 is None else np.array(x0, dtype=np.float64)
    r = s - apply_A(x) if x0 is not None else s.copy()
    bnorm = float(np.sqrt(s @ s))
    beta = float(np.linalg.norm(r))
    hist = [beta / bnorm if bnorm > 0 else 0.0]
    if bnorm == 0.0 or beta <= tol * bnorm:
        return (x, 0, hist) if history else (x, 0)
    v_prev = np.zeros_like(s)
    v = r / beta
    d_prev = np.zeros_like(s)
    d_prev2 = np.zeros_like(s)
    c, sn = -1.0, 0.0
    delta1, eps = 0.0, 0.0
    phi = beta
    it = 0
    while it < maxiter:
        q = apply_A(v)
        alpha = float(v @ q)
        q = q - alpha * v - beta * v_prev
        beta_next = float(np.linalg.norm(q))
        # Givens QR of the new column of the tridiagonal matrix
        delta2 = c * delta1 + sn * alpha
        gamma1 = sn * delta1 - c * alpha
        eps_next = sn * beta_next
        delta1_next = -c * beta_next
        gamma2 = float(np.hypot(gamma1, beta_next))
        c, sn = gamma1 / gamma2, beta_next / gamma2
        tau = c * phi
        phi = sn * phi
        d = (v - delta2 * d_prev - eps * d_prev2) / gamma2
        x = x + tau * d
        it += 1
        hist.append(abs(phi) / bnorm)
        if abs(phi) <= tol * bnorm or beta_next == 0.0:
            break
        d_prev2, d_prev = d_prev, d
        v_prev, v = v, q / beta_next
        beta = beta_next
        delta1, eps = delta1_next, eps_next
    return (x, it, hist) if history else (x, it)
