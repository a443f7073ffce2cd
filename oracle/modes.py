"""Low-order mode removal (§2.F "Mode removal"), in float64.

Per sensor i the tip/tilt/focus modal matrix Z_s,i (2 n_vs x 3) holds the
Hudgin slopes of the phase modes x, y and x^2 + y^2 on the valid
subapertures (up to a scale per column, which a projector ignores):
  tip   x slopes 1, y slopes 0;   tilt  x slopes 0, y slopes 1;
  focus x slopes 2 x d, y slopes 2 y d (the difference of (x +- d/2)^2 + y^2).
M_s,i = I - Z_s,i Z_s,i^+ and M_s is their block diagonal.  In phase space
Z_phi (n_vphi x 3) holds x, y, x^2 + y^2 at the valid phase points and
M_phi = I - Z_phi Z_phi^+.  The system of §2.F with mode removal is
  (M_s W_s)(Sigma_ss + Sigma_eta)(M_s W_s)^T zeta = M_s s,   zeta = M_s zeta,
  phi = M_phi W_phi Sigma_phi_s zeta.
The matrix M_s A M_s is singular (its null space holds the modes) but the
system is consistent; its solution in the range of M_s is the solution of the
non-singular system (M_s A M_s + I - M_s) zeta = M_s s, computed here by
Cholesky.

TEST INFRASTRUCTURE ONLY, like the rest of this package.
"""
import numpy as np

from . import geometry as G


def slope_modes(wl):
    """Z_s,i for one sensor (the same for every sensor: one valid mask), 2 n_vs x 3."""
    n, d = wl.n, wl.d
    r = G.subap_centers(n, d)[G.valid_index(wl.valid)]      # (n_vs, 2): x, y
    nv = r.shape[0]
    Z = np.zeros((2 * nv, 3))
    Z[:nv, 0] = 1.0
    Z[nv:, 1] = 1.0
    Z[:nv, 2] = 2.0 * r[:, 0] * d
    Z[nv:, 2] = 2.0 * r[:, 1] * d
    return Z


def slope_projector(wl):
    """M_s: block diagonal over the sensors of I - Z Z^+."""
    Z = slope_modes(wl)
    Mi = np.eye(Z.shape[0]) - Z @ np.linalg.pinv(Z)
    return np.kron(np.eye(wl.n_gs), Mi)


def phase_modes(wl):
    """Z_phi at the valid phase points (corners of valid subapertures), n_vphi x 3."""
    p = G.phase_points(wl.n, wl.d)[G.valid_phase_mask(wl.valid).ravel()]
    return np.column_stack([p[:, 0], p[:, 1], p[:, 0] ** 2 + p[:, 1] ** 2])


def phase_projector(wl):
    Z = phase_modes(wl)
    return np.eye(Z.shape[0]) - Z @ np.linalg.pinv(Z)


def solve_mode_removed(A, M, s):
    """zeta in the range of M with (M A M) zeta = M s: Cholesky of M A M + I - M."""
    from .solve import cholesky_solve
    B = M @ A @ M + np.eye(M.shape[0]) - M
    return cholesky_solve(0.5 * (B + B.T), M @ s)
