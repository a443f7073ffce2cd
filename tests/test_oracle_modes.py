"""Pins of the oracle's low-order mode removal (oracle.modes, §2.F).

* The slope modes are the Hudgin slopes of the phase modes x, y, x^2 + y^2:
  phase differences across each valid subaperture evaluated from the phase
  functions at the edge midpoints, equal to the columns of Z_s up to scale.
* M_s and M_phi are orthogonal projectors that annihilate their modes, with
  the expected rank.
* The mode-removed solution lies in the range of M_s, solves M A M zeta = M s,
  equals the minimum-norm (pseudo-inverse) solution, and CG on M A M from zero
  reaches it."""
import numpy as np

import workloads as W
from oracle import geometry as G
from oracle.covariance import system_matrix
from oracle.modes import (phase_modes, phase_projector, slope_modes, slope_projector, solve_mode_removed)
from oracle.solve import cg


def test_slope_modes_are_hudgin_slopes_of_phase_modes():
    wl = W.lgs3_10x10()
    d = wl.d
    r = G.subap_centers(wl.n, d)[G.valid_index(wl.valid)]
    Z = slope_modes(wl)
    nv = r.shape[0]
    for col, f in enumerate((lambda x, y: x, lambda x, y: y, lambda x, y: x * x + y * y)):
        sx = f(r[:, 0] + d / 2, r[:, 1]) - f(r[:, 0] - d / 2, r[:, 1])
        sy = f(r[:, 0], r[:, 1] + d / 2) - f(r[:, 0], r[:, 1] - d / 2)
        ref = np.concatenate([sx, sy])
        scale = (ref @ Z[:, col]) / (Z[:, col] @ Z[:, col])
        assert np.abs(ref - scale * Z[:, col]).max() <= 1e-12 * np.abs(ref).max()
    assert Z.shape == (2 * nv, 3)


def test_projectors():
    wl = W.lgs3_10x10()
    M = slope_projector(wl)
    assert np.allclose(M, M.T, atol=1e-13) and np.allclose(M @ M, M, atol=1e-12)
    Z = slope_modes(wl)
    for g in range(wl.n_gs):
        Zg = np.zeros((M.shape[0], 3))
        Zg[g * Z.shape[0]:(g + 1) * Z.shape[0]] = Z
        assert np.abs(M @ Zg).max() <= 1e-12
    assert round(np.trace(M)) == wl.n_gs * (Z.shape[0] - 3)
    Mp = phase_projector(wl)
    Zp = phase_modes(wl)
    assert np.allclose(Mp, Mp.T, atol=1e-13) and np.allclose(Mp @ Mp, Mp, atol=1e-12)
    assert np.abs(Mp @ Zp).max() <= 1e-10 * np.abs(Zp).max()
    assert round(np.trace(Mp)) == Zp.shape[0] - 3


def test_mode_removed_solution():
    wl = W.lgs3_10x10()
    A = system_matrix(wl)
    M = slope_projector(wl)
    s = W.turbulent_slopes(wl)[0]
    z = solve_mode_removed(A, M, s)
    MAM = M @ A @ M
    assert np.linalg.norm(M @ z - z) <= 1e-12 * np.linalg.norm(z)
    assert np.linalg.norm(MAM @ z - M @ s) <= 1e-10 * np.linalg.norm(M @ s)
    zp = np.linalg.pinv(MAM, rcond=1e-12) @ (M @ s)
    assert np.linalg.norm(z - zp) <= 1e-8 * np.linalg.norm(z)
    zc, k = cg(lambda v: MAM @ v, M @ s, tol=1e-12)
    assert np.linalg.norm(zc - z) <= 1e-6 * np.linalg.norm(z)
