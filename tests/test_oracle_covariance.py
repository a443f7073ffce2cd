"""Pins of the Hudgin-like covariances (App. A.2) and of the dense Sigma_ss
(§2.D, §2.F) against the slope model's own definition.

A Hudgin-like slope is phi(P) - phi(Q) with P, Q the edge midpoints of the
subaperture (App. A.2).  With <phi(u) phi(v)> = sigma^2 - D(u - v)/2 every
slope covariance is the textbook product G C_phiphi G^T of a +/-1 difference
matrix G with the point covariance C_phiphi; the sigma^2 term cancels because
each row of G sums to zero.  These tests build that product independently of
the four-term closed forms in oracle.covariance.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import covariance as C
from oracle import geometry as G
from oracle.vonkarman import structure_function


def stencil_product_cov(wl):
    """Sigma_ss = sum_k w_k G_k C_k G_k^T from explicit edge points."""
    idx = G.valid_index(wl.valid)
    r = G.subap_centers(wl.n, wl.d)[idx]
    s = G.cone_scale(wl.h, wl.h_lgs)
    nv = r.shape[0]
    nslope = 2 * wl.n_gs * nv
    total = np.zeros((nslope, nslope))
    for k in range(wl.n_layer):
        pts = []
        Gm = np.zeros((nslope, 2 * nslope))
        row = 0
        for g in range(wl.n_gs):
            for p in range(2):
                e = np.array([1.0, 0.0]) if p == 0 else np.array([0.0, 1.0])
                for v in range(nv):
                    base = s[k] * r[v] + wl.h[k] * wl.gs[g]
                    pts.append(base + 0.5 * s[k] * wl.d * e)
                    pts.append(base - 0.5 * s[k] * wl.d * e)
                    Gm[row, 2 * row] = 1.0
                    Gm[row, 2 * row + 1] = -1.0
                    row += 1
        pts = np.array(pts)
        diff = pts[:, None, :] - pts[None, :, :]
        Cpp = 7.0 - 0.5 * structure_function(np.hypot(diff[..., 0], diff[..., 1]), wl.r0, wl.L0)
        total += wl.w[k] * (Gm @ Cpp @ Gm.T)
    return total


CASES = [
    dict(n=3, n_gs=1, lgs=False, n_layer=1, seed=1, mask="full"),
    dict(n=4, n_gs=2, lgs=True, n_layer=2, seed=2),
    dict(n=5, n_gs=3, lgs=True, n_layer=3, seed=3),
    dict(n=4, n_gs=3, lgs=False, n_layer=2, seed=4),
    dict(n=2, n_gs=4, lgs=True, n_layer=4, seed=5, mask="full"),
]


@pytest.mark.parametrize("case", CASES)
def test_dense_matches_stencil_product(case):
    wl = W.tiny(**case)
    S = C.slope_covariance(wl)
    R = stencil_product_cov(wl)
    assert np.abs(S - R).max() <= 1e-10 * np.abs(R).max()


def test_printed_xy_sign_fails_the_definition():
    # Plant the printed sign of the last xy term in a copy of the formula: it
    # disagrees with the stencil product and gives xy(0) != 0.
    wl = W.tiny(n=3, n_gs=1, lgs=False, n_layer=1, seed=7, mask="full")
    d = wl.d

    def xy_printed(dx, dy):
        h = 0.5 * d
        D = lambda a, b: structure_function(np.hypot(a, b), wl.r0, wl.L0)
        return 0.5 * (D(dx + h, dy + h) - D(dx - h, dy + h) - D(dx + h, dy - h) - D(dx - h, dy - h))

    assert abs(xy_printed(np.array([0.0]), np.array([0.0]))[0]) > 1.0
    assert abs(C.hudgin_xy(np.array([0.0]), np.array([0.0]), d, wl.r0, wl.L0)[0]) < 1e-12


@pytest.mark.parametrize("case", CASES)
def test_symmetric_positive_definite(case):
    wl = W.tiny(**case)
    A = C.system_matrix(wl)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    ev = np.linalg.eigvalsh(C.slope_covariance(wl))
    assert ev.min() >= -1e-10 * ev.max()
    assert np.linalg.eigvalsh(A).min() >= 0.999 * wl.noise_var


@pytest.mark.parametrize("case", CASES)
def test_blocks_are_2rbt(case):
    # Theta^{gh}_{pq}[a, b] depends only on the lag of b relative to a (§2.D),
    # and equals the unique-element table at that lag.
    wl = W.tiny(**dict(case, mask="full"))
    n, nv = wl.n, wl.n * wl.n
    S = C.slope_covariance(wl)
    tabs = C.kernel_tables(wl)
    ii, jj = np.divmod(np.arange(nv), n)
    for (gi, gj, p, q), t in tabs.items():
        a0, b0 = (2 * gi + p) * nv, (2 * gj + q) * nv
        blk = S[a0:a0 + nv, b0:b0 + nv]
        u = jj[None, :] - jj[:, None]
        v = ii[None, :] - ii[:, None]
        assert np.abs(blk - t[v + n - 1, u + n - 1]).max() <= 1e-12 * max(1.0, np.abs(t).max())


def test_same_sensor_xy_vanishes_at_zero_lag_and_blocks_are_even():
    wl = W.tiny(n=5, n_gs=2, lgs=True, n_layer=3, seed=11, mask="full")
    tabs = C.kernel_tables(wl)
    n = wl.n
    for g in range(wl.n_gs):
        for p in range(2):
            for q in range(2):
                t = tabs[(g, g, p, q)]
                assert np.allclose(t, t[::-1, ::-1], rtol=0, atol=1e-12 * np.abs(t).max())
        assert abs(tabs[(g, g, 0, 1)][n - 1, n - 1]) < 1e-12
        assert np.allclose(tabs[(g, g, 0, 1)], tabs[(g, g, 1, 0)], rtol=0, atol=1e-13)
    # xy = yx as functions of the separation, for different sensors too
    assert np.allclose(tabs[(0, 1, 0, 1)], tabs[(0, 1, 1, 0)], rtol=0, atol=1e-12)


def test_lgs_with_ground_layers_equals_ngs():
    wl = W.tiny(n=4, n_gs=2, lgs=True, n_layer=2, seed=3)
    wl.h = np.zeros_like(wl.h)
    ngs = W.tiny(n=4, n_gs=2, lgs=False, n_layer=2, seed=3)
    ngs.h = wl.h
    assert np.abs(C.slope_covariance(wl) - C.slope_covariance(ngs)).max() < 1e-12


def test_rows_match_dense():
    wl = W.tiny(n=5, n_gs=2, lgs=True, n_layer=2, seed=9)
    S = C.slope_covariance(wl)
    rows = [0, 3, S.shape[0] - 1]
    assert np.abs(C.slope_covariance_rows(wl, rows) - S[rows]).max() < 1e-12


def test_config1_counts():
    wl = W.lgs3_10x10()
    assert wl.n_vs == 76 and wl.n_slopes == 456
    assert W.pupil_mask(74, 39.0, 0.28).sum() == 3972


def fried_stencil_product_cov(wl):
    """Fried slopes (App. A.3) as +-1/2 combinations of the four corner phases."""
    idx = G.valid_index(wl.valid)
    r = G.subap_centers(wl.n, wl.d)[idx]
    s = G.cone_scale(wl.h, wl.h_lgs)
    nv = r.shape[0]
    nslope = 2 * wl.n_gs * nv
    corners = np.array([[1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=float)   # a, b, c, d
    wx = np.array([1, -1, -1, 1]) * 0.5
    wy = np.array([1, 1, -1, -1]) * 0.5
    total = np.zeros((nslope, nslope))
    for k in range(wl.n_layer):
        pts, Gm = [], np.zeros((nslope, 4 * nslope))
        row = 0
        for g in range(wl.n_gs):
            for p in range(2):
                wts = wx if p == 0 else wy
                for v in range(nv):
                    base = s[k] * r[v] + wl.h[k] * wl.gs[g]
                    for q in range(4):
                        pts.append(base + 0.5 * s[k] * wl.d * corners[q])
                        Gm[row, len(pts) - 1] = wts[q]
                    row += 1
        pts = np.array(pts)
        diff = pts[:, None, :] - pts[None, :, :]
        Cpp = 5.0 - 0.5 * structure_function(np.hypot(diff[..., 0], diff[..., 1]), wl.r0, wl.L0)
        total += wl.w[k] * (Gm @ Cpp @ Gm.T)
    return total


@pytest.mark.parametrize("case", CASES[1:4])
def test_fried_matches_corner_stencil(case):
    wl = W.tiny(**case)
    wl.model = "fried"
    S = C.slope_covariance(wl)
    R = fried_stencil_product_cov(wl)
    assert np.abs(S - R).max() <= 1e-10 * np.abs(R).max()
    tabs = C.kernel_tables(wl)
    assert np.allclose(tabs[(0, 1, 0, 1)], tabs[(0, 1, 1, 0)], rtol=0, atol=1e-12)


def test_fried_has_an_invisible_waffle_mode():
    # App. A.3: the Fried model does not see the checkerboard (waffle) phase
    wl = W.tiny(n=4, n_gs=1, lgs=False, n_layer=1, seed=1, mask="full")
    n, d = wl.n, wl.d
    i, j = np.divmod(np.arange((n + 1) ** 2), n + 1)
    waffle = (-1.0) ** (i + j)
    sx = np.zeros((n, n))
    sy = np.zeros((n, n))
    ph = waffle.reshape(n + 1, n + 1)
    for a in range(n):
        for b in range(n):
            pa, pb, pc, pd = ph[a + 1, b + 1], ph[a + 1, b], ph[a, b], ph[a, b + 1]
            sx[a, b] = 0.5 * (pa - pb - pc + pd)
            sy[a, b] = 0.5 * (pa + pb - pc - pd)
    assert np.abs(sx).max() == 0 and np.abs(sy).max() == 0


# --- elongated-spot noise (§2.F) ----------------------------------------------

def test_noise_covariance_structure():
    wl = W.tiny(n=4, n_gs=2, seed=3)
    var, cxy = W.elongated_noise(wl)
    E = C.noise_covariance(wl, var, cxy)
    nvs = wl.n_slopes // (2 * wl.n_gs)
    assert np.array_equal(E, E.T)
    assert np.allclose(np.diag(E), var)
    off = E - np.diag(np.diag(E))
    for i, j in zip(*np.nonzero(off)):
        # only the x and y slopes of one subaperture of one sensor are coupled
        assert i // (2 * nvs) == j // (2 * nvs) and i % nvs == j % nvs and i != j
    assert np.linalg.eigvalsh(E).min() > 0
    assert np.array_equal(C.noise_covariance(wl, var, None), np.diag(var))


def test_elongated_noise_principal_axes_radial():
    wl = W.lgs3_10x10()
    var, cxy = W.elongated_noise(wl)
    n, d = wl.n, wl.d
    idx = np.flatnonzero(wl.valid.ravel())
    cx = (idx % n - (n - 1) / 2.0) * d
    cy = (idx // n - (n - 1) / 2.0) * d
    v = var.reshape(wl.n_gs, 2, -1)
    for g in range(wl.n_gs):
        for t in range(idx.size):
            B = np.array([[v[g, 0, t], cxy[g, t]], [cxy[g, t], v[g, 1, t]]])
            lam, U = np.linalg.eigh(B)
            assert abs(lam[0] - wl.noise_var) <= 1e-12           # across the radial direction: sigma^2
            radial = np.array([cx[t], cy[t]]) / np.hypot(cx[t], cy[t])
            assert abs(abs(U[:, 1] @ radial) - 1.0) <= 1e-9       # the larger axis is radial


def test_correlated_noise_sample_covariance():
    wl = W.tiny(n=3, n_gs=1, seed=2, mask="full")
    var, cxy = W.elongated_noise(wl, elongation=4.0)
    E = C.noise_covariance(wl, var, cxy)
    X = np.array([W.correlated_noise(var, cxy, seed=k) for k in range(20000)])
    emp = X.T @ X / X.shape[0]
    assert np.abs(emp - E).max() <= 0.05 * np.abs(E).max()
